"""Pins for the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: grid search,
corner enumeration, hand-derived optima, the textbook 1-D algorithm, brute
force, closed forms and the lemmas/theorem of the paper.
"""
import itertools
import json
import os

import numpy as np
import pytest

import datagen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- primitives

@pytest.mark.parametrize("d", [1, 2, 3])
def test_point_box_min_dist_vs_grid_search(orc, d):
    """Section 3.1 closed form == min over a fine lattice of the box."""
    rng = np.random.default_rng(10 + d)
    m = {1: 4097, 2: 257, 3: 41}[d]
    for _ in range(30):
        lo = rng.uniform(-1, 0.5, d)
        hi = lo + rng.uniform(0.0, 1.0, d)
        x = rng.uniform(-2, 2, d)
        v = orc.point_box_min_dist2(x, lo, hi)
        axes = [np.linspace(lo[a], hi[a], m) for a in range(d)]
        grid = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, d)
        g = ((grid - x) ** 2).sum(1).min()
        h = np.sqrt((((hi - lo) / (m - 1) / 2) ** 2).sum())  # lattice covering radius
        assert g >= v - 1e-12
        assert g <= (np.sqrt(v) + h) ** 2 + 1e-12


def test_point_box_min_dist_special_cases(orc):
    rng = np.random.default_rng(3)
    for _ in range(50):
        lo = rng.uniform(-1, 0, 3)
        hi = lo + rng.uniform(0, 1, 3)
        inside = lo + rng.uniform(0, 1, 3) * (hi - lo)
        assert orc.point_box_min_dist2(inside, lo, hi) == 0.0
    for x, lo, hi in [(-3.0, -1.0, 2.0), (5.0, -1.0, 2.0), (0.5, -1.0, 2.0)]:
        want = max(lo - x, 0.0, x - hi) ** 2
        assert orc.point_box_min_dist2([x], [lo], [hi]) == want


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_point_box_max_dist_vs_corners(orc, d):
    """Section 4.2.1 closed form == max over all 2^d corners (convex function)."""
    rng = np.random.default_rng(20 + d)
    for _ in range(40):
        lo = rng.uniform(-1, 0.5, d)
        hi = lo + rng.uniform(0.0, 1.0, d)
        x = rng.uniform(-2, 2, d)
        v = orc.point_box_max_dist2(x, lo, hi)
        corners = np.array(list(itertools.product(*[(lo[a], hi[a]) for a in range(d)])))
        want = ((corners - x) ** 2).sum(1).max()
        assert abs(v - want) <= 1e-12 * max(1.0, want)


def test_objective_hand_values(orc):
    """Eq (12) on configurations whose value is known by geometry."""
    ang = np.arange(12) * (2 * np.pi / 12)
    X = np.stack([np.cos(ang), np.sin(ang)], 1) * 2.0
    X = np.vstack([X, [[0.0, 0.0]]])
    # center at the origin: every circle point at squared radius 4
    obj, am = orc.objective(X, np.array([[[0.0, 0.0]]]))
    assert abs(obj[0] - 4.0) < 1e-12 and am[0] == 0
    # center on a circle point: farthest is the antipode at squared distance 16
    obj, am = orc.objective(X, X[None, [3]])
    assert abs(obj[0] - 16.0) < 1e-12 and am[0] == 9
    # every sample a center: 0
    obj, _ = orc.objective(X[:5], X[None, :5])
    assert obj[0] == 0.0


def test_lower_bound_special_cases(orc):
    X = datagen.small_mixture(1).astype(np.float64)
    n, d = X.shape
    lo0, hi0 = X.min(0), X.max(0)
    # root region contains every sample: LB = 0, argmax the first sample
    k = 3
    lb, am = orc.lower_bound(X, [0, k], np.tile(lo0, (k, 1)), np.tile(hi0, (k, 1)))
    assert lb[0] == 0.0 and am[0] == 0
    # a node whose boxes are single points: LB = objective at those points
    c = X[[5, 50, 500]]
    lb, am = orc.lower_bound(X, [0, 3], c, c)
    obj, oam = orc.objective(X, c[None])
    assert lb[0] == obj[0] and am[0] == oam[0]


def test_lower_bound_monotone_and_valid(orc):
    """Child LB >= parent LB; LB <= objective of any centers inside the node."""
    X = datagen.gaussian_mixture(300, 2, 3, 0.08, 7).astype(np.float64)
    rng = np.random.default_rng(0)
    for _ in range(25):
        ids = rng.choice(len(X), 3, replace=False)
        c = X[ids]
        w = rng.uniform(0, 0.3, (3, 2))
        lo, hi = c - w * rng.uniform(0, 1, (3, 2)), c + w * rng.uniform(0, 1, (3, 2))
        lbp, _ = orc.lower_bound(X, [0, 3], lo, hi)
        obj, _ = orc.objective(X, c[None])
        assert lbp[0] <= obj[0]
        kk, a = rng.integers(3), rng.integers(2)
        lo2, hi2 = lo.copy(), hi.copy()
        hi2[kk, a] = 0.5 * (lo[kk, a] + hi[kk, a])
        lbc, _ = orc.lower_bound(X, [0, 3], lo2, hi2)
        assert lbc[0] >= lbp[0]


def test_candidates_inside_and_closest(orc):
    X = datagen.gaussian_mixture(500, 2, 3, 0.08, 2).astype(np.float64)
    off, lo, hi = datagen.random_boxes(20, 3, 2, 5, wmin=1e-2, wmax=0.6)
    cand = orc.candidates(X, lo.astype(np.float64), hi.astype(np.float64))
    for b in range(lo.shape[0]):
        inside = np.all((X >= lo[b]) & (X <= hi[b]), 1)
        if not inside.any():
            assert cand[b] == -1
            continue
        mid = 0.5 * (lo[b].astype(np.float64) + hi[b])
        dist = ((X - mid) ** 2).sum(1)
        dist[~inside] = np.inf
        assert cand[b] == int(np.argmin(dist))


# ------------------------------------------------------------- brute force

def _golden():
    with open(os.path.join(GOLDEN, "hand_instances.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["name"])
def test_brute_force_and_solve_hand_instances(orc, case):
    X = np.array(case["points"], dtype=np.float64)
    for ks, want in case["opt"].items():
        k = int(ks)
        best, ids = orc.brute_force(X, k)
        assert best == want
        obj, _ = orc.objective(X, X[ids][None])
        assert obj[0] == want
        if k <= len(X):
            r = orc.solve(X, k, i_sr=2)
            assert r["obj"] == want and r["status"] == 0


def test_k1_full_size(orc):
    """K=1 at N=2000: the plain O(N^2) minimax over all sample centers."""
    X = datagen.small_mixture(2).astype(np.float64)
    D = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    want = D.max(0).min()
    r = orc.solve(X, 1)
    assert r["obj"] == want and r["lb"] == want


@pytest.mark.slow
def test_k2_full_size(orc):
    """K=2 at N=2000 against exhaustive search over all C(2000,2) pairs."""
    X = datagen.small_mixture(3).astype(np.float64)
    best, ids = orc.brute_force(X, 2)
    r = orc.solve(X, 2)
    assert r["obj"] == best


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_solve_vs_brute_force_slice(orc, seed):
    """B&B optimum == brute force on the first 30 samples of the small workload."""
    X = datagen.small_mixture(seed).astype(np.float64)[:30]
    for k in (2, 3, 4):
        best, _ = orc.brute_force(X, k)
        for use_bt, mr in ((True, 50), (True, 0), (False, 50)):
            r = orc.solve(X, k, use_bt=use_bt, i_sr=3, max_refs=mr)
            assert r["obj"] == best, (k, use_bt, mr)
            assert r["lb"] == best


@pytest.mark.parametrize("seed", range(6))
def test_solve_vs_brute_force_random(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(20, 61))
    d = int(rng.integers(1, 4))
    X = datagen.gaussian_mixture(n, d, 3, 0.15, 100 + seed).astype(np.float64)
    best, _ = orc.brute_force(X, 3)
    r = orc.solve(X, 3, i_sr=int(rng.integers(1, 5)), fft_start=int(rng.integers(n)))
    assert r["obj"] == best


def _exact_1d(x, k):
    """Textbook exact discrete k-center on a line: bisection on the radius with
    the greedy cover (leftmost uncovered point, farthest center reaching it)."""
    xs = np.sort(np.asarray(x, dtype=np.float64))

    def centers_for(r):
        cs, i, n = [], 0, len(xs)
        while i < n:
            p = xs[i]
            # rightmost sample c >= p with (c - p)^2 <= r
            lo, hi = i, n - 1
            while lo < hi:
                mid = (lo + hi + 1) // 2
                if (xs[mid] - p) ** 2 <= r:
                    lo = mid
                else:
                    hi = mid - 1
            c = xs[lo]
            cs.append(c)
            j = lo
            while j < n and (xs[j] - c) ** 2 <= r:
                j += 1
            i = j
            if len(cs) > k:
                return None
        return cs

    lo_r, hi_r = 0.0, (xs[-1] - xs[0]) ** 2
    if centers_for(0.0) is not None:
        return 0.0
    for _ in range(200):
        mid = 0.5 * (lo_r + hi_r)
        if mid <= lo_r or mid >= hi_r:
            break
        if centers_for(mid) is None:
            lo_r = mid
        else:
            hi_r = mid
    cs = np.array(centers_for(hi_r))
    return float(((xs[:, None] - cs[None, :]) ** 2).min(1).max())


@pytest.mark.parametrize("seed,n,k", [(0, 200, 2), (1, 2000, 3), (2, 20000, 4), (3, 100000, 3)])
def test_one_dimensional_vs_textbook(orc, seed, n, k):
    x = datagen.gaussian_mixture(n, 1, k, 0.05, seed)[:, 0].astype(np.float64)
    want = _exact_1d(x, k)
    r = orc.solve(x[:, None], k)
    assert r["obj"] == want


def test_fft_two_approximation_and_determinism(orc):
    """Gonzalez: the FFT radius is at most twice the optimum, i.e. 4x squared."""
    for seed in range(5):
        X = datagen.small_mixture(seed).astype(np.float64)[:40]
        best, _ = orc.brute_force(X, 3)
        for s0 in (0, 7, 39):
            T = orc.fft(X, 3, s0)
            assert T[0] == s0 and len(set(T.tolist())) == 3
            obj, _ = orc.objective(X, X[T][None])
            assert obj[0] <= 4.0 * best + 1e-15
            assert np.array_equal(T, orc.fft(X, 3, s0))


def test_fft_picks_farthest(orc):
    X = np.array([[0.0], [1.0], [5.0], [2.0], [5.0]])
    T = orc.fft(X, 3, 1)
    # from x=1 the farthest is 5 (first at index 2); then 0 beats 2 (1 vs 1: tie -> lowest)
    assert T.tolist() == [1, 2, 0]


# ------------------------------------------------- tightening and reduction

def _node_containing(X, ids, rng, width=0.25):
    c = X[ids]
    lo = c - rng.uniform(0, width, c.shape)
    hi = c + rng.uniform(0, width, c.shape)
    return lo, hi


@pytest.mark.parametrize("seed", range(4))
def test_tightening_keeps_optimal_centers(orc, seed):
    """Lemmas 1-2: optimal centers inside a node stay inside its tightened box,
    and every sample assigned to cluster k is within alpha of mu*^k."""
    X = datagen.gaussian_mixture(40, 2, 3, 0.1, 200 + seed).astype(np.float64)
    z, ids = orc.brute_force(X, 3)
    rng = np.random.default_rng(seed)
    for trial in range(10):
        lo, hi = _node_containing(X, ids, rng)
        alpha = z * (1.0 + rng.uniform(0, 0.5))
        use_refs = trial % 2 == 0
        if use_refs:
            ref_off = np.arange(4, dtype=np.int32)
            ref = X[ids]
        else:
            ref_off, ref = None, None
        agg = orc.tighten_node(X, lo, hi, alpha, ref_off, ref, want_labels=True)
        mu = X[ids]
        lab = agg["labels"]
        for s in np.nonzero(lab >= 0)[0]:
            assert ((X[s] - mu[lab[s]]) ** 2).sum() <= alpha
        assert agg["n_excluded"] == 0
        inf, lo2, hi2 = orc.tightened_box(lo, hi, alpha, agg, ref_off, ref)
        assert not inf
        assert np.all(lo2 <= mu) and np.all(mu <= hi2)


def test_tightening_aggregates_by_hand(orc):
    """Center-based assignment and box tightening on a 1-D node worked by hand
    (binary fractions, so every value below is exact)."""
    X = np.array([[0.0], [0.25], [0.5], [0.875], [1.0]])
    lo = np.array([[0.0], [0.875]])
    hi = np.array([[0.25], [1.0]])
    alpha = 0.0625
    # beta to box0 / box1: 0 / .765625, 0 / .390625, .0625 / .140625, .390625 / 0, .5625 / 0
    agg = orc.tighten_node(X, lo, hi, alpha, want_labels=True)
    assert agg["labels"].tolist() == [0, 0, 0, 1, 1]
    assert agg["n_asg"].tolist() == [3, 2]
    assert agg["asg_min"][:, 0].tolist() == [0.0, 0.875] and agg["asg_max"][:, 0].tolist() == [0.5, 1.0]
    assert agg["n_in"].tolist() == [2, 2]
    assert agg["bb_lo"][:, 0].tolist() == [0.0, 0.875] and agg["bb_hi"][:, 0].tolist() == [0.25, 1.0]
    # farthest assigned from the midpoints .125 and .9375: x = .5 (index 2);
    # .875 and 1.0 tie at .0625 -> the lower index 3
    assert agg["asg_far"].tolist() == [2, 3]
    inf, lo2, hi2 = orc.tightened_box(lo, hi, alpha, agg)
    # box0: bbox [0, .25] cap [.5 - .25, 0 + .25] = [.25, .25]; box1 unchanged
    assert not inf
    assert lo2[:, 0].tolist() == [0.25, 0.875] and hi2[:, 0].tolist() == [0.25, 1.0]
    # a smaller alpha rules x = 0.5 out of both clusters: the node is infeasible
    agg = orc.tighten_node(X, lo, hi, 0.05, want_labels=True)
    assert agg["labels"][2] == -2 and agg["n_excluded"] == 1


def test_symmetry_breaking_propagation(orc):
    lo = np.array([[0.5, 0.0], [0.0, 0.0], [0.2, 0.0]])
    hi = np.array([[1.0, 1.0], [0.7, 1.0], [0.6, 1.0]])
    empty, lo2, hi2 = orc.symmetry(lo, hi)
    assert not empty
    assert lo2[:, 0].tolist() == [0.5, 0.5, 0.5] and hi2[:, 0].tolist() == [0.6, 0.6, 0.6]
    empty, _, _ = orc.symmetry(np.array([[0.5, 0], [0.0, 0]]), np.array([[1.0, 1], [0.4, 1]]))
    assert empty


@pytest.mark.parametrize("seed", range(3))
def test_reduction_flags_are_sound(orc, seed):
    """A deleted sample is LB- and UB-redundant in every node, checked with the
    corner enumeration of Section 4.2.1 and plain distances."""
    X = datagen.gaussian_mixture(400, 2, 3, 0.08, 300 + seed).astype(np.float64)
    off, lo, hi = datagen.random_boxes(6, 3, 2, seed, wmin=0.05, wmax=0.4)
    lo, hi = lo.astype(np.float64), hi.astype(np.float64)
    rng = np.random.default_rng(seed)
    ref_ids = rng.choice(len(X), 3, replace=False)
    ref_off = np.arange(0, lo.shape[0] + 1, dtype=np.int32)
    ref = X[ref_ids][np.arange(lo.shape[0]) % 3]
    beta, alpha = 0.3, 0.02
    keep = orc.reduce_flags(X, off, lo, hi, ref_off, ref, beta, alpha)
    assert 0 < keep.sum() < len(X)
    for s in np.nonzero(keep == 0)[0]:
        x = X[s]
        for m in range(len(off) - 1):
            far = []
            for b in range(off[m], off[m + 1]):
                corners = np.array(list(itertools.product(*[(lo[b, a], hi[b, a]) for a in range(2)])))
                far.append(((corners - x) ** 2).sum(1).max())
                inside = np.all((lo[b] <= x) & (x <= hi[b]))
                if inside:
                    assert ((x - ref[b]) ** 2).sum() > alpha
            assert min(far) < beta


@pytest.mark.parametrize("seed", range(3))
def test_reduction_preserves_optimum(orc, seed):
    X = datagen.small_mixture(seed).astype(np.float64)[:400]
    base = orc.solve(X, 3, i_sr=0)
    for i_sr in (1, 2, 5):
        r = orc.solve(X, 3, i_sr=i_sr)
        assert r["obj"] == base["obj"]
        obj, _ = orc.objective(X, X[r["centers"]][None])
        assert obj[0] == r["obj"]


def test_solve_reports_consistent_centers(orc):
    X = datagen.small_mixture(4).astype(np.float64)
    r = orc.solve(X, 3, i_sr=10)
    obj, _ = orc.objective(X, X[r["centers"]][None])
    assert obj[0] == r["obj"] and r["lb"] == r["obj"] and r["status"] == 0
    assert r["obj"] <= r["fft_obj"]


def test_planted_mistake_is_caught(orc):
    """A closed form with a wrong sign in the clamp must fail the grid pin;
    this keeps the grid-search test honest."""
    rng = np.random.default_rng(1)
    bad = 0
    for _ in range(50):
        lo = rng.uniform(-1, 0, 2)
        hi = lo + rng.uniform(0.1, 1, 2)
        x = rng.uniform(-2, 2, 2)
        wrong = (((x - np.clip(x, hi, lo)) ** 2).sum())  # operands swapped
        right = orc.point_box_min_dist2(x, lo, hi)
        bad += abs(wrong - right) > 1e-12
    assert bad > 0


@pytest.mark.parametrize("seed", [0, 1, 3])
def test_node_reduction_carries_over_to_descendants(orc, seed):
    """Section 4.2 applied to one node with its own lower bound as beta: the
    samples deleted there change nothing below it. For descendants reached by
    midpoint splits, the inherited lower bound max(LB(M), LB(M')) is the same
    over the kept samples as over all, the objective of centers inside M' is
    the same, and so are the count and bounding box of S_+ per box."""
    X = datagen.gaussian_mixture(600, 2, 3, 0.06, 500 + seed).astype(np.float64)
    T = orc.fft(X, 3)
    c = X[T]
    lo, hi = c - 0.08, c + 0.08
    lb_m = orc.lower_bound(X, [0, 3], lo, hi)[0][0]
    alpha = orc.objective(X, c[None])[0][0]
    ref_off = np.arange(4, dtype=np.int32)
    keep = orc.reduce_flags(X, [0, 3], lo, hi, ref_off, c, lb_m, alpha).astype(bool)
    assert 0 < keep.sum() < len(X)
    Xk = X[keep]
    rng = np.random.default_rng(seed)
    checked = 0
    for _ in range(12):
        l2, h2 = lo.copy(), hi.copy()
        for _depth in range(int(rng.integers(1, 7))):
            k, a = int(rng.integers(3)), int(rng.integers(2))
            mid = 0.5 * (l2[k, a] + h2[k, a])
            if rng.integers(2):
                h2[k, a] = mid
            else:
                l2[k, a] = mid
        full = orc.lower_bound(X, [0, 3], l2, h2)[0][0]
        kept = orc.lower_bound(Xk, [0, 3], l2, h2)[0][0]
        assert max(lb_m, kept) == max(lb_m, full)
        cand = orc.candidates(X, l2, h2)
        if np.all(cand >= 0):
            C = X[cand][None]
            assert orc.objective(Xk, C)[0][0] == orc.objective(X, C)[0][0]
            checked += 1
        ta = orc.tighten_node(X, l2, h2, alpha, ref_off, c)
        tk = orc.tighten_node(Xk, l2, h2, alpha, ref_off, c)
        assert np.array_equal(ta["n_in"], tk["n_in"])
        has = ta["n_in"] > 0
        assert np.array_equal(ta["bb_lo"][has], tk["bb_lo"][has])
        assert np.array_equal(ta["bb_hi"][has], tk["bb_hi"][has])
    assert checked > 0


def _hand_reduce_candidates():
    with open(os.path.join(os.path.dirname(__file__), "golden", "reduce_and_candidates_hand.json")) as f:
        return json.load(f)


def test_candidates_hand_worked(orc):
    """Section 3.2 on a hand-worked fixture: a nearer sample outside the box is
    not a candidate, exact ties go to the lowest index, point boxes and empty
    boxes."""
    c = _hand_reduce_candidates()["candidates"]
    X = np.array(c["points"], dtype=np.float64)
    cand = orc.candidates(X, np.array(c["lo"]), np.array(c["hi"]))
    assert cand.tolist() == c["cand"]


def _reduce_case(node_list):
    lo = np.concatenate([np.array(n["lo"]) for n in node_list])
    hi = np.concatenate([np.array(n["hi"]) for n in node_list])
    off = np.arange(0, 2 * len(node_list) + 1, 2, dtype=np.int32)
    rows, roff = [], [0]
    for n in node_list:
        for refs in n["refs"]:
            rows.extend(refs)
            roff.append(len(rows))
    return off, lo, hi, np.array(roff, dtype=np.int32), np.array(rows, dtype=np.float64)


def test_reduction_flags_hand_worked(orc):
    """Algorithm 5 on a hand-worked 1-D fixture: one far ref of a box suffices
    for UB-redundancy, the LB test is strict, and a sample is deleted only when
    redundant in every node."""
    r = _hand_reduce_candidates()["reduce"]
    X = np.array(r["points"], dtype=np.float64)
    for nodes, want in (([r["node1"]], r["keep_node1"]), ([r["node1"], r["node2"]], r["keep_both"])):
        keep = orc.reduce_flags(X, *_reduce_case(nodes), r["beta"], r["alpha"])
        assert keep.tolist() == want


def _far_corner(x, lo, hi):
    corners = np.array(list(itertools.product(*[(lo[a], hi[a]) for a in range(len(x))])))
    return ((corners - x) ** 2).sum(1).max()


def _redundant_everywhere(x, off, lo, hi, ref_off, ref, beta, alpha, every_ref=False):
    """Section 4.2 by brute force: corner enumeration for the farthest point of
    each box, plain distances to every ref. every_ref=True plants a mistake
    (all refs of a box must be far instead of one)."""
    for m in range(len(off) - 1):
        far, ub_red = [], True
        for b in range(off[m], off[m + 1]):
            far.append(_far_corner(x, lo[b], hi[b]))
            inside = np.all((lo[b] <= x) & (x <= hi[b]))
            dist = ((ref[ref_off[b]:ref_off[b + 1]] - x) ** 2).sum(1)
            far_ok = np.all(dist > alpha) if every_ref else np.any(dist > alpha)
            if inside and not far_ok:
                ub_red = False
        if not (min(far) < beta and ub_red):
            return False
    return True


@pytest.mark.parametrize("seed", range(4))
def test_reduction_flags_complete(orc, seed):
    """Deleted exactly when redundant: every sample the oracle keeps fails the
    LB or UB test in some node and every sample it deletes passes both in all
    nodes (brute force over corners and refs), with several refs per box so
    that some but not all refs of a box are far."""
    X = datagen.gaussian_mixture(300, 2, 3, 0.08, 700 + seed).astype(np.float64)
    off, lo, hi = datagen.random_boxes(3, 3, 2, 40 + seed, wmin=0.1, wmax=0.6)
    lo, hi = lo.astype(np.float64), hi.astype(np.float64)
    rng = np.random.default_rng(seed)
    nb = lo.shape[0]
    # per box: the sample nearest its midpoint (near the box's samples), then
    # one to three random samples (mostly far from them)
    counts = rng.integers(2, 5, nb)
    ref_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    rows = []
    for b in range(nb):
        mid = 0.5 * (lo[b] + hi[b])
        rows.append(X[np.argmin(((X - mid) ** 2).sum(1))][None])
        rows.append(X[rng.choice(len(X), counts[b] - 1, replace=False)])
    ref = np.concatenate(rows)
    # beta where about half of the samples pass the LB test in every node
    worst = np.array([max(min(_far_corner(x, lo[b], hi[b]) for b in range(off[m], off[m + 1]))
                          for m in range(len(off) - 1)) for x in X])
    beta, alpha = float(np.quantile(worst, 0.5)), 0.01
    keep = orc.reduce_flags(X, off, lo, hi, ref_off, ref, beta, alpha)
    want = np.array([not _redundant_everywhere(x, off, lo, hi, ref_off, ref, beta, alpha) for x in X])
    assert 0 < want.sum() < len(X)
    assert np.array_equal(keep.astype(bool), want)
    # the instance tells one far ref from all refs far
    planted = np.array([not _redundant_everywhere(x, off, lo, hi, ref_off, ref, beta, alpha, True)
                        for x in X])
    assert not np.array_equal(planted, want)
