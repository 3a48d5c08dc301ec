"""Parity at the benchmark's full sizes, in the launch configuration the bench
times (the autotuner's tile for the same shapes): sampled outputs against the
oracle over all samples, properties that hold at any size, and the float64
certificate over 10^9 samples bit for bit."""
import numpy as np
import pytest
import torch

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2301_00061_amd import api
    return api


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(x, n):
    """[d, ld] device samples -> [n, d] float64 host array."""
    return x[:, :n].T.contiguous().cpu().numpy().astype(np.float64)


def _check_node(kc, X64, x, m, off, lo, hi, lb_raw, lb_safe, am, d):
    """Node m's bound equals the oracle's over all samples within the margin,
    and the device's argmax sample attains it."""
    g, eta = kc.rel_margin(d), kc.abs_margin(d)
    b0, b1 = int(off[m]), int(off[m + 1])
    lo64, hi64 = lo[b0:b1].astype(np.float64), hi[b0:b1].astype(np.float64)
    box_off = np.array([0, b1 - b0], dtype=np.int32)
    lb_o, _ = oracle.lower_bound(X64, box_off, lo64, hi64)
    assert abs(float(lb_raw[m]) - lb_o[0]) <= g * lb_o[0] + eta, (m, lb_raw[m], lb_o[0])
    assert lb_safe[m] <= lb_o[0]
    xs = x[:, int(am[m])].cpu().numpy().astype(np.float64)[None]
    v, _ = oracle.lower_bound(xs, box_off, lo64, hi64)
    assert v[0] >= lb_o[0] - 2 * (g * lb_o[0] + eta)
    return lo64, hi64


def test_mixture_10m_batched_bound_with_candidates(kc):
    n, d, k = 10_000_000, 4, 5
    print("full size: mixture_10m_d4_k5, 128 nodes x 5 boxes, bound + candidates", flush=True)
    x = datagen.gaussian_mixture_device(n, d, k, 0.1, 0, outlier_frac=0.01)
    off, lo, hi = datagen.random_boxes(128, k, d, 1, wmin=0.05, wmax=1.0)
    kc.autotune(x, n, _dev(off), _dev(lo), _dev(hi), with_cand=True, k_max=k)
    lb_raw, lb_safe, am, cand = kc.lower_bound(x, n, _dev(off), _dev(lo), _dev(hi), k_max=k,
                                               want_cand=True)
    lb_raw, lb_safe, am, cand = (t.cpu().numpy() for t in (lb_raw, lb_safe, am, cand))
    X64 = _host(x, n)
    g = kc.rel_margin(d)
    for m in (0, 41, 86, 127):
        lo64, hi64 = _check_node(kc, X64, x, m, off, lo, hi, lb_raw, lb_safe, am, d)
        cand_o = oracle.candidates(X64, lo64, hi64)
        for j in range(k):
            cg = int(cand[off[m] + j])
            if cand_o[j] < 0:
                assert cg == -1
                continue
            assert np.all((X64[cg] >= lo64[j]) & (X64[cg] <= hi64[j]))
            mid = 0.5 * (lo64[j] + hi64[j])
            dg, do = ((X64[cg] - mid) ** 2).sum(), ((X64[cand_o[j]] - mid) ** 2).sum()
            assert dg <= do + 2 * g * do + 1e-6 * (1 + np.sqrt(do)) * max(1.0, np.abs(mid).max())


def _mixture_1b(kc):
    n, d, k = 1_000_000_000, 2, 3
    x = datagen.gaussian_mixture_device(n, d, k, 0.05, 0)
    means = datagen._means(0, k, d).astype(np.float32)
    off = np.array([0, k], dtype=np.int32)
    return n, d, k, x, off, means - 0.05, means + 0.05


def test_mixture_1b_one_node_pass(kc):
    n, d, k, x, off, lo, hi = _mixture_1b(kc)
    print("full size: lb_1b_d2_k3, one node of 3 boxes over 10^9 samples", flush=True)
    kc.autotune(x, n, _dev(off), _dev(lo), _dev(hi), with_cand=False, k_max=k)
    lb_raw, lb_safe, am, _ = kc.lower_bound(x, n, _dev(off), _dev(lo), _dev(hi), k_max=k)
    lb_raw, lb_safe, am = (t.cpu().numpy() for t in (lb_raw, lb_safe, am))
    g, eta = kc.rel_margin(d), kc.abs_margin(d)
    lo64, hi64 = lo.astype(np.float64), hi.astype(np.float64)
    # the argmax sample attains the value
    xs = x[:, int(am[0])].cpu().numpy().astype(np.float64)[None]
    v, _ = oracle.lower_bound(xs, off, lo64, hi64)
    assert abs(float(lb_raw[0]) - v[0]) <= g * v[0] + eta
    assert lb_safe[0] <= v[0]
    # no sample lies farther: 4 * 10^6 random samples and the ragged tail
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([rng.integers(0, n, 4_000_000), np.arange(n - 5000, n)]))
    sub = x[:, torch.from_numpy(idx).cuda()].T.contiguous().cpu().numpy().astype(np.float64)
    lb_sub, _ = oracle.lower_bound(sub, off, lo64, hi64)
    assert lb_sub[0] <= float(lb_raw[0]) * (1 + g) + eta


def test_mixture_1b_certificate_is_exact(kc):
    n, d, k, x, _, _, _ = _mixture_1b(kc)
    print("full size: float64 objective of 3 centers over 10^9 samples", flush=True)
    ids = torch.tensor([7, n // 2, n - 1], device="cuda")
    C = x[:, ids].T.contiguous()[None]  # [1, k, d]
    o64, a64 = kc.objective(x, n, C, precision=64)
    o64, a64 = float(o64.cpu()[0]), int(a64.cpu()[0])
    C64 = C.cpu().numpy().astype(np.float64)
    best, best_i = -1.0, -1
    step = 100_000_000
    for c0 in range(0, n, step):  # the maximum of chunk maxima, first chunk on ties
        c1 = min(n, c0 + step)
        X = x[:, c0:c1].T.contiguous().cpu().numpy().astype(np.float64)
        o, a = oracle.objective(X, C64)
        if o[0] > best:
            best, best_i = float(o[0]), c0 + int(a[0])
    assert o64 == best and a64 == best_i


def test_uniform_100m_batched_launch(kc):
    n, d, k = 100_000_000, 3, 10
    print("full size: batched_100m_d3_k10, 256 nodes x 10 boxes", flush=True)
    x = datagen.uniform_points_device(n, d, 0)
    off, lo, hi = datagen.random_boxes(256, k, d, 0, wmin=1e-3, wmax=0.5)
    kc.autotune(x, n, _dev(off), _dev(lo), _dev(hi), with_cand=False, k_max=k)
    lb_raw, lb_safe, am, _ = kc.lower_bound(x, n, _dev(off), _dev(lo), _dev(hi), k_max=k)
    lb_raw, lb_safe, am = (t.cpu().numpy() for t in (lb_raw, lb_safe, am))
    X64 = _host(x, n)
    for m in (0, 99, 255):
        _check_node(kc, X64, x, m, off, lo, hi, lb_raw, lb_safe, am, d)
