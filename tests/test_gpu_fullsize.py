"""Parity at the benchmark's full sizes, in the launch configuration the bench
times (the autotuner's tile for the same shapes): every node's bound and every
box's candidate against the oracle over all samples (the oracle run on chunks
of the samples in parallel host threads, its chunk results combined by max /
min), and the float64 certificate over 10^9 samples bit for bit."""
import concurrent.futures as cf
import os

import numpy as np
import pytest
import torch

import datagen
import oracle

pytestmark = pytest.mark.gpu

# host threads for the oracle over all samples (the oracle's C calls run
# without the interpreter lock); the machine's CPU share is 16 threads
THREADS = max(1, min(16, os.cpu_count() or 1))


def _chunks(n, parts):
    step = (n + parts - 1) // parts
    return [(c0, min(n, c0 + step)) for c0 in range(0, n, step)]


def _oracle_lb_all(X64, off, lo64, hi64):
    """The oracle's lower bound of every node (CSR off) over all rows of X64:
    the maximum of its values over contiguous chunks of samples, evaluated in
    parallel."""
    parts = _chunks(len(X64), 4 * THREADS)
    with cf.ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(lambda c: oracle.lower_bound(X64[c[0]:c[1]], off, lo64, hi64)[0], parts))
    return np.max(np.stack(res), axis=0)


def _oracle_cand_dist_all(X64, lo64, hi64):
    """Per box: the oracle's least squared distance to the box midpoint over
    the samples inside the box (chunked, in parallel), +inf when it holds
    none."""
    parts = _chunks(len(X64), 4 * THREADS)
    mid = 0.5 * (lo64 + hi64)

    def one(c):
        sub = X64[c[0]:c[1]]
        cand = oracle.candidates(sub, lo64, hi64)
        dist = np.full(len(cand), np.inf)
        ok = cand >= 0
        dist[ok] = ((sub[cand[ok]] - mid[ok]) ** 2).sum(1)
        return dist

    with cf.ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(one, parts))
    return np.min(np.stack(res), axis=0)


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


def _check_nodes(kc, X64, off, lo, hi, lb_raw, lb_safe, am, d):
    """Every node's bound equals the oracle's over all samples within the
    margin, the safe bound lies below it, and the device's argmax sample
    attains it."""
    g, eta = kc.rel_margin(d), kc.abs_margin(d)
    lo64, hi64 = lo.astype(np.float64), hi.astype(np.float64)
    lb_o = _oracle_lb_all(X64, off, lo64, hi64)
    assert np.all(np.abs(lb_raw.astype(np.float64) - lb_o) <= g * lb_o + eta)
    assert np.all(lb_safe <= lb_o)
    for m in range(len(off) - 1):
        b0, b1 = int(off[m]), int(off[m + 1])
        v, _ = oracle.lower_bound(X64[int(am[m])][None], np.array([0, b1 - b0], dtype=np.int32),
                                  lo64[b0:b1], hi64[b0:b1])
        assert v[0] >= lb_o[m] - 2 * (g * lb_o[m] + eta), m
    return lo64, hi64


@pytest.mark.timeout(900)
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
    # every one of the 128 nodes and 640 boxes against the oracle over all samples
    lo64, hi64 = _check_nodes(kc, X64, off, lo, hi, lb_raw, lb_safe, am, d)
    do_all = _oracle_cand_dist_all(X64, lo64, hi64)
    assert np.any(np.isfinite(do_all)) and np.any(cand >= 0)
    for b in range(len(lo64)):
        cg, do = int(cand[b]), do_all[b]
        if not np.isfinite(do):
            assert cg == -1, b
            continue
        assert cg >= 0 and np.all((X64[cg] >= lo64[b]) & (X64[cg] <= hi64[b])), b
        mid = 0.5 * (lo64[b] + hi64[b])
        dg = ((X64[cg] - mid) ** 2).sum()
        assert dg <= do + 2 * g * do + 1e-6 * (1 + np.sqrt(do)) * max(1.0, np.abs(mid).max()), b


def _mixture_1b(kc):
    n, d, k = 1_000_000_000, 2, 3
    x = datagen.gaussian_mixture_device(n, d, k, 0.05, 0)
    means = datagen._means(0, k, d).astype(np.float32)
    off = np.array([0, k], dtype=np.int32)
    return n, d, k, x, off, means - 0.05, means + 0.05


@pytest.mark.timeout(900)
def test_mixture_1b_one_node_pass(kc):
    n, d, k, x, off, lo, hi = _mixture_1b(kc)
    print("full size: lb_1b_d2_k3, one node of 3 boxes over 10^9 samples", flush=True)
    kc.autotune(x, n, _dev(off), _dev(lo), _dev(hi), with_cand=False, k_max=k)
    lb_raw, lb_safe, am, _ = kc.lower_bound(x, n, _dev(off), _dev(lo), _dev(hi), k_max=k)
    lb_raw, lb_safe, am = (t.cpu().numpy() for t in (lb_raw, lb_safe, am))
    g, eta = kc.rel_margin(d), kc.abs_margin(d)
    lo64, hi64 = lo.astype(np.float64), hi.astype(np.float64)
    # the oracle's bound over all 10^9 samples, in chunks of 10^8
    lb_o = -1.0
    for c0 in range(0, n, 100_000_000):
        c1 = min(n, c0 + 100_000_000)
        X64 = x[:, c0:c1].T.contiguous().cpu().numpy().astype(np.float64)
        lb_o = max(lb_o, float(_oracle_lb_all(X64, off, lo64, hi64)[0]))
        del X64
    assert abs(float(lb_raw[0]) - lb_o) <= g * lb_o + eta
    assert lb_safe[0] <= lb_o
    # the argmax sample attains the value
    xs = x[:, int(am[0])].cpu().numpy().astype(np.float64)[None]
    v, _ = oracle.lower_bound(xs, off, lo64, hi64)
    assert v[0] >= lb_o - 2 * (g * lb_o + eta)


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


@pytest.mark.timeout(1200)
def test_uniform_100m_batched_launch(kc):
    n, d, k = 100_000_000, 3, 10
    print("full size: batched_100m_d3_k10, 256 nodes x 10 boxes", flush=True)
    x = datagen.uniform_points_device(n, d, 0)
    off, lo, hi = datagen.random_boxes(256, k, d, 0, wmin=1e-3, wmax=0.5)
    kc.autotune(x, n, _dev(off), _dev(lo), _dev(hi), with_cand=False, k_max=k)
    lb_raw, lb_safe, am, _ = kc.lower_bound(x, n, _dev(off), _dev(lo), _dev(hi), k_max=k)
    lb_raw, lb_safe, am = (t.cpu().numpy() for t in (lb_raw, lb_safe, am))
    X64 = _host(x, n)
    # every one of the 256 nodes against the oracle over all samples
    _check_nodes(kc, X64, off, lo, hi, lb_raw, lb_safe, am, d)
