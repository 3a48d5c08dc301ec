"""CPU oracle for the K-center branch-and-bound: TEST INFRASTRUCTURE ONLY.

A plain, serial, float64 implementation of what the device path computes,
written from the paper (Ren et al., arXiv 2301.00061). Only the test suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
it; the device library never does. It shares no code with the device path.

The arithmetic lives in ``kc_oracle.c`` (built with gcc into
``libkc_oracle.so`` by :func:`build`); this module only marshals numpy arrays.
``mlp.py`` holds the float64 reference of the branching network.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libkc_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
               os.path.join(_HERE, "kc_oracle.c"), "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        P = C.POINTER
        d64, i64, i32 = C.c_double, C.c_int64, C.c_int32
        pd, pi64, pi32 = P(d64), P(i64), P(i32)
        L.kco_point_box_min_dist2.restype = d64
        L.kco_point_box_min_dist2.argtypes = [pd, pd, pd, C.c_int]
        L.kco_point_box_max_dist2.restype = d64
        L.kco_point_box_max_dist2.argtypes = [pd, pd, pd, C.c_int]
        L.kco_dist2.restype = d64
        L.kco_dist2.argtypes = [pd, pd, C.c_int]
        L.kco_lower_bound.argtypes = [pd, i64, C.c_int, i32, pi32, pd, pd, pd, pi64]
        L.kco_candidates.argtypes = [pd, i64, C.c_int, i32, pd, pd, pi64]
        L.kco_objective.argtypes = [pd, i64, C.c_int, i32, C.c_int, pd, pd, pi64]
        L.kco_tighten_node.restype = i64
        L.kco_tighten_node.argtypes = [pd, i64, C.c_int, C.c_int, pd, pd, d64, pi32, pd,
                                       pd, pd, pi64, pd, pd, pi64, pi64, P(C.c_int8)]
        L.kco_tightened_box.restype = C.c_int
        L.kco_tightened_box.argtypes = [C.c_int, C.c_int, pd, pd, d64, pi32, pd, pd, pd, pi64,
                                        pd, pd, pi64, pd, pd]
        L.kco_symmetry.restype = C.c_int
        L.kco_symmetry.argtypes = [C.c_int, C.c_int, pd, pd]
        L.kco_reduce_flags.argtypes = [pd, i64, C.c_int, i32, pi32, pd, pd, pi32, pd, d64, d64,
                                       P(C.c_uint8)]
        L.kco_fft.argtypes = [pd, i64, C.c_int, C.c_int, i64, pi64]
        L.kco_brute_force.argtypes = [pd, i64, C.c_int, C.c_int, pd, pi64]
        L.kco_solve.restype = C.c_int
        L.kco_solve.argtypes = [pd, i64, C.c_int, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


class Opts(C.Structure):
    _fields_ = [("k", C.c_int32), ("i_sr", C.c_int32), ("use_bt", C.c_int32),
                ("use_seeds", C.c_int32), ("max_refs", C.c_int32), ("fft_start", C.c_int64),
                ("max_nodes", C.c_int64), ("eps", C.c_double)]


class Result(C.Structure):
    _fields_ = [("obj", C.c_double), ("lb", C.c_double), ("fft_obj", C.c_double),
                ("centers", C.c_int64 * 64), ("nodes", C.c_int64), ("n_active", C.c_int64),
                ("seeds_found", C.c_int32), ("status", C.c_int32)]


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _pts(X):
    X = _f64(X)
    if X.ndim == 1:
        X = X[:, None]
    return X, X.shape[0], X.shape[1]


def point_box_min_dist2(x, lo, hi) -> float:
    x, lo, hi = _f64(x), _f64(lo), _f64(hi)
    return lib().kco_point_box_min_dist2(_p(x, C.c_double), _p(lo, C.c_double), _p(hi, C.c_double), x.size)


def point_box_max_dist2(x, lo, hi) -> float:
    x, lo, hi = _f64(x), _f64(lo), _f64(hi)
    return lib().kco_point_box_max_dist2(_p(x, C.c_double), _p(lo, C.c_double), _p(hi, C.c_double), x.size)


def lower_bound(X, box_off, lo, hi):
    """Per node (CSR boxes) beta(M) and its argmax sample."""
    X, n, d = _pts(X)
    box_off, lo, hi = _i32(box_off), _f64(lo), _f64(hi)
    m = box_off.size - 1
    lb = np.zeros(m)
    am = np.zeros(m, dtype=np.int64)
    lib().kco_lower_bound(_p(X, C.c_double), n, d, m, _p(box_off, C.c_int32), _p(lo, C.c_double),
                          _p(hi, C.c_double), _p(lb, C.c_double), _p(am, C.c_int64))
    return lb, am


def candidates(X, lo, hi):
    X, n, d = _pts(X)
    lo, hi = _f64(lo).reshape(-1, d), _f64(hi).reshape(-1, d)
    nb = lo.shape[0]
    cand = np.zeros(nb, dtype=np.int64)
    lib().kco_candidates(_p(X, C.c_double), n, d, nb, _p(lo, C.c_double), _p(hi, C.c_double),
                         _p(cand, C.c_int64))
    return cand


def objective(X, centers):
    """centers [n_sets, k, d] -> (obj[n_sets], argmax[n_sets])."""
    X, n, d = _pts(X)
    c = _f64(centers)
    if c.ndim == 2:
        c = c[None]
    ns, k = c.shape[0], c.shape[1]
    obj = np.zeros(ns)
    am = np.zeros(ns, dtype=np.int64)
    lib().kco_objective(_p(X, C.c_double), n, d, ns, k, _p(c, C.c_double), _p(obj, C.c_double),
                        _p(am, C.c_int64))
    return obj, am


def tighten_node(X, lo, hi, alpha, ref_off=None, ref=None, want_labels=False):
    X, n, d = _pts(X)
    lo, hi = _f64(lo).reshape(-1, d), _f64(hi).reshape(-1, d)
    k = lo.shape[0]
    if ref_off is None:
        ref_off = np.zeros(k + 1, dtype=np.int32)
        ref = np.zeros((1, d))
    ref_off, ref = _i32(ref_off), _f64(ref).reshape(-1, d)
    if ref.size == 0:
        ref = np.zeros((1, d))
    bbl, bbh = np.zeros((k, d)), np.zeros((k, d))
    amn, amx = np.zeros((k, d)), np.zeros((k, d))
    nin, nasg = np.zeros(k, dtype=np.int64), np.zeros(k, dtype=np.int64)
    labels = np.zeros(n, dtype=np.int8) if want_labels else None
    far = np.zeros(k, dtype=np.int64)
    n_ex = lib().kco_tighten_node(
        _p(X, C.c_double), n, d, k, _p(lo, C.c_double), _p(hi, C.c_double), float(alpha),
        _p(ref_off, C.c_int32), _p(ref, C.c_double), _p(bbl, C.c_double), _p(bbh, C.c_double),
        _p(nin, C.c_int64), _p(amn, C.c_double), _p(amx, C.c_double), _p(nasg, C.c_int64),
        _p(far, C.c_int64), _p(labels, C.c_int8) if labels is not None else None)
    return dict(bb_lo=bbl, bb_hi=bbh, n_in=nin, asg_min=amn, asg_max=amx, n_asg=nasg,
                asg_far=far, n_excluded=int(n_ex), labels=labels)


def tightened_box(lo, hi, alpha, agg, ref_off=None, ref=None):
    lo, hi = _f64(lo), _f64(hi)
    k, d = lo.shape
    if ref_off is None:
        ref_off = np.zeros(k + 1, dtype=np.int32)
        ref = np.zeros((1, d))
    ref_off, ref = _i32(ref_off), _f64(ref).reshape(-1, d)
    if ref.size == 0:
        ref = np.zeros((1, d))
    lo2, hi2 = np.zeros((k, d)), np.zeros((k, d))
    inf = lib().kco_tightened_box(
        d, k, _p(lo, C.c_double), _p(hi, C.c_double), float(alpha), _p(ref_off, C.c_int32),
        _p(ref, C.c_double), _p(_f64(agg["bb_lo"]), C.c_double), _p(_f64(agg["bb_hi"]), C.c_double),
        _p(np.ascontiguousarray(agg["n_in"], dtype=np.int64), C.c_int64),
        _p(_f64(agg["asg_min"]), C.c_double), _p(_f64(agg["asg_max"]), C.c_double),
        _p(np.ascontiguousarray(agg["n_asg"], dtype=np.int64), C.c_int64),
        _p(lo2, C.c_double), _p(hi2, C.c_double))
    return bool(inf), lo2, hi2


def symmetry(lo, hi):
    lo, hi = _f64(lo).copy(), _f64(hi).copy()
    k, d = lo.shape
    empty = lib().kco_symmetry(d, k, _p(lo, C.c_double), _p(hi, C.c_double))
    return bool(empty), lo, hi


def reduce_flags(X, box_off, lo, hi, ref_off, ref, beta, alpha):
    X, n, d = _pts(X)
    box_off, lo, hi = _i32(box_off), _f64(lo), _f64(hi)
    ref_off = _i32(ref_off)
    ref = _f64(ref).reshape(-1, d)
    if ref.size == 0:
        ref = np.zeros((1, d))
    keep = np.zeros(n, dtype=np.uint8)
    lib().kco_reduce_flags(_p(X, C.c_double), n, d, box_off.size - 1, _p(box_off, C.c_int32),
                           _p(lo, C.c_double), _p(hi, C.c_double), _p(ref_off, C.c_int32),
                           _p(ref, C.c_double), float(beta), float(alpha), _p(keep, C.c_uint8))
    return keep


def fft(X, k, s0=0):
    X, n, d = _pts(X)
    T = np.zeros(k, dtype=np.int64)
    lib().kco_fft(_p(X, C.c_double), n, d, k, int(s0), _p(T, C.c_int64))
    return T


def brute_force(X, k):
    X, n, d = _pts(X)
    best = np.zeros(1)
    ids = np.zeros(k, dtype=np.int64)
    lib().kco_brute_force(_p(X, C.c_double), n, d, k, _p(best, C.c_double), _p(ids, C.c_int64))
    return float(best[0]), ids


def solve(X, k, i_sr=10, use_bt=True, use_seeds=True, max_refs=50, fft_start=0, max_nodes=0,
          eps=0.0):
    """Algorithm 1 to the global optimum; returns a dict of the result."""
    X, n, d = _pts(X)
    o = Opts(k=k, i_sr=i_sr, use_bt=int(use_bt), use_seeds=int(use_seeds), max_refs=int(max_refs),
             fft_start=int(fft_start), max_nodes=int(max_nodes), eps=float(eps))
    r = Result()
    rc = lib().kco_solve(_p(X, C.c_double), n, d, C.byref(o), C.byref(r))
    if rc != 0:
        raise ValueError("kco_solve rejected its arguments")
    return dict(obj=r.obj, lb=r.lb, fft_obj=r.fft_obj, centers=np.array(r.centers[:k]),
                nodes=r.nodes, n_active=r.n_active, seeds_found=bool(r.seeds_found),
                status=r.status)
