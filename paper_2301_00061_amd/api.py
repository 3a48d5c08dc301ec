"""Torch-tensor front end of libkc: the same calls as include/kc.h.

Torch supplies device memory and the current stream; every computation runs in
the library's HIP kernels. Samples are a float32 CUDA tensor ``x`` of shape
``[d, ld]`` (structure of arrays) with ``n <= ld`` valid columns.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import Nodes, Opts, Points, Refs, Result


class KCError(RuntimeError):
    pass


class Handle:
    """Owns a kc_handle (scratch memory and autotune table) for one device."""

    def __init__(self, device: int = 0, tune_cache: str | None = None):
        self.lib = _lib.load()
        self.ptr = C.c_void_p()
        self.device = device
        rc = self.lib.kc_create(C.byref(self.ptr), device,
                                tune_cache.encode() if tune_cache else None)
        if rc != 0:
            raise KCError(f"kc_create failed with status {rc}")

    def check(self, rc: int, what: str) -> None:
        if rc != 0:
            msg = self.lib.kc_last_error(self.ptr)
            raise KCError(f"{what}: status {rc}: {msg.decode() if msg else ''}")

    def close(self) -> None:
        if self.ptr:
            self.lib.kc_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles: dict[int, Handle] = {}


def handle(device: int | None = None) -> Handle:
    if device is None:
        device = torch.cuda.current_device()
    if device not in _handles:
        _handles[device] = Handle(device)
    return _handles[device]


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(0 if t is None else t.data_ptr())


def points(x: torch.Tensor, n: int) -> Points:
    assert x.is_cuda and x.dtype == torch.float32 and x.dim() == 2 and x.is_contiguous()
    d, ld = x.shape
    assert 0 < n <= ld
    return Points(x.data_ptr(), int(n), int(ld), int(d), 0)


def nodes(box_off: torch.Tensor, lo: torch.Tensor, hi: torch.Tensor, k_max: int | None = None) -> Nodes:
    assert box_off.dtype == torch.int32 and lo.dtype == torch.float32 and hi.dtype == torch.float32
    assert lo.is_contiguous() and hi.is_contiguous() and box_off.is_contiguous()
    n_nodes = box_off.numel() - 1
    n_boxes = lo.shape[0]
    if k_max is None:
        off = box_off.cpu().numpy()
        k_max = int(np.max(np.diff(off))) if n_nodes > 0 else 1
    return Nodes(int(n_nodes), int(n_boxes), int(max(1, k_max)), 0, box_off.data_ptr(),
                 lo.data_ptr(), hi.data_ptr())


def refs(ref_off: torch.Tensor | None, ref: torch.Tensor | None, max_per_box: int | None = None):
    if ref_off is None:
        return None
    assert ref_off.dtype == torch.int32 and ref.dtype == torch.float32
    n_refs = ref.shape[0] if ref.dim() > 1 else 0
    if max_per_box is None:
        off = ref_off.cpu().numpy()
        max_per_box = int(np.max(np.diff(off))) if off.size > 1 else 0
    return Refs(int(n_refs), int(max_per_box), ref_off.data_ptr(), ref.data_ptr() if n_refs else 0)


def lower_bound(x, n, box_off, lo, hi, k_max=None, want_cand=False, h: Handle | None = None,
                out=None, noalloc: bool = False):
    """Section 3.1 lower bound per node; returns (lb_raw, lb_safe, argmax, cand|None).

    ``out`` (optional) is a tuple of preallocated output tensors in that order;
    ``noalloc`` calls ``kc_lower_bound_noalloc`` (static device scratch)."""
    h = h or handle()
    P = points(x, n)
    M = nodes(box_off, lo, hi, k_max)
    dev = x.device
    if out is None:
        lb_raw = torch.empty(M.n_nodes, dtype=torch.float32, device=dev)
        lb_safe = torch.empty(M.n_nodes, dtype=torch.float64, device=dev)
        am = torch.empty(M.n_nodes, dtype=torch.int64, device=dev)
        cand = torch.empty(max(1, M.n_boxes), dtype=torch.int64, device=dev) if want_cand else None
    else:
        lb_raw, lb_safe, am, cand = out
    fn = h.lib.kc_lower_bound_noalloc if noalloc else h.lib.kc_lower_bound
    name = "kc_lower_bound_noalloc" if noalloc else "kc_lower_bound"
    h.check(fn(h.ptr, C.byref(P), C.byref(M), _ptr(lb_raw), _ptr(lb_safe), _ptr(am), _ptr(cand),
               _stream()), name)
    return lb_raw, lb_safe, am, (cand[:M.n_boxes] if cand is not None else None)


def objective(x, n, centers: torch.Tensor, precision: int = 32, h: Handle | None = None):
    """Eq (12) per candidate set: centers [n_sets, k, d] float32 -> (obj f64, argmax i64)."""
    h = h or handle()
    P = points(x, n)
    centers = centers.contiguous()
    if centers.dim() == 2:
        centers = centers[None]
    ns, k = centers.shape[0], centers.shape[1]
    obj = torch.empty(ns, dtype=torch.float64, device=x.device)
    am = torch.empty(ns, dtype=torch.int64, device=x.device)
    h.check(h.lib.kc_objective(h.ptr, C.byref(P), ns, k, _ptr(centers), precision, _ptr(obj),
                               _ptr(am), _stream()), "kc_objective")
    return obj, am


def objective_screen(x, n, centers: torch.Tensor, cut: float, floor=None,
                     h: Handle | None = None):
    """Float32 eq (12) screened at `cut` (see kc_objective_screen): exact for
    sets at or below the cut; a set above it may report a lower value above
    the cut. floor (float64 device tensor [n_sets], optional): lower bounds of
    the sets' objectives. Returns (obj f64, argmax i64)."""
    h = h or handle()
    P = points(x, n)
    centers = centers.contiguous()
    if centers.dim() == 2:
        centers = centers[None]
    ns, k = centers.shape[0], centers.shape[1]
    obj = torch.empty(ns, dtype=torch.float64, device=x.device)
    am = torch.empty(ns, dtype=torch.int64, device=x.device)
    if floor is not None:
        floor = floor.to(dtype=torch.float64).contiguous()
    h.check(h.lib.kc_objective_screen(h.ptr, C.byref(P), ns, k, _ptr(centers), float(cut),
                                      _ptr(floor), _ptr(obj), _ptr(am), _stream()),
            "kc_objective_screen")
    return obj, am


def tighten(x, n, box_off, lo, hi, alpha, ref_off=None, ref=None, labels=False, k_max=None,
            max_refs=None, h: Handle | None = None):
    """Algorithms 3-4 aggregates per box (see kc_tighten)."""
    h = h or handle()
    P = points(x, n)
    M = nodes(box_off, lo, hi, k_max)
    R = refs(ref_off, ref, max_refs)
    dev, nb, d = x.device, M.n_boxes, P.d
    out = dict(
        bb_lo=torch.empty((nb, d), dtype=torch.float32, device=dev),
        bb_hi=torch.empty((nb, d), dtype=torch.float32, device=dev),
        n_in=torch.empty(nb, dtype=torch.int32, device=dev),
        asg_min=torch.empty((nb, d), dtype=torch.float32, device=dev),
        asg_max=torch.empty((nb, d), dtype=torch.float32, device=dev),
        n_asg=torch.empty(nb, dtype=torch.int32, device=dev),
        n_excl=torch.empty(M.n_nodes, dtype=torch.int32, device=dev),
        asg_far=torch.empty(max(1, nb), dtype=torch.int64, device=dev),
        labels=torch.empty(n, dtype=torch.int8, device=dev) if labels else None)
    h.check(h.lib.kc_tighten(h.ptr, C.byref(P), C.byref(M), float(alpha),
                             C.byref(R) if R is not None else None, _ptr(out["bb_lo"]),
                             _ptr(out["bb_hi"]), _ptr(out["n_in"]), _ptr(out["asg_min"]),
                             _ptr(out["asg_max"]), _ptr(out["n_asg"]), _ptr(out["n_excl"]),
                             _ptr(out["asg_far"]), _ptr(out["labels"]), _stream()), "kc_tighten")
    out["asg_far"] = out["asg_far"][:nb]
    return out


def reduce(x, n, box_off, lo, hi, beta, alpha, ref_off=None, ref=None, idx_in=None,
           want_keep=False, k_max=None, max_refs=None, h: Handle | None = None):
    """Algorithm 5: returns (x_out [d, ld], idx_out uint32 as int32 tensor, n_out, keep|None)."""
    h = h or handle()
    P = points(x, n)
    M = nodes(box_off, lo, hi, k_max)
    R = refs(ref_off, ref, max_refs)
    dev = x.device
    x_out = torch.empty_like(x)
    idx_out = torch.empty(x.shape[1], dtype=torch.int32, device=dev)
    n_out = torch.empty(1, dtype=torch.int64, device=dev)
    keep = torch.empty(n, dtype=torch.uint8, device=dev) if want_keep else None
    h.check(h.lib.kc_reduce(h.ptr, C.byref(P), _ptr(idx_in), C.byref(M),
                            C.byref(R) if R is not None else None, float(beta), float(alpha),
                            _ptr(keep), _ptr(x_out), _ptr(idx_out), x.shape[1], _ptr(n_out),
                            _stream()), "kc_reduce")
    return x_out, idx_out, n_out, keep


def fft(x, n, k, starts, h: Handle | None = None):
    """Algorithm 2 from every start in `starts` (one float64 objective launch per
    step over all trials): returns (ids int64 [trials, k], obj float64 [trials])."""
    h = h or handle()
    P = points(x, n)
    st = np.ascontiguousarray(np.asarray(starts, dtype=np.int64))
    ids = np.zeros((len(st), k), dtype=np.int64)
    obj = np.zeros(len(st), dtype=np.float64)
    h.check(h.lib.kc_fft(h.ptr, C.byref(P), int(k), len(st), st.ctypes.data, ids.ctypes.data,
                         obj.ctypes.data, _stream()), "kc_fft")
    return ids, obj


def autotune_tighten(x, n, box_off, lo, hi, alpha, ref_off=None, ref=None, k_max=None,
                     max_refs=None, h: Handle | None = None) -> float:
    """Tile sweep of kc_tighten for this shape; returns the best time in ms."""
    h = h or handle()
    P = points(x, n)
    M = nodes(box_off, lo, hi, k_max)
    R = refs(ref_off, ref, max_refs)
    ms = C.c_double()
    h.check(h.lib.kc_autotune_tighten(h.ptr, C.byref(P), C.byref(M), float(alpha),
                                      C.byref(R) if R is not None else None, C.byref(ms),
                                      _stream()), "kc_autotune_tighten")
    return ms.value


def autotune(x, n, box_off, lo, hi, with_cand=False, k_max=None, h: Handle | None = None) -> float:
    h = h or handle()
    P = points(x, n)
    M = nodes(box_off, lo, hi, k_max)
    ms = C.c_double()
    h.check(h.lib.kc_autotune(h.ptr, C.byref(P), C.byref(M), int(with_cand), C.byref(ms),
                              _stream()), "kc_autotune")
    return ms.value


# --------------------------------------------------------- branching network

def mlp_forward(w_bf16, feat, want_act=False, h: Handle | None = None):
    h = h or handle()
    rows = feat.shape[0]
    score = torch.empty(rows, dtype=torch.float32, device=feat.device)
    act = torch.empty((rows, 192), dtype=torch.float32, device=feat.device) if want_act else None
    h.check(h.lib.kc_mlp_forward(h.ptr, _ptr(w_bf16), _ptr(feat.contiguous()), rows, _ptr(score),
                                 _ptr(act), _stream()), "kc_mlp_forward")
    return score, act


def mlp_backward(w_bf16, feat, act, dscore, h: Handle | None = None):
    h = h or handle()
    dw = torch.empty(_lib.MLP_PARAMS, dtype=torch.float32, device=feat.device)
    h.check(h.lib.kc_mlp_backward(h.ptr, _ptr(w_bf16), _ptr(feat.contiguous()), _ptr(act),
                                  _ptr(dscore.contiguous()), feat.shape[0], _ptr(dw), _stream()),
            "kc_mlp_backward")
    return dw


def mlp_loss(score, grp_off, target, h: Handle | None = None):
    h = h or handle()
    rows = score.shape[0]
    dscore = torch.empty(rows, dtype=torch.float32, device=score.device)
    loss = torch.empty(1, dtype=torch.float32, device=score.device)
    h.check(h.lib.kc_mlp_loss(h.ptr, _ptr(score), _ptr(grp_off), _ptr(target),
                              grp_off.numel() - 1, rows, _ptr(dscore), _ptr(loss), _stream()),
            "kc_mlp_loss")
    return loss, dscore


def mlp_adam(w32, w_bf16, dw, m, v, step, lr, h: Handle | None = None):
    h = h or handle()
    h.check(h.lib.kc_mlp_adam(h.ptr, _ptr(w32), _ptr(w_bf16), _ptr(dw), _ptr(m), _ptr(v),
                              int(step), float(lr), _stream()), "kc_mlp_adam")


# ---------------------------------------------------------------- driver

def solve(x, n, k, batch=64, i_sr=4, use_bt=True, use_seeds=True, max_refs=50, branching=0,
          fft_start=0, max_nodes=0, eps_rel=1e-6, time_limit_s=0.0, mlp_w=None, verbose=False,
          sb=None, keep_order=False, node_sr=0, autotune=False, h: Handle | None = None) -> dict:
    """Algorithm 1 on device-resident samples (synchronous)."""
    h = h or handle()
    P = points(x, n)
    o = Opts(k=k, batch=batch, i_sr=i_sr, use_bt=int(use_bt), use_seeds=int(use_seeds),
             max_refs=int(max_refs), branching=int(branching), fft_start=int(fft_start),
             max_nodes=int(max_nodes), eps_rel=float(eps_rel), time_limit_s=float(time_limit_s),
             mlp_w=mlp_w.data_ptr() if mlp_w is not None else None, verbose=int(verbose),
             keep_order=int(bool(keep_order)), node_sr=int(node_sr), autotune=int(bool(autotune)))
    if sb is not None:
        # strong-branching label recording into host arrays (see StrongBranchingBuffer)
        o.sb_first, o.sb_every, o.sb_cap = sb.first, sb.every, sb.cap
        o.sb_feat = sb.feat.ctypes.data
        o.sb_score = sb.score.ctypes.data
        o.sb_node = sb.node.ctypes.data
        if sb.lo is not None:
            o.sb_lo = sb.lo.ctypes.data
            o.sb_hi = sb.hi.ctypes.data
            o.sb_ka = sb.ka.ctypes.data
            o.sb_bounds = sb.bounds.ctypes.data
    r = Result()
    torch.cuda.synchronize()
    h.check(h.lib.kc_solve(h.ptr, C.byref(P), C.byref(o), C.byref(r)), "kc_solve")
    return dict(obj=r.obj, lb=r.lb, gap=r.gap, fft_obj=r.fft_obj,
                centers=np.array(r.centers[:k]), nodes=r.nodes, passes=r.passes, evals=r.evals,
                n_active=r.n_active, seconds=r.seconds, lb_kernel_ms=r.lb_kernel_ms,
                tighten_kernel_ms=r.tighten_kernel_ms, tighten_evals=r.tighten_evals,
                seeds_found=bool(r.seeds_found), status=r.status, sb_rows=r.sb_rows,
                sb_nodes=r.sb_nodes, node_sr_tries=r.node_sr_tries, node_sr_kept=r.node_sr_kept,
                obj_kernel_ms=r.obj_kernel_ms, obj_evals=r.obj_evals)


class StrongBranchingBuffer:
    """Host arrays kc_solve fills with strong-branching rows (features,
    product score, labelled-node ordinal)."""

    def __init__(self, cap: int, first: int = 32, every: int = 8, kd: int | None = None):
        self.cap, self.first, self.every = int(cap), int(first), int(every)
        self.feat = np.zeros((self.cap, 32), dtype=np.float32)
        self.score = np.zeros(self.cap, dtype=np.float32)
        self.node = np.zeros(self.cap, dtype=np.int32)
        # with kd = K*D: each row's node boxes, candidate (k, a), node LB and alpha
        self.lo = self.hi = self.ka = self.bounds = None
        if kd is not None:
            self.lo = np.zeros((self.cap, kd), dtype=np.float32)
            self.hi = np.zeros((self.cap, kd), dtype=np.float32)
            self.ka = np.zeros((self.cap, 2), dtype=np.int32)
            self.bounds = np.zeros((self.cap, 2), dtype=np.float64)


def rel_margin(d: int) -> float:
    return _lib.load().kc_rel_margin(d)


def abs_margin(d: int) -> float:
    return _lib.load().kc_abs_margin(d)


def to_device_soa(x_rows: np.ndarray, device="cuda", ld: int | None = None) -> torch.Tensor:
    """Row-major float32 [n, d] host array -> SoA device tensor [d, ld] (ld % 64 == 0)."""
    n, d = x_rows.shape
    if ld is None:
        ld = (n + 63) // 64 * 64
    t = torch.zeros((d, ld), dtype=torch.float32)
    t[:, :n] = torch.from_numpy(np.ascontiguousarray(x_rows.T))
    return t.to(device)
