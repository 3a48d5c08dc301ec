"""Seeded synthetic inputs for the K-center bound evaluation.

This module only draws random numbers and arranges them into arrays; it holds
none of the clustering arithmetic. Both the CPU oracle side (tests) and the GPU
side (tests, bench) take their inputs from here, so the two see identical data.

Conventions
-----------
* Every generator uses numpy's PCG64. Values are drawn in float64 and rounded
  once to float32; that float32 array *is* the dataset (the fp64 oracle sees the
  same values promoted exactly).
* Points are returned row-major ``(n, d)`` float32. ``to_soa`` produces the
  structure-of-arrays layout ``x[a*ld + s]`` the device library consumes.
* Large arrays are drawn in fixed-size chunks, each from its own child seed of
  ``SeedSequence(seed)``, so the result does not depend on the thread count.

The paper's synthetic sets are Gaussian clusters in two attributes with unstated
parameters (Section 6.1); the workloads below fix those parameters.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np

CHUNK = 1 << 22  # samples per independently seeded chunk


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _means(seed: int, k: int, d: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x6D65616E])))
    return rng.uniform(0.0, 1.0, size=(k, d))


def gaussian_mixture(n: int, d: int, k: int, std: float, seed: int,
                     outlier_frac: float = 0.0, outlier_lo: float = -0.5,
                     outlier_hi: float = 1.5, out: np.ndarray | None = None) -> np.ndarray:
    """Equal-weight mixture of ``k`` isotropic Gaussians, means ~ U[0,1]^d.

    With ``outlier_frac > 0`` the last ``round(n*outlier_frac)`` rows are drawn
    uniform in ``[outlier_lo, outlier_hi]^d`` and the rows are then shuffled.
    Component labels are i.i.d. categorical, so the inlier rows are already in
    random order.
    """
    n = int(n)
    means = _means(seed, k, d)
    n_out = int(round(n * outlier_frac))
    n_in = n - n_out
    x = out if out is not None else np.empty((n, d), dtype=np.float32)
    assert x.shape == (n, d) and x.dtype == np.float32
    n_chunks = (n + CHUNK - 1) // CHUNK
    children = np.random.SeedSequence([seed, 0x78]).spawn(max(1, n_chunks))

    def fill(ci: int) -> None:
        lo = ci * CHUNK
        hi = min(n, lo + CHUNK)
        rng = np.random.Generator(np.random.PCG64(children[ci]))
        m = hi - lo
        lab = rng.integers(0, k, size=m)
        z = rng.standard_normal(size=(m, d))
        v = means[lab] + std * z
        if hi > n_in:  # rows in the outlier range
            s = max(lo, n_in) - lo
            v[s:] = rng.uniform(outlier_lo, outlier_hi, size=(m - s, d))
        x[lo:hi] = v.astype(np.float32)

    if n_chunks <= 1:
        fill(0)
    else:
        with _cf.ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, range(n_chunks)))
    if n_out > 0:
        perm = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x70]))).permutation(n)
        x[:] = x[perm]
    return x


def uniform_points(n: int, d: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """``n`` points uniform in ``[lo, hi]^d`` (float32, row-major)."""
    n = int(n)
    x = np.empty((n, d), dtype=np.float32)
    n_chunks = (n + CHUNK - 1) // CHUNK
    children = np.random.SeedSequence([seed, 0x75]).spawn(max(1, n_chunks))

    def fill(ci: int) -> None:
        a = ci * CHUNK
        b = min(n, a + CHUNK)
        rng = np.random.Generator(np.random.PCG64(children[ci]))
        x[a:b] = rng.uniform(lo, hi, size=(b - a, d)).astype(np.float32)

    if n_chunks <= 1:
        fill(0)
    else:
        with _cf.ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, range(n_chunks)))
    return x


def random_boxes(n_nodes: int, k, d: int, seed: int, wmin: float = 1e-3,
                 wmax: float = 0.5, ragged: bool = False):
    """Ragged batch of center boxes in CSR form.

    Per node ``k`` boxes (or ``U{1..k}`` boxes when ``ragged``); each box has a
    center ~ U[0,1]^d and per-dimension width ``exp(U[ln wmin, ln wmax])``.
    Returns ``(box_off int32[n_nodes+1], lo float32[nb,d], hi float32[nb,d])``.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x62])))
    if ragged:
        ks = rng.integers(1, int(k) + 1, size=n_nodes)
    else:
        ks = np.full(n_nodes, int(k))
    off = np.zeros(n_nodes + 1, dtype=np.int32)
    off[1:] = np.cumsum(ks)
    nb = int(off[-1])
    c = rng.uniform(0.0, 1.0, size=(nb, d))
    w = np.exp(rng.uniform(np.log(wmin), np.log(wmax), size=(nb, d)))
    lo = (c - 0.5 * w).astype(np.float32)
    hi = (c + 0.5 * w).astype(np.float32)
    hi = np.maximum(hi, lo)
    return off, lo, hi


def random_centers(n_sets: int, k: int, d: int, seed: int) -> np.ndarray:
    """Candidate center sets ``[n_sets, k, d]`` uniform in [0,1]^d (float32)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x63])))
    return rng.uniform(0.0, 1.0, size=(n_sets, k, d)).astype(np.float32)


def to_soa(x: np.ndarray, ld: int | None = None) -> tuple[np.ndarray, int]:
    """Row-major ``(n, d)`` -> flat SoA ``x[a*ld + s]`` with ``ld`` a multiple of 64."""
    n, d = x.shape
    if ld is None:
        ld = (n + 63) // 64 * 64
    soa = np.zeros(d * ld, dtype=np.float32)
    for a in range(d):
        soa[a * ld: a * ld + n] = x[:, a]
    return soa, ld


# --- named workloads -------------------------------------------------------

def small_mixture(seed: int) -> np.ndarray:
    """N=2,000, D=2: three Gaussians (std 0.08), means ~ U[0,1]^2."""
    return gaussian_mixture(2000, 2, 3, 0.08, seed)


def mixture_10m_d4(seed: int) -> np.ndarray:
    """N=10^7, D=4: five Gaussians (std 0.1) plus 1% outliers ~ U[-0.5,1.5]^4."""
    return gaussian_mixture(10_000_000, 4, 5, 0.1, seed, outlier_frac=0.01)


def uniform_100m_d3(seed: int) -> np.ndarray:
    """N=10^8 points uniform in [0,1]^3."""
    return uniform_points(100_000_000, 3, seed)


def mixture_1b_d2(seed: int, n: int = 1_000_000_000) -> np.ndarray:
    """N=10^9, D=2: three Gaussians (std 0.05), means ~ U[0,1]^2 (8 GB as fp32)."""
    return gaussian_mixture(n, 2, 3, 0.05, seed)


def learned_instance(seed: int, n: int, d: int = 5, k: int | None = None):
    """Learned-branching instance: mixture of K Gaussians (std 0.1) in D=5.

    K ~ U{4..8} drawn from the seed unless given. Returns ``(x, K)``.
    """
    if k is None:
        k = learned_instance_k(seed)
    return gaussian_mixture(n, d, k, 0.1, seed), k


def mlp_init_weights(seed: int) -> np.ndarray:
    """Initial weights of the 32-64-64-64-1 branching network, flat float32 in
    the layout W1[64,32] b1 W2[64,64] b2 W3[64,64] b3 W4[1,64] b4: He-uniform
    matrices, zero biases."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x6D6C70])))
    parts = []
    for o, i in ((64, 32), (64, 64), (64, 64), (1, 64)):
        lim = np.sqrt(6.0 / i)
        parts.append(rng.uniform(-lim, lim, o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def gaussian_mixture_device(n: int, d: int, k: int, std: float, seed: int,
                            outlier_frac: float = 0.0, outlier_lo: float = -0.5,
                            outlier_hi: float = 1.5, device="cuda", ld: int | None = None):
    """Device-side generator for the large workloads (10^7..10^9 samples).

    Same family as ``gaussian_mixture`` (means from the same seed, i.i.d.
    categorical labels, float64 draws rounded once to float32) but drawn with
    torch's seeded device generator straight into the structure-of-arrays
    layout ``[d, ld]`` (padding zeroed). It is a different stream from the host
    generator: parity checks on these sizes copy the samples they need back to
    the host. Returns the float32 tensor ``[d, ld]``.
    """
    import torch
    n = int(n)
    if ld is None:
        ld = (n + 63) // 64 * 64
    means = torch.from_numpy(_means(seed, k, d)).to(device)  # [k, d] float64
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + 17)
    x = torch.zeros((d, ld), dtype=torch.float32, device=device)
    n_out = int(round(n * outlier_frac))
    n_in = n - n_out
    step = 1 << 25
    for a0 in range(0, n_in, step):
        m = min(step, n_in - a0)
        lab = torch.randint(0, k, (m,), generator=g, device=device)
        z = torch.randn((d, m), generator=g, device=device, dtype=torch.float64)
        x[:, a0:a0 + m] = (means[lab].T + std * z).to(torch.float32)
    for a0 in range(n_in, n, step):
        m = min(step, n - a0)
        u = torch.rand((d, m), generator=g, device=device, dtype=torch.float64)
        x[:, a0:a0 + m] = (outlier_lo + (outlier_hi - outlier_lo) * u).to(torch.float32)
    if n_out > 0:
        perm = torch.randperm(n, generator=g, device=device)
        for a in range(d):
            x[a, :n] = x[a, :n][perm]
    return x


def uniform_points_device(n: int, d: int, seed: int, device="cuda", ld: int | None = None):
    """Device-side ``n`` points uniform in [0,1]^d, layout ``[d, ld]``."""
    import torch
    n = int(n)
    if ld is None:
        ld = (n + 63) // 64 * 64
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + 29)
    x = torch.zeros((d, ld), dtype=torch.float32, device=device)
    step = 1 << 25
    for a0 in range(0, n, step):
        m = min(step, n - a0)
        x[:, a0:a0 + m] = torch.rand((d, m), generator=g, device=device, dtype=torch.float64).to(torch.float32)
    return x


def learned_instance_k(seed: int) -> int:
    """K ~ U{4..8} of the learned-branching instance with this seed."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x4B])))
    return int(rng.integers(4, 9))


def learned_instance_device(seed: int, n: int, d: int = 5, k: int | None = None, device="cuda"):
    """Device-side learned-branching instance (see ``learned_instance``):
    returns ``(x [d, ld] float32 tensor, K)``."""
    if k is None:
        k = learned_instance_k(seed)
    return gaussian_mixture_device(n, d, k, 0.1, seed, device=device), k
