"""GPU parity of the branching-network kernels against the float64 reference
(oracle/mlp.py) on identical bf16 weights and bf16-rounded features."""
import numpy as np
import pytest
import torch

import datagen
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2301_00061_amd import api
    return api


def _weights(seed):
    w32 = datagen.mlp_init_weights(seed)
    rng = np.random.default_rng(seed)
    p = 0
    for o, i in mlp.SIZES:  # nonzero biases so every ReLU sees both signs
        p += o * i
        w32[p:p + o] = rng.uniform(-0.3, 0.3, o).astype(np.float32)
        p += o
    wb = mlp.bf16_round(w32)
    bits = (wb.view(np.uint32) >> 16).astype(np.uint16)
    return w32, wb.astype(np.float64), torch.from_numpy(bits.view(np.int16)).cuda()


def _feat(rows, seed):
    f = np.random.default_rng(seed).normal(size=(rows, 32)).astype(np.float32)
    return f, mlp.bf16_round(f).astype(np.float64)


@pytest.mark.parametrize("rows", [1, 255, 4097])
def test_forward_parity(kc, rows):
    _, w64, wd = _weights(rows)
    f32, f64 = _feat(rows, rows + 1)
    s_o, acts = mlp.forward(w64, f64)
    s_g, act_g = kc.mlp_forward(wd, torch.from_numpy(f32).cuda(), want_act=True)
    s_g = s_g.cpu().numpy().astype(np.float64)
    scale = np.abs(s_o).max() + 1e-30
    assert np.max(np.abs(s_g - s_o)) <= 2e-5 * scale
    a = act_g.cpu().numpy().astype(np.float64)
    for li in range(3):
        ref = acts[li]
        assert np.max(np.abs(a[:, 64 * li:64 * (li + 1)] - ref)) <= 2e-5 * (np.abs(ref).max() + 1e-30)


@pytest.mark.parametrize("rows", [1, 300, 5000])
def test_backward_parity(kc, rows):
    _, w64, wd = _weights(7 + rows)
    f32, f64 = _feat(rows, rows)
    ds = np.random.default_rng(rows).normal(size=rows).astype(np.float32)
    g_o = mlp.backward(w64, f64, ds.astype(np.float64))
    fd = torch.from_numpy(f32).cuda()
    _, act = kc.mlp_forward(wd, fd, want_act=True)
    g_g = kc.mlp_backward(wd, fd, act, torch.from_numpy(ds).cuda()).cpu().numpy().astype(np.float64)
    err = np.abs(g_g - g_o)
    assert np.max(err) <= 1e-3 * np.abs(g_o).max()
    # each parameter block to 1e-3 of its own scale
    p = 0
    for o, i in mlp.SIZES:
        for n in (o * i, o):
            blk = slice(p, p + n)
            assert np.max(err[blk]) <= 1e-3 * (np.abs(g_o[blk]).max() + 1e-30)
            p += n
    # reproducible
    g2 = kc.mlp_backward(wd, fd, act, torch.from_numpy(ds).cuda()).cpu().numpy()
    assert np.array_equal(g2.astype(np.float64), g_g)


def test_loss_parity(kc):
    rng = np.random.default_rng(3)
    sizes = rng.integers(1, 40, 200)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    rows = int(off[-1])
    score = rng.normal(size=rows).astype(np.float32)
    tgt = np.array([rng.integers(0, s) for s in sizes], dtype=np.int32)
    l_o, d_o = mlp.loss_grad(score.astype(np.float64), off, tgt)
    l_g, d_g = kc.mlp_loss(torch.from_numpy(score).cuda(), torch.from_numpy(off).cuda(),
                           torch.from_numpy(tgt).cuda())
    assert abs(l_g.item() - l_o) <= 1e-5 * abs(l_o)
    assert np.max(np.abs(d_g.cpu().numpy() - d_o)) <= 1e-6


def test_adam_parity(kc):
    w32, _, wd = _weights(11)
    rng = np.random.default_rng(11)
    g = rng.normal(size=w32.size).astype(np.float32) * 0.01
    m = np.zeros_like(w32)
    v = np.zeros_like(w32)
    W, M, V = (torch.from_numpy(a.copy()).cuda() for a in (w32, m, v))
    G = torch.from_numpy(g).cuda()
    w_o, m_o, v_o = w32.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in (1, 2, 3):
        kc.mlp_adam(W, wd, G, M, V, step, 1e-3)
        w_o, m_o, v_o = mlp.adam(w_o, m_o, v_o, g.astype(np.float64), step, 1e-3)
    wg = W.cpu().numpy()
    assert np.max(np.abs(wg - w_o)) <= 1e-6 * max(1.0, np.abs(w_o).max())
    bits = (mlp.bf16_round(wg).view(np.uint32) >> 16).astype(np.uint16)
    assert np.array_equal(wd.cpu().numpy().view(np.uint16), bits)


def test_training_reduces_loss(kc):
    """A few hundred Adam steps of the device kernels learn to pick the row
    with the largest first feature in each group."""
    rng = np.random.default_rng(5)
    sizes = rng.integers(2, 12, 256)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    rows = int(off[-1])
    f = rng.normal(size=(rows, 32)).astype(np.float32)
    tgt = np.array([int(np.argmax(f[off[i]:off[i + 1], 0])) for i in range(len(sizes))], dtype=np.int32)
    w32, _, wd = _weights(5)
    W = torch.from_numpy(w32.copy()).cuda()
    M = torch.zeros_like(W)
    V = torch.zeros_like(W)
    fd = torch.from_numpy(f).cuda()
    od, td = torch.from_numpy(off).cuda(), torch.from_numpy(tgt).cuda()
    losses = []
    for step in range(1, 301):
        s, act = kc.mlp_forward(wd, fd, want_act=True)
        loss, ds = kc.mlp_loss(s, od, td)
        dw = kc.mlp_backward(wd, fd, act, ds)
        kc.mlp_adam(W, wd, dw, M, V, step, 3e-3)
        losses.append(loss.item())
    assert losses[-1] < 0.3 * losses[0]
