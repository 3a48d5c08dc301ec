"""Pins for the float64 branching-network reference (oracle/mlp.py)."""
import numpy as np
import pytest

import datagen
from oracle import mlp


def _rand(seed, rows=17):
    w = mlp.bf16_round(datagen.mlp_init_weights(seed)).astype(np.float64)
    w[mlp.N_PARAMS - 1] = 0.3
    rng = np.random.default_rng(seed)
    # nonzero biases so every ReLU sees both signs
    for (o, i), p in zip(mlp.SIZES, np.cumsum([0] + [o * i + o for o, i in mlp.SIZES])[:-1]):
        w[p + o * i: p + o * i + o] = rng.uniform(-0.2, 0.2, o)
    feat = mlp.bf16_round(rng.normal(size=(rows, 32))).astype(np.float64)
    return w, feat


def test_parameter_count():
    assert mlp.N_PARAMS == 10497


def test_forward_hand_network():
    """Only feature 3 -> unit 0 -> unit 0 -> unit 0 -> output: a chain of ReLUs."""
    layers = [(np.zeros((o, i)), np.zeros(o)) for o, i in mlp.SIZES]
    layers[0][0][0, 3] = 2.0
    layers[1][0][0, 0] = 0.5
    layers[2][0][0, 0] = 3.0
    layers[3][0][0, 0] = -1.0
    layers[3][1][0] = 0.25
    w = mlp.pack(layers)
    f = np.zeros((3, 32))
    f[:, 3] = [1.0, -1.0, 0.5]
    s, _ = mlp.forward(w, f)
    # relu(relu(relu(2 f) * .5) * 3) * -1 + .25 = -3 relu(f) + .25
    assert np.allclose(s, [-2.75, 0.25, -1.25], rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_vs_central_differences(seed):
    w, feat = _rand(seed)
    rng = np.random.default_rng(seed + 5)
    ds = rng.normal(size=feat.shape[0])
    g = mlp.backward(w, feat, ds)
    idx = rng.choice(mlp.N_PARAMS, 300, replace=False)
    idx = np.concatenate([idx, [mlp.N_PARAMS - 1, mlp.N_PARAMS - 2, 0, 2048]])
    h = 1e-6
    for j in idx:
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        fd = (np.dot(ds, mlp.forward(wp, feat)[0]) - np.dot(ds, mlp.forward(wm, feat)[0])) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])), j


def test_loss_closed_form_and_gradient():
    # two candidates: loss = log(1 + exp(s_other - s_target))
    s = np.array([0.3, -1.2, 2.0, 0.1, 0.7])
    off = np.array([0, 2, 5])
    tgt = np.array([1, 0])
    loss, d = mlp.loss_grad(s, off, tgt)
    l0 = np.log1p(np.exp(0.3 + 1.2))
    l1 = -(2.0 - np.log(np.exp(2.0) + np.exp(0.1) + np.exp(0.7)))
    assert abs(loss - (l0 + l1) / 2) < 1e-14
    h = 1e-6
    for j in range(5):
        sp, sm = s.copy(), s.copy()
        sp[j] += h
        sm[j] -= h
        fd = (mlp.loss_grad(sp, off, tgt)[0] - mlp.loss_grad(sm, off, tgt)[0]) / (2 * h)
        assert abs(fd - d[j]) < 1e-8
    # gradients of one node sum to zero
    assert abs(d[:2].sum()) < 1e-15 and abs(d[2:].sum()) < 1e-15


def test_adam_first_step_is_signed_lr():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w2, m, v = mlp.adam(w, np.zeros(3), np.zeros(3), g, 1, 0.01)
    assert np.allclose(w2, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_bf16_rounding_ties_to_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -3.14159], dtype=np.float32)
    r = mlp.bf16_round(vals)
    # 1 + 2^-8 is the midpoint of 1 and 1 + 2^-7: ties to even -> 1
    # 1 + 3*2^-8 is the midpoint of 1+2^-7 and 1+2^-6: ties to even -> 1 + 2^-6
    assert r.tolist()[:4] == [1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7]
    assert abs(r[4] - (-3.140625)) < 1e-7
