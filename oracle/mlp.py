"""Float64 reference of the branching-score network: TEST INFRASTRUCTURE ONLY.

The paper branches on the widest center box at its midpoint (Section 3.3) and
has no learned component; the network here scores the (cluster, attribute)
candidates of a node instead, and this module is the plain reference its
device kernels are checked against.

Network: 32 features -> 64 -> 64 -> 64 -> 1, ReLU after each hidden layer.
Flat parameter layout (10,497 values), each matrix row-major [out][in]:
    W1[64,32] b1[64] W2[64,64] b2[64] W3[64,64] b3[64] W4[1,64] b4[1]
The device keeps bf16 weights (fp32 master copy) and bf16 inputs with fp32
accumulation; callers pass the bf16-rounded values here so both sides start
from identical numbers.

Loss: softmax cross-entropy over the candidates of each node (rows
grp_off[g]..grp_off[g+1]-1), averaged over nodes; target = index within the
node of the strong-branching winner.
"""
from __future__ import annotations

import numpy as np

SIZES = [(64, 32), (64, 64), (64, 64), (1, 64)]
N_IN = 32
N_PARAMS = sum(o * i + o for o, i in SIZES)  # 10497


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == N_PARAMS
    out, p = [], 0
    for o, i in SIZES:
        W = w[p:p + o * i].reshape(o, i)
        p += o * i
        b = w[p:p + o]
        p += o
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as
    float32 (IEEE-754 binary32 with the low 16 mantissa bits cleared)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    out = np.where(nan, a, out)
    return out


def forward(w, feat):
    """Scores [rows] and the hidden activations after each ReLU."""
    h = np.asarray(feat, dtype=np.float64)
    acts = []
    layers = unpack(w)
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if li < len(layers) - 1:
            h = np.maximum(z, 0.0)
            acts.append(h)
        else:
            h = z
    return h[:, 0], acts


def backward(w, feat, dscore):
    """Gradient of sum(dscore * score) with respect to the flat parameters."""
    feat = np.asarray(feat, dtype=np.float64)
    layers = unpack(w)
    _, acts = forward(w, feat)
    ins = [feat] + acts
    g = np.asarray(dscore, dtype=np.float64)[:, None]
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        grads[li] = (g.T @ ins[li], g.sum(0))
        if li > 0:
            g = (g @ W) * (acts[li - 1] > 0.0)
    return pack(grads)


def loss_grad(score, grp_off, target):
    """Mean over nodes of the softmax cross-entropy; returns (loss, dscore)."""
    score = np.asarray(score, dtype=np.float64)
    d = np.zeros_like(score)
    G = len(grp_off) - 1
    loss = 0.0
    for g in range(G):
        a, b = int(grp_off[g]), int(grp_off[g + 1])
        s = score[a:b]
        m = s.max()
        e = np.exp(s - m)
        z = e.sum()
        loss += -(s[target[g]] - m - np.log(z))
        p = e / z
        p[target[g]] -= 1.0
        d[a:b] = p / G
    return loss / G, d


def adam(w32, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on the master weights; returns new arrays."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    w = w32 - lr * mh / (np.sqrt(vh) + eps)
    return w, m, v
