"""Float64 reference of the candidate-ordering MLP -- TEST INFRASTRUCTURE ONLY.

Not part of the paper's method (the paper has no learning); this is the
oracle for the learned candidate order that only changes which exact gain
evaluations happen first.  numpy only, shares no code with the GPU library.

Network: 8 features -> 64 -> 64 -> 1, ReLU.  Master parameters are a float32
vector of 4801 entries: W1 (64x8, row j = hidden unit j), b1 (64), W2 (64x64),
b2 (64), W3 (64), b3.  Rounding points (the GPU kernels use the same ones):
  x = bf16(feature); h1 = bf16(relu(W1 x + b1)); h2 = bf16(relu(W2 h1 + b2));
  out = W3 h2 + b3; weights enter as bf16, biases as float32.
Here the arithmetic between rounding points is float64; ``rounding=False``
turns every bf16 rounding into the identity (used for finite differences).

Loss: mean squared error against y = log2(1 + gain).  Optimiser: Adam
(Kingma and Ba, "Adam: A Method for Stochastic Optimization", ICLR 2015).
"""
from __future__ import annotations

import numpy as np

IN, H = 8, 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + H * IN
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
NPARAM = OFF_B3 + 1


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via float32; returns float64."""
    a = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    u = np.where(finite, r, u).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[OFF_W1:OFF_B1].reshape(H, IN), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(H, H),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, W3, [b3]])


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation, float32 (the caller passes these to the GPU)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2.0 / IN), (H, IN))
    W2 = rng.normal(0, np.sqrt(2.0 / H), (H, H))
    W3 = rng.normal(0, np.sqrt(1.0 / H), H)
    return pack(W1, np.zeros(H), W2, np.zeros(H), W3, 0.0).astype(np.float32)


def forward(p, X, rounding=True, h1_in=None, h2_in=None):
    """Returns (x, h1, h2, out).  h1_in / h2_in replace the computed
    activations of that layer (to compare one layer at a time)."""
    r = bf16 if rounding else (lambda z: np.asarray(z, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p)
    if rounding:  # biases are float32 on the device
        b1 = np.asarray(b1, np.float32).astype(np.float64)
        b2 = np.asarray(b2, np.float32).astype(np.float64)
        b3 = np.float64(np.float32(b3))
    x = r(X)
    h1 = r(np.maximum(x @ r(W1).T + b1, 0.0)) if h1_in is None else np.asarray(h1_in, np.float64)
    h2 = r(np.maximum(h1 @ r(W2).T + b2, 0.0)) if h2_in is None else np.asarray(h2_in, np.float64)
    out = h2 @ r(W3) + b3
    return x, h1, h2, out


def loss(p, X, y, rounding=True) -> float:
    out = forward(p, X, rounding)[3]
    return float(np.mean((out - np.asarray(y, np.float64)) ** 2))


def backward(p, x, h1, h2, out, y, rounding=True) -> np.ndarray:
    """Gradient of the mean squared error w.r.t. the master vector, given the
    forward activations.  ReLU derivative: 1 where the activation is > 0."""
    r = bf16 if rounding else (lambda z: np.asarray(z, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p)
    N = x.shape[0]
    dout = 2.0 * (np.asarray(out, np.float64) - np.asarray(y, np.float64)) / N
    gW3 = dout @ h2
    gb3 = dout.sum()
    dh2 = np.outer(dout, r(W3)) * (h2 > 0)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ r(W2)) * (h1 > 0)
    gW1 = dh1.T @ x
    gb1 = dh1.sum(axis=0)
    return pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam(w, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns (w, m, v) as float64."""
    w, m, v, g = (np.asarray(a, np.float64) for a in (w, m, v, g))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def features(rp, ci, dist, ub, last_eval, dist_at_eval, round_, k, ecc1, cand=None) -> np.ndarray:
    """The 8 features of the learned order, from their definitions (float32)."""
    rp = np.asarray(rp, np.int64)
    n = rp.shape[0] - 1
    cand = np.arange(n) if cand is None else np.asarray(cand, np.int64)
    deg = np.diff(rp).astype(np.float64)
    two = np.array([deg[ci[rp[v]:rp[v + 1]]].sum() for v in range(n)], dtype=np.float64)
    d = np.asarray(dist, np.float64)
    ubv = np.maximum(np.asarray(ub, np.float64), 0.0)
    le = np.asarray(last_eval, np.int64)
    since = np.where(le >= 0, round_ - le, round_).astype(np.float64)
    dat = np.where(le >= 0, np.asarray(dist_at_eval, np.float64), d)
    F = np.stack([np.log2(1 + deg), d / max(ecc1, 1), np.log2(1 + ubv), np.log2(1 + two),
                  np.log2(1 + since), dat - d, np.full(n, round_ / max(k, 1)), np.log2(1 + d)],
                 axis=1)
    return F[cand].astype(np.float32)
