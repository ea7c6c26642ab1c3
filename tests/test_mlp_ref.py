"""Pins of the float64 MLP reference (oracle/mlp_ref.py), CPU only.

* bf16 rounding against hand-computed round-to-nearest-even cases;
* backward formulas against central finite differences with rounding off;
* Adam's first step against its closed form w - lr * g / (|g| + eps);
* feature definitions on a graph small enough to work out by hand.
"""
import numpy as np
import pytest

import graphgen
from oracle import mlp_ref as M


def test_bf16_rounding_cases():
    one = 1.0
    ulp = 2.0 ** -7  # bf16 keeps 7 fraction bits
    cases = {
        one: one,
        one + ulp: one + ulp,
        one + ulp / 2: one,                  # tie -> even (1.0)
        one + 3 * ulp / 2: one + 2 * ulp,    # tie -> even (1 + 2 ulp)
        one + ulp / 2 + 2.0 ** -20: one + ulp,  # above the tie
        -3.0: -3.0,
        0.0: 0.0,
        65504.0: 65536.0,                    # 0x477FE000 rounds up to 0x47800000
    }
    for x, want in cases.items():
        assert float(M.bf16(x)) == want, x
    assert np.isinf(M.bf16(np.inf))


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = M.init_params(1).astype(np.float64)
    p[M.OFF_B1:M.OFF_W2] = rng.normal(0, 0.1, M.H)
    p[M.OFF_B2:M.OFF_W3] = rng.normal(0, 0.1, M.H)
    X = rng.normal(0, 1, (16, M.IN))
    y = rng.normal(0, 1, 16)
    x, h1, h2, out = M.forward(p, X, rounding=False)
    g = M.backward(p, x, h1, h2, out, y, rounding=False)
    idx = np.concatenate([rng.choice(M.NPARAM, 300, replace=False),
                          np.arange(M.OFF_B1, M.OFF_W2), [M.OFF_B3]])
    eps = 1e-6
    for q in idx:
        pp, pm = p.copy(), p.copy()
        pp[q] += eps
        pm[q] -= eps
        fd = (M.loss(pp, X, y, rounding=False) - M.loss(pm, X, y, rounding=False)) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(g[q])), (q, fd, g[q])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    w = rng.normal(0, 1, 50)
    g = rng.normal(0, 1, 50)
    lr, eps = 1e-3, 1e-8
    w1, m1, v1 = M.adam(w, np.zeros(50), np.zeros(50), g, 1, lr=lr, eps=eps)
    assert np.allclose(w1, w - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    # a constant gradient keeps the step at lr * sign(g) for every step count
    w2, m2, v2 = M.adam(w1, m1, v1, g, 2, lr=lr, eps=0.0)
    assert np.allclose(w2, w1 - lr * np.sign(g), atol=1e-12)


def test_forward_rounding_points_idempotent():
    rng = np.random.default_rng(3)
    p = M.init_params(4)
    X = rng.normal(0, 1, (32, M.IN)).astype(np.float32)
    x, h1, h2, out = M.forward(p, X)
    # every rounded activation is already a bf16 value
    for a in (x, h1, h2):
        assert np.array_equal(M.bf16(a), a)
    assert np.all(h1 >= 0) and np.all(h2 >= 0)


def test_features_by_hand():
    g = graphgen.path(5)  # 0-1-2-3-4
    dist = np.array([2, 1, 0, 1, 2])  # S = {2}
    ub = np.array([4, 3, 0, 3, 4])
    le = np.array([1, 1, -1, 0, -1])
    dat = np.array([3, 2, 0, 1, 0])
    F = M.features(g.row_ptr, g.col_idx, dist, ub, le, dat, round_=3, k=6, ecc1=2)
    # node 0: deg 1, neighbour degree sum 2
    assert np.allclose(F[0], [1.0, 1.0, np.log2(5), np.log2(3), np.log2(3), 1.0, 0.5, np.log2(3)])
    # node 4: never evaluated -> rounds since = round, drop = 0
    assert np.allclose(F[4], [1.0, 1.0, np.log2(5), np.log2(3), 2.0, 0.0, 0.5, np.log2(3)])
    # node 1: deg 2, neighbour degree sum 1 + 2
    assert np.allclose(F[1][:4], [np.log2(3), 0.5, 2.0, 2.0])
