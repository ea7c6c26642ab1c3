"""Learned candidate order: training data from the method's own exact
evaluations, GPU training with the library's MLP kernels.

The network predicts log2(1 + gain) of a candidate from 8 features of the
lazy loop's state at the start of a round; GC_ORDER_LEARNED evaluates
candidates in descending min(2^prediction - 1, stale gain).  Exact pruned BFS
decides every pick, so the group never depends on the network.
"""
from __future__ import annotations

import numpy as np

from . import gc


def collect(runs, block: int = 64, order: str = "plain"):
    """Run the greedy with evaluation logging on each (Graph, k) and return
    (features float32 [N x 8], targets log2(1 + gain) float32 [N])."""
    feats, ys = [], []
    for G, k in runs:
        cap = 64 * k * max(block, 64) + 4 * G.n
        _, _, st = G.greedy_group(k, order=order, block=block, log_capacity=cap)
        log = st["log"]
        feats.append(log["feat"])
        ys.append(np.log2(1.0 + log["gain"].astype(np.float64)).astype(np.float32))
    return np.concatenate(feats), np.concatenate(ys)


def init_master(seed: int) -> np.ndarray:
    """He-style initial weights (float32), drawn on the host with a seed."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2.0 / gc.MLP_IN), (gc.MLP_HIDDEN, gc.MLP_IN))
    W2 = rng.normal(0, np.sqrt(2.0 / gc.MLP_HIDDEN), (gc.MLP_HIDDEN, gc.MLP_HIDDEN))
    W3 = rng.normal(0, np.sqrt(1.0 / gc.MLP_HIDDEN), gc.MLP_HIDDEN)
    p = np.concatenate([W1.ravel(), np.zeros(gc.MLP_HIDDEN), W2.ravel(), np.zeros(gc.MLP_HIDDEN),
                        W3, [0.0]])
    return p.astype(np.float32)


def train(X, Y, steps: int = 1500, batch: int = 1024, lr: float = 3e-3, seed: int = 7):
    """Train a fresh network on (X, Y) on the GPU; returns (Mlp, loss trace)."""
    net = gc.Mlp(init_master(seed))
    losses = net.train(X, Y, steps=steps, batch=batch, lr=lr, seed=seed)
    return net, losses
