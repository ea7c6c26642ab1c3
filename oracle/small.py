"""Tier C of the oracle: exhaustive and matrix forms for tiny graphs.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  numpy only; no BFS code is
shared with oracle.c, so these routines pin it from outside:

  * all-pairs distances by Floyd-Warshall (a different algorithm from BFS);
  * F(S) and brute-force optimum over all k-subsets (the quantity the ILP of
    Section 5 optimises);
  * the greedy of Chen et al. in its matrix form (Section 3.2, Algorithm
    "greedy"), with the matrix update read as M[u,w] <- min(M[u,w], d[s,w]);
  * the marginal gain through the bit-vector identity of the theorem in
    Section 4.3, with the bit vectors built by the OR recurrence over
    neighbours (the recurrence also keeps the node's own previous vector).
"""
from __future__ import annotations

import itertools

import numpy as np

INF = np.iinfo(np.int64).max // 4


def adjacency(g) -> np.ndarray:
    n = g.n
    A = np.zeros((n, n), dtype=bool)
    for u in range(n):
        A[u, g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]] = True
    return A


def floyd_warshall(g) -> np.ndarray:
    """All-pairs shortest-path lengths (int64, INF if unreachable); edge
    lengths from ``g.weight`` when the graph has them, else 1."""
    n = g.n
    D = np.full((n, n), INF, dtype=np.int64)
    w = getattr(g, "weight", None)
    for u in range(n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            D[u, int(g.col_idx[e])] = 1 if w is None else int(w[e])
    np.fill_diagonal(D, 0)
    for m in range(n):
        D = np.minimum(D, D[:, m:m + 1] + D[m:m + 1, :])
    return D


def farness(D: np.ndarray, S) -> int:
    """F(S) = sum_w min_{s in S} d(s, w)  (Section 2)."""
    S = list(S)
    return int(D[S].min(axis=0).sum())


def closeness_group(D: np.ndarray, S) -> float:
    """c(S) = n / sum_{v notin S} d(S, v) (Section 2, normalisation of the paper)."""
    n = D.shape[0]
    return n / farness(D, S)


def brute_force_opt(D: np.ndarray, k: int):
    """min over all k-subsets of F(S): (F*, lexicographically smallest argmin)."""
    n = D.shape[0]
    best, arg = None, None
    for S in itertools.combinations(range(n), k):
        f = farness(D, S)
        if best is None or f < best:
            best, arg = f, S
    return best, arg


def greedy_matrix(D: np.ndarray, k: int):
    """Greedy of Chen et al. in matrix form (Section 3.2, Algorithm "greedy").

    M[u, w] holds d(S u {u}, w).  Score[u] is the farness sum_w M[u, w]; the
    pick minimises it, ties to the smallest id.  After a pick s,
    M[u, w] <- min(M[u, w], d[s, w]) for all u.
    """
    n = D.shape[0]
    M = D.copy()
    S = []
    Fs = []
    for _ in range(k):
        score = M.sum(axis=1)
        score[S] = INF
        s = int(np.argmin(score))  # argmin returns the first (smallest id) minimum
        S.append(s)
        Fs.append(int(score[s]))
        M = np.minimum(M, D[s][None, :])
    return S, Fs


def gain_def(D: np.ndarray, S, v: int) -> int:
    """g(v,S) = F(S) - F(S u {v})."""
    return farness(D, S) - farness(D, list(S) + [v])


def bit_vectors(g, levels: int) -> list:
    """b^i_u for i = 0..levels as a list of (n x n) bool matrices.

    b^0_u = {u}; b^i_u = b^{i-1}_u OR (OR over neighbours v of b^{i-1}_v).
    Bit j of b^i_u is set iff d(u, j) <= i.
    """
    A = adjacency(g)
    n = g.n
    b = np.eye(n, dtype=bool)
    out = [b]
    for _ in range(levels):
        nb = b.copy()
        for u in range(n):
            nb[u] |= b[A[u]].any(axis=0)
        b = nb
        out.append(b)
    return out


def theorem_gain(bits: list, S, u: int) -> int:
    """sum_{i=0}^{maxD(u)} |b^i_u AND NOT b^i_S| (theorem of Section 4.3)."""
    total = 0
    for b in bits:  # terms beyond maxD(u) are zero, so summing every level is the same sum
        bS = b[list(S)].any(axis=0)
        total += int((b[u] & ~bS).sum())
    return total
