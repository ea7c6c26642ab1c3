"""CPU oracle for group-closeness maximisation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library: the C part
(``oracle.c``) is compiled by gcc on its own, and the pure-Python part
(``small.py``, ``mlp_ref.py``) uses numpy only.

Contents
  * ``oracle.c`` / this module: tier A plain greedy (full BFS per candidate),
    tier B CPU Greedy++ (pruned BFS, lazy skip, BFScut), single gains,
    group distances and farness, top-k closeness by definition.
  * ``small.py``: tier C -- Floyd-Warshall, brute force over k-subsets, the
    matrix form of the greedy of Chen et al., the bit-vector identity of the
    paper's theorem, all for tiny graphs.
  * ``mlp_ref.py``: float64 reference of the candidate-ordering MLP with the
    same bfloat16 rounding points as the GPU kernels.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OR_OK = 0
OR_EINVAL = -1
OR_ENOTSYM = -2
OR_EDISCONNECTED = -3
OR_EINVARIANT = -100


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        I64, I32 = ctypes.c_int64, ctypes.c_int32
        lib.or_bfs.restype = I64
        lib.or_bfs.argtypes = [I64, i32p, i32p, I32, i32p, i32p]
        lib.or_group_dist.restype = ctypes.c_int
        lib.or_group_dist.argtypes = [I64, i32p, i32p, i32p, I32, i32p]
        lib.or_farness.restype = I64
        lib.or_farness.argtypes = [I64, i32p, i32p, i32p, I32]
        lib.or_farness_all.restype = ctypes.c_int
        lib.or_farness_all.argtypes = [I64, i32p, i32p, i64p]
        lib.or_gain.restype = I64
        lib.or_gain.argtypes = [I64, i32p, i32p, i32p, I32]
        lib.or_gains.restype = ctypes.c_int
        lib.or_gains.argtypes = [I64, i32p, i32p, i32p, i32p, I64, i64p]
        lib.or_greedy.restype = ctypes.c_int
        lib.or_greedy.argtypes = [I64, i32p, i32p, I32, i32p, i64p, ctypes.c_void_p, I32]
        lib.or_greedypp.restype = ctypes.c_int
        lib.or_greedypp.argtypes = [I64, i32p, i32p, I32, I32, I32, i32p, i64p, i64p, i64p, I32, I32,
                                    i64p, I32]
        lib.or_pruned_stats.restype = ctypes.c_int
        lib.or_pruned_stats.argtypes = [I64, i32p, i32p, i32p, i32p, I64, i64p, i64p, i64p]
        lib.or_gains_cut.restype = ctypes.c_int
        lib.or_gains_cut.argtypes = [I64, i32p, i32p, i32p, i32p, I64, I64, I32, i64p, i32p]
        lib.or_validate_graph.restype = ctypes.c_int
        lib.or_validate_graph.argtypes = [I64, i32p, i32p, I32]
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        lib.or_sssp_w.restype = I64
        lib.or_sssp_w.argtypes = [I64, i32p, i32p, u8p, I32, i32p]
        lib.or_validate_w.restype = ctypes.c_int
        lib.or_validate_w.argtypes = [I64, i32p, i32p, u8p, I32]
        lib.or_group_dist_w.restype = ctypes.c_int
        lib.or_group_dist_w.argtypes = [I64, i32p, i32p, u8p, i32p, I32, i32p]
        lib.or_farness_all_w.restype = ctypes.c_int
        lib.or_farness_all_w.argtypes = [I64, i32p, i32p, u8p, i64p]
        lib.or_gains_w.restype = ctypes.c_int
        lib.or_gains_w.argtypes = [I64, i32p, i32p, u8p, i32p, i32p, I64, i64p]
        lib.or_pruned_stats_w.restype = ctypes.c_int
        lib.or_pruned_stats_w.argtypes = [I64, i32p, i32p, u8p, i32p, i32p, I64, i64p, i64p, i64p]
        lib.or_greedy_w.restype = ctypes.c_int
        lib.or_greedy_w.argtypes = [I64, i32p, i32p, u8p, I32, i32p, i64p, I32]
        lib.or_greedypp_w.restype = ctypes.c_int
        lib.or_greedypp_w.argtypes = [I64, i32p, i32p, u8p, I32, I32, I32, i32p, i64p, i64p, i64p, I32]
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_num_threads.argtypes = []
        _lib = lib
    return _lib


def _csr(g):
    return (int(g.n), np.ascontiguousarray(g.row_ptr, dtype=np.int32),
            np.ascontiguousarray(g.col_idx, dtype=np.int32))


def _directed(g) -> int:
    """1 for a directed graph (rows are out-neighbour lists; graphgen marks
    such graphs), else 0."""
    return 1 if getattr(g, "directed", False) else 0


def _weights(g):
    """uint8[nnz] edge lengths of a weighted graph, or None (unweighted)."""
    w = getattr(g, "weight", None)
    if w is None:
        return None
    w = np.ascontiguousarray(w, dtype=np.uint8)
    if w.shape != (int(g.col_idx.shape[0]),):
        raise OracleError("invalid argument: one weight per CSR entry")
    return w


def _check(rc):
    if rc == OR_EDISCONNECTED:
        raise OracleError("graph is disconnected")
    if rc == OR_ENOTSYM:
        raise OracleError("adjacency is not symmetric")
    if rc == OR_EINVAL:
        raise OracleError("invalid argument or malformed CSR (range, order, self-loop, duplicate)")
    if rc == OR_EINVARIANT:
        raise OracleError("greedy invariant violated")
    if rc != OR_OK:
        raise OracleError("oracle error %d" % rc)


def num_threads() -> int:
    return int(_load().or_num_threads())


def validate(g) -> None:
    """The input contract of Section 2 (connected, undirected, simple; or, for
    a graph marked directed, strongly connected): raises OracleError for a bad
    row_ptr, an id out of range, an unsorted or duplicate entry, a self-loop,
    a missing reverse edge (undirected) or a node that cannot be reached."""
    n, rp, ci = _csr(g)
    if rp.shape[0] != n + 1 or int(rp[n]) != ci.shape[0]:
        raise OracleError("invalid argument or malformed CSR (row_ptr length or nnz)")
    w = _weights(g)
    if w is None:
        _check(_load().or_validate_graph(n, rp, ci, _directed(g)))
    else:
        _check(_load().or_validate_w(n, rp, ci, w, _directed(g)))


def sssp(g, src: int) -> np.ndarray:
    """d(src, w) for all w (-1 if unreachable): Dijkstra on a weighted graph,
    BFS otherwise."""
    w = _weights(g)
    if w is None:
        return bfs(g, src)
    n, rp, ci = _csr(g)
    d = np.empty(n, dtype=np.int32)
    _load().or_sssp_w(n, rp, ci, w, int(src), d)
    return d


def bfs(g, src: int) -> np.ndarray:
    """d(src, w) for all w (-1 if unreachable)."""
    if _weights(g) is not None:
        raise OracleError("bfs() ignores weights; use sssp()")
    n, rp, ci = _csr(g)
    d = np.empty(n, dtype=np.int32)
    q = np.empty(n, dtype=np.int32)
    _load().or_bfs(n, rp, ci, int(src), d, q)
    return d


def group_dist(g, S) -> np.ndarray:
    """d(w, S) = min_{s in S} d(w, s)."""
    n, rp, ci = _csr(g)
    S = np.ascontiguousarray(S, dtype=np.int32)
    dS = np.empty(n, dtype=np.int32)
    w = _weights(g)
    if w is None:
        _check(_load().or_group_dist(n, rp, ci, S, int(S.shape[0]), dS))
    else:
        _check(_load().or_group_dist_w(n, rp, ci, w, S, int(S.shape[0]), dS))
    return dS


def farness(g, S) -> int:
    """Integer group farness F(S) = sum_w d(S, w)."""
    if _weights(g) is not None:
        return int(group_dist(g, S).astype(np.int64).sum())
    n, rp, ci = _csr(g)
    S = np.ascontiguousarray(S, dtype=np.int32)
    F = int(_load().or_farness(n, rp, ci, S, int(S.shape[0])))
    if F < 0:
        raise OracleError("bad group or disconnected graph")
    return F


def farness_all(g) -> np.ndarray:
    """F({v}) for every node v."""
    n, rp, ci = _csr(g)
    F = np.empty(n, dtype=np.int64)
    w = _weights(g)
    if w is None:
        _check(_load().or_farness_all(n, rp, ci, F))
    else:
        _check(_load().or_farness_all_w(n, rp, ci, w, F))
    return F


def topk_closeness(g, k: int):
    """Top-k closeness (the TopKCloseness search of Section 3.1 for general k):
    the k nodes of least F({v}), in increasing (F({v}), v) order -- ties go to
    the smaller id.  Written as its definition: every F({v}) by full BFS, then
    a sort.  Returns (nodes int32[k], F int64[k])."""
    n = int(g.n)
    if k < 1 or k > n:
        raise OracleError("k out of range")
    F = farness_all(g)
    order = np.lexsort((np.arange(n), F))[:k]
    return order.astype(np.int32), F[order].astype(np.int64)


def gain(g, dS, v: int) -> int:
    """g(v,S) = F(S) - F(S u {v}) by a full BFS (Dijkstra if weighted) from v."""
    if _weights(g) is not None:
        return int(gains(g, dS, [v])[0])
    n, rp, ci = _csr(g)
    return int(_load().or_gain(n, rp, ci, np.ascontiguousarray(dS, dtype=np.int32), int(v)))


def gains(g, dS, cand) -> np.ndarray:
    n, rp, ci = _csr(g)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    out = np.empty(cand.shape[0], dtype=np.int64)
    w = _weights(g)
    if w is None:
        _check(_load().or_gains(n, rp, ci, np.ascontiguousarray(dS, dtype=np.int32), cand,
                                int(cand.shape[0]), out))
    else:
        _check(_load().or_gains_w(n, rp, ci, w, np.ascontiguousarray(dS, dtype=np.int32), cand,
                                  int(cand.shape[0]), out))
    return out


def greedy(g, k: int, with_gains: bool = False):
    """Tier A plain greedy.  Returns (group, F) or (group, F, gains[(k-1), n]).
    The CSR is checked first (validate); a violation raises OracleError."""
    n, rp, ci = _csr(g)
    if rp.shape[0] != n + 1 or int(rp[n]) != ci.shape[0]:
        raise OracleError("invalid argument or malformed CSR (row_ptr length or nnz)")
    group = np.empty(k, dtype=np.int32)
    F = np.empty(k, dtype=np.int64)
    w = _weights(g)
    if w is not None:
        if with_gains:
            raise OracleError("with_gains is for unweighted graphs")
        _check(_load().or_greedy_w(n, rp, ci, w, int(k), group, F, _directed(g)))
        return group, F
    G = np.empty((max(k - 1, 1), n), dtype=np.int64) if with_gains else None
    ptr = G.ctypes.data_as(ctypes.c_void_p) if with_gains else None
    _check(_load().or_greedy(n, rp, ci, int(k), group, F, ptr, _directed(g)))
    if with_gains:
        return group, F, G[: k - 1]
    return group, F


def greedypp(g, k: int, block: int = 64, growth: int = 1):
    """Tier B CPU Greedy++.  Returns (group, F, evals per round, edges per round).
    Candidates are evaluated in batches of `block` between threshold updates;
    from the second round on each further batch of a round is `growth` times
    the one before (up to 16 x block).  The batches only change the counts.
    The CSR is checked first, as for greedy()."""
    n, rp, ci = _csr(g)
    if rp.shape[0] != n + 1 or int(rp[n]) != ci.shape[0]:
        raise OracleError("invalid argument or malformed CSR (row_ptr length or nnz)")
    group = np.empty(k, dtype=np.int32)
    F = np.empty(k, dtype=np.int64)
    ev = np.zeros(k, dtype=np.int64)
    ed = np.zeros(k, dtype=np.int64)
    w = _weights(g)
    if w is not None:
        _check(_load().or_greedypp_w(n, rp, ci, w, int(k), int(block), int(growth), group, F, ev, ed,
                                     _directed(g)))
        return group, F, ev, ed
    cuts = np.zeros(k, dtype=np.int64)
    _check(_load().or_greedypp(n, rp, ci, int(k), int(block), int(growth), group, F, ev, ed, 0, 0, cuts,
                               _directed(g)))
    return group, F, ev, ed


def greedypp_cut(g, k: int, block: int = 64, growth: int = 1, mode: int = 1, seed: int = 1024):
    """Tier B with the early exit inside each candidate's pruned BFS (the
    BFScut-style bound g <= g_l + e_l + T[l+1], see oracle.c): mode 1 in the
    first round (after the `seed` candidates of largest degree, evaluated
    exactly), mode 2 in every round.  Returns (group, F, evals per round,
    edges per round, cut candidates per round)."""
    if _weights(g) is not None:
        raise OracleError("the early exit is for unweighted graphs")
    n, rp, ci = _csr(g)
    if rp.shape[0] != n + 1 or int(rp[n]) != ci.shape[0]:
        raise OracleError("invalid argument or malformed CSR (row_ptr length or nnz)")
    group = np.empty(k, dtype=np.int32)
    F = np.empty(k, dtype=np.int64)
    ev = np.zeros(k, dtype=np.int64)
    ed = np.zeros(k, dtype=np.int64)
    cuts = np.zeros(k, dtype=np.int64)
    _check(_load().or_greedypp(n, rp, ci, int(k), int(block), int(growth), group, F, ev, ed, int(mode),
                               int(seed), cuts, _directed(g)))
    return group, F, ev, ed, cuts


def gains_cut(g, dS, cand, thr: int, thr_id: int):
    """The early-exit pruned BFS of tier B against one threshold: (value,
    cut) per candidate -- the exact gain (cut 0) or the bound it stopped at
    (cut 1)."""
    if _weights(g) is not None:
        raise OracleError("the early exit is for unweighted graphs")
    n, rp, ci = _csr(g)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    out = np.empty(cand.shape[0], dtype=np.int64)
    cut = np.empty(cand.shape[0], dtype=np.int32)
    _check(_load().or_gains_cut(n, rp, ci, np.ascontiguousarray(dS, dtype=np.int32), cand,
                                int(cand.shape[0]), int(thr), int(thr_id), out, cut))
    return out, cut


def pruned_stats(g, dS, cand):
    """Per-candidate (gain, |V(v)|, sum_{w in V(v)} deg w) by pruned BFS."""
    n, rp, ci = _csr(g)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    c = int(cand.shape[0])
    gg = np.empty(c, dtype=np.int64)
    vv = np.empty(c, dtype=np.int64)
    ee = np.empty(c, dtype=np.int64)
    w = _weights(g)
    if w is None:
        _check(_load().or_pruned_stats(n, rp, ci, np.ascontiguousarray(dS, dtype=np.int32), cand, c,
                                       gg, vv, ee))
    else:
        _check(_load().or_pruned_stats_w(n, rp, ci, w, np.ascontiguousarray(dS, dtype=np.int32), cand,
                                         c, gg, vv, ee))
    return gg, vv, ee
