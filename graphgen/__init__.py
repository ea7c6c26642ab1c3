"""Seeded synthetic graph inputs shared by the CPU oracle and the GPU library.

This module produces graphs only; it contains no distance, farness or gain
arithmetic.  Every random draw comes from SplitMix64 in counter form
(``graphgen.c``), so a given (generator, seed) always yields the same CSR.

The method's basic input contract is a connected, undirected, unweighted graph
(paper, Section 2 "Preliminaries"): every generator here returns such a graph
as CSR int32 with rows sorted ascending, no self-loops and no duplicates.  The
large generators keep the largest connected component and relabel it in
ascending order of the old ids.

Workload families (sizes follow the synthetic stand-ins for the paper's
complex networks):
  * ``ba``      Barabasi-Albert, clique K_{m+1} seed, m distinct targets per node
  * ``rmat``    R-MAT (a,b,c,d)=(.57,.19,.19,.05), permuted ids, symmetrised, LCC
  * ``grid``    2D lattice with 5% of edges dropped and 0.1%*n random shortcuts, LCC
  * ``batch_ba``  256 BA graphs with n ~ U{1000..50000}, m ~ U{2..8}, k ~ U{5..50}
  * closed families: path, cycle, star, complete, complete bipartite
  * ``gnp_connected``  tiny random connected graphs for brute force
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C generator (gcc, OpenMP) next to this file."""
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
        lib.gg_ba.restype = ctypes.c_int64
        lib.gg_ba.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, i32p, i32p]
        lib.gg_rmat.restype = ctypes.c_int
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64, i32p, i32p]
        lib.gg_grid.restype = ctypes.c_int64
        lib.gg_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_uint64, i32p, i32p]
        lib.gg_build_csr.restype = ctypes.c_int
        lib.gg_build_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p, ctypes.c_int32,
                                     i64p, i32p, i32p, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64)]
        lib.gg_build_csr_directed.restype = ctypes.c_int
        lib.gg_build_csr_directed.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p, ctypes.c_int32,
                                              i64p, i32p, i32p, ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_int64)]
        lib.gg_edge_weights.restype = ctypes.c_int
        lib.gg_edge_weights.argtypes = [ctypes.c_int64, i32p, i32p, ctypes.c_int32, ctypes.c_uint64,
                                        ctypes.c_int32, np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")]
        lib.gg_splitmix_at.restype = ctypes.c_uint64
        lib.gg_splitmix_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        _lib = lib
    return _lib


@dataclass
class Graph:
    """CSR graph: row_ptr int32[n+1], col_idx int32[nnz] (undirected: both
    directions stored; directed: out-neighbour rows).  ``weight`` (uint8[nnz],
    every entry >= 1, the same in both rows of an undirected edge) makes it a
    weighted graph; None means every edge has length 1."""
    name: str
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    old_id: np.ndarray | None = None
    directed: bool = False
    weight: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.col_idx, dtype=np.int32).tobytes())
        if self.weight is not None:
            h.update(b"w")
            h.update(np.ascontiguousarray(self.weight, dtype=np.uint8).tobytes())
        return h.hexdigest()


def splitmix_at(key: int, i: int) -> int:
    return int(_load().gg_splitmix_at(ctypes.c_uint64(key & (2**64 - 1)), ctypes.c_uint64(i)))


def from_edges(name: str, nv: int, src, dst, keep_lcc: bool = True) -> Graph:
    """Symmetrise, dedupe, drop self-loops, optionally keep the LCC, relabel, sort rows."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    ne = int(src.shape[0])
    row_ptr = np.zeros(nv + 1, dtype=np.int64)
    col_idx = np.zeros(max(2 * ne, 1), dtype=np.int32)
    old_id = np.zeros(max(nv, 1), dtype=np.int32)
    out_n, out_nnz = ctypes.c_int64(), ctypes.c_int64()
    rc = lib.gg_build_csr(nv, ne, src, dst, 1 if keep_lcc else 0, row_ptr, col_idx, old_id,
                          ctypes.byref(out_n), ctypes.byref(out_nnz))
    if rc != 0:
        raise ValueError("edge list holds an id outside [0, nv)")
    n, nnz = out_n.value, out_nnz.value
    if nnz >= 2**31:
        raise ValueError("nnz does not fit int32")
    rp = row_ptr[: n + 1].astype(np.int32)
    ci = col_idx[:nnz].copy()
    return Graph(name, int(n), rp, ci, old_id[:n].copy())


def from_arcs(name: str, nv: int, src, dst, keep_scc: bool = True) -> Graph:
    """Directed graph: arcs src -> dst (rows are out-neighbours), self-loops and
    repeated arcs dropped, optionally the largest strongly connected component,
    relabelled in ascending old-id order, rows sorted."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    ne = int(src.shape[0])
    row_ptr = np.zeros(nv + 1, dtype=np.int64)
    col_idx = np.zeros(max(ne, 1), dtype=np.int32)
    old_id = np.zeros(max(nv, 1), dtype=np.int32)
    out_n, out_nnz = ctypes.c_int64(), ctypes.c_int64()
    rc = lib.gg_build_csr_directed(nv, ne, src, dst, 1 if keep_scc else 0, row_ptr, col_idx, old_id,
                                   ctypes.byref(out_n), ctypes.byref(out_nnz))
    if rc != 0:
        raise ValueError("arc list holds an id outside [0, nv)")
    n, nnz = out_n.value, out_nnz.value
    g = Graph(name, int(n), row_ptr[: n + 1].astype(np.int32), col_idx[:nnz].copy(), old_id[:n].copy())
    g.directed = True
    return g


# ---------------------------------------------------------------- generators

def ba(n: int, m: int, seed: int) -> Graph:
    """Barabasi-Albert: clique K_{m+1}, then m distinct degree-proportional targets per node."""
    lib = _load()
    ne = (m + 1) * m // 2 + m * (n - m - 1)
    src = np.zeros(ne, dtype=np.int32)
    dst = np.zeros(ne, dtype=np.int32)
    got = lib.gg_ba(n, m, seed, src, dst)
    if got != ne:
        raise ValueError("bad BA arguments")
    return from_edges("ba_n%d_m%d_s%d" % (n, m, seed), n, src, dst, keep_lcc=True)


def rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19) -> Graph:
    """R-MAT scale/edge factor, permuted ids, symmetrised, simple, largest component."""
    lib = _load()
    nv = 1 << scale
    m = edge_factor * nv
    src = np.zeros(m, dtype=np.int32)
    dst = np.zeros(m, dtype=np.int32)
    if lib.gg_rmat(scale, m, a, b, c, seed, src, dst) != 0:
        raise ValueError("bad R-MAT arguments")
    g = from_edges("rmat%d_ef%d_s%d" % (scale, edge_factor, seed), nv, src, dst, keep_lcc=True)
    del src, dst
    return g


def grid(rows: int, cols: int, seed: int, drop_frac: float = 0.05, shortcut_frac: float = 0.001) -> Graph:
    """Row-major lattice, round(drop_frac*E) edges dropped, round(shortcut_frac*n) shortcuts, LCC.

    The shortcut count is read as 0.1% of the node count (1,049 for 1024x1024).
    """
    lib = _load()
    nv = rows * cols
    nl = rows * (cols - 1) + (rows - 1) * cols
    drop = int(round(drop_frac * nl))
    short = int(round(shortcut_frac * nv))
    cap = nl + short
    src = np.zeros(max(cap, 1), dtype=np.int32)
    dst = np.zeros(max(cap, 1), dtype=np.int32)
    ne = lib.gg_grid(rows, cols, drop, short, seed, src, dst)
    if ne < 0:
        raise ValueError("bad grid arguments")
    return from_edges("grid%dx%d_s%d" % (rows, cols, seed), nv, src[:ne], dst[:ne], keep_lcc=True)


def batch_ba_params(master_seed: int = 3, count: int = 256):
    """(seed_g, n_g, m_g, k_g) for the batched workload: n~U{1000..50000}, m~U{2..8}, k~U{5..50}."""
    out = []
    for g in range(count):
        sg = splitmix_at(master_seed, g)
        n_g = 1000 + splitmix_at(sg, 0) % 49001
        m_g = 2 + splitmix_at(sg, 1) % 7
        k_g = 5 + splitmix_at(sg, 2) % 46
        out.append((splitmix_at(sg, 3), int(n_g), int(m_g), int(k_g)))
    return out


def batch_ba(master_seed: int = 3, count: int = 256):
    """List of (Graph, k) for the batched workload."""
    res = []
    for (sg, n_g, m_g, k_g) in batch_ba_params(master_seed, count):
        g = ba(n_g, m_g, sg)
        g.name = "batchba_%d" % len(res)
        res.append((g, k_g))
    return res


# ------------------------------------------------------- closed-form families

def _from_pairs(name, n, pairs, keep_lcc=False) -> Graph:
    if len(pairs) == 0:
        src = np.zeros(0, dtype=np.int32)
        dst = np.zeros(0, dtype=np.int32)
    else:
        arr = np.asarray(pairs, dtype=np.int32)
        src, dst = arr[:, 0].copy(), arr[:, 1].copy()
    return from_edges(name, n, src, dst, keep_lcc=keep_lcc)


def path(n: int) -> Graph:
    return _from_pairs("path%d" % n, n, [(i, i + 1) for i in range(n - 1)])


def cycle(n: int) -> Graph:
    return _from_pairs("cycle%d" % n, n, [(i, (i + 1) % n) for i in range(n)])


def star(n: int) -> Graph:
    """Centre 0, leaves 1..n-1."""
    return _from_pairs("star%d" % n, n, [(0, i) for i in range(1, n)])


def complete(n: int) -> Graph:
    return _from_pairs("K%d" % n, n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def complete_bipartite(a: int, b: int) -> Graph:
    """Side A = 0..a-1, side B = a..a+b-1."""
    return _from_pairs("K%d_%d" % (a, b), a + b, [(i, a + j) for i in range(a) for j in range(b)])


def gnp_connected(n: int, p: float, seed: int) -> Graph:
    """G(n,p) plus a random spanning tree (so it is connected); tiny n only."""
    pairs = set()
    draw = 0
    for v in range(1, n):
        u = splitmix_at(seed, draw) % v
        draw += 1
        pairs.add((u, v))
    thr = int(p * 2**64)
    for i in range(n):
        for j in range(i + 1, n):
            if splitmix_at(seed ^ 0x5DEECE66D, i * n + j) < thr:
                pairs.add((i, j))
    return _from_pairs("gnp%d_%g_s%d" % (n, p, seed), n, sorted(pairs))


# ------------------------------------------------------- directed graphs

def directed_cycle(n: int) -> Graph:
    """Arcs v -> v+1 (mod n)."""
    v = np.arange(n, dtype=np.int32)
    return from_arcs("dcycle%d" % n, n, v, (v + 1) % n)


def gnp_directed(n: int, p: float, seed: int) -> Graph:
    """A directed cycle through a seeded random permutation (so the graph is
    strongly connected) plus each other arc u -> v with probability p."""
    perm = sorted(range(n), key=lambda i: splitmix_at(seed, i))
    arcs = {(perm[i], perm[(i + 1) % n]) for i in range(n)} if n > 1 else set()
    thr = int(p * 2**64)
    for u in range(n):
        for v in range(n):
            if u != v and splitmix_at(seed ^ 0x2545F4914F6CDD1D, u * n + v) < thr:
                arcs.add((u, v))
    arcs = sorted(arcs)
    src = np.array([a for a, _ in arcs], dtype=np.int32)
    dst = np.array([b for _, b in arcs], dtype=np.int32)
    return from_arcs("gnpdir%d_%g_s%d" % (n, p, seed), n, src, dst, keep_scc=True)


def rmat_directed(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19) -> Graph:
    """R-MAT arcs (permuted ids, not symmetrised), largest strongly connected
    component."""
    lib = _load()
    nv = 1 << scale
    m = edge_factor * nv
    src = np.zeros(m, dtype=np.int32)
    dst = np.zeros(m, dtype=np.int32)
    if lib.gg_rmat(scale, m, a, b, c, seed, src, dst) != 0:
        raise ValueError("bad R-MAT arguments")
    return from_arcs("rmatdir%d_ef%d_s%d" % (scale, edge_factor, seed), nv, src, dst, keep_scc=True)


# -------------------------------------------------------- weighted graphs

def with_weights(g: Graph, wmax: int, seed: int) -> Graph:
    """The same graph with integer edge lengths drawn uniformly from
    [1, wmax] (seeded, keyed by the endpoint pair)."""
    w = np.zeros(g.nnz, dtype=np.uint8)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    if _load().gg_edge_weights(g.n, rp, ci, int(wmax), seed, 1 if g.directed else 0, w) != 0:
        raise ValueError("wmax must be in [1, 255]")
    return Graph("%s_w%d_s%d" % (g.name, wmax, seed), g.n, rp, ci, g.old_id, g.directed, w)


def with_weight_array(g: Graph, w) -> Graph:
    """The same graph with the given per-arc lengths (uint8[nnz])."""
    w = np.ascontiguousarray(w, dtype=np.uint8)
    if w.shape != (g.nnz,):
        raise ValueError("one weight per CSR entry")
    return Graph(g.name + "_w", g.n, g.row_ptr, g.col_idx, g.old_id, g.directed, w)


# --------------------------------------------------------- named workloads

def workload(name: str) -> Graph:
    """Graphs by workload name: ba2000, rmat16, rmat20, rmat24, grid1024, and
    grid256 (the grid recipe at 256 x 256)."""
    if name == "ba2000":
        return ba(2000, 4, 1)
    if name == "rmat16":
        return rmat(16, 16, 2)
    if name == "grid1024":
        return grid(1024, 1024, 4)
    if name == "grid256":
        return grid(256, 256, 7)
    if name == "rmat20":
        return rmat(20, 16, 5)
    if name == "rmat24":
        return rmat(24, 16, 6)
    raise KeyError(name)
