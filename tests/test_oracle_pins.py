"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here uses the GPU library.  Each test pins a part of the oracle to
something other than the oracle itself:
  * the printed K5 example of Section 3.2 (tests/golden/k5_example.json);
  * closed forms of F({v}) and of greedy sequences on paths, cycles, stars,
    complete and complete bipartite graphs, from the definitions of Section 2;
  * Floyd-Warshall distances, brute force over all k-subsets and the matrix
    form of the greedy of Chen et al. (Section 3.2) on tiny graphs;
  * the bit-vector identity of the theorem of Section 4.3;
  * the supermodularity lemma of Section 3.2, exhaustively on tiny graphs;
  * tier B (pruned, lazy Greedy++) against tier A (plain greedy).
"""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import graphgen
import oracle
from oracle import small

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------ printed values

def test_k5_printed_example():
    with open(os.path.join(HERE, "golden", "k5_example.json")) as f:
        gold = json.load(f)
    g = graphgen.complete(5)
    n = g.n
    vals = {}
    for row in gold["closeness"]:
        S = row["S"]
        F = oracle.farness(g, S)
        c = Fraction(n, F)  # c(S) = n / sum_{v notin S} d(S,v); members contribute 0
        assert c == Fraction(row["c_num"], row["c_den"]), S
        vals[tuple(S)] = c
    d1 = vals[(0, 1, 3)] - vals[(0, 1)]
    d2 = vals[(0, 1, 2, 3)] - vals[(0, 1, 2)]
    assert d1 == Fraction(*gold["differences"]["c(S+v)-c(S)"])
    assert d2 == Fraction(*gold["differences"]["c(T+v)-c(T)"])
    assert d1 < d2  # closeness is not submodular
    # farness is supermodular on the same sets (Section 3.2 lemma)
    fS = oracle.farness(g, [0, 1, 3]) - oracle.farness(g, [0, 1])
    fT = oracle.farness(g, [0, 1, 2, 3]) - oracle.farness(g, [0, 1, 2])
    assert fS <= fT


# --------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 10, 31])
def test_path_single_farness(n):
    g = graphgen.path(n)
    F = oracle.farness_all(g)
    exp = np.array([v * (v + 1) // 2 + (n - 1 - v) * (n - v) // 2 for v in range(n)])
    assert np.array_equal(F, exp)
    grp, Fs = oracle.greedy(g, 1)
    assert int(grp[0]) == (n - 1) // 2
    assert int(Fs[0]) == n * n // 4


@pytest.mark.parametrize("n", [3, 4, 5, 8, 11])
def test_cycle_single_farness(n):
    g = graphgen.cycle(n)
    F = oracle.farness_all(g)
    assert np.all(F == n * n // 4)
    grp, _ = oracle.greedy(g, 1)
    assert int(grp[0]) == 0


@pytest.mark.parametrize("n", [3, 5, 9])
def test_star(n):
    g = graphgen.star(n)
    F = oracle.farness_all(g)
    assert int(F[0]) == n - 1
    assert np.all(F[1:] == 2 * n - 3)
    for k in range(1, n + 1):
        grp, Fs = oracle.greedy(g, k)
        assert grp.tolist() == list(range(k))
        assert Fs.tolist() == [n - i for i in range(1, k + 1)]


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_complete(n):
    g = graphgen.complete(n)
    for k in range(1, n + 1):
        grp, Fs = oracle.greedy(g, k)
        assert grp.tolist() == list(range(k))
        assert Fs.tolist() == [n - i for i in range(1, k + 1)]


@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (3, 5), (4, 4)])
def test_complete_bipartite(a, b):
    g = graphgen.complete_bipartite(a, b)
    F = oracle.farness_all(g)
    assert np.all(F[:a] == b + 2 * (a - 1))
    assert np.all(F[a:] == a + 2 * (b - 1))


# top-k closeness: rankings the closed forms above fix

@pytest.mark.parametrize("n", [1, 2, 5, 8, 31])
def test_topk_closeness_path(n):
    g = graphgen.path(n)
    # |v - (n-1)/2| orders the path's farness; ties (even n) to the smaller id
    exp = sorted(range(n), key=lambda v: (abs(2 * v - (n - 1)), v))
    for k in sorted({1, min(2, n), max(n // 2, 1), n}):
        nodes, F = oracle.topk_closeness(g, k)
        assert nodes.tolist() == exp[:k]
        assert F.tolist() == [v * (v + 1) // 2 + (n - 1 - v) * (n - v) // 2 for v in exp[:k]]


@pytest.mark.parametrize("n", [3, 6, 9])
def test_topk_closeness_star_and_cycle(n):
    nodes, F = oracle.topk_closeness(graphgen.star(n), n)
    assert nodes.tolist() == list(range(n))
    assert F.tolist() == [n - 1] + [2 * n - 3] * (n - 1)
    nodes, F = oracle.topk_closeness(graphgen.cycle(n), 3)
    assert nodes.tolist() == [0, 1, 2] and F.tolist() == [n * n // 4] * 3


@pytest.mark.parametrize("a,b", [(2, 3), (3, 5), (4, 4)])
def test_topk_closeness_complete_bipartite(a, b):
    # the smaller side is closer (b + 2(a-1) < a + 2(b-1) when a < b)
    nodes, _ = oracle.topk_closeness(graphgen.complete_bipartite(a, b), a + 1)
    exp = list(range(a)) + [a] if a < b else list(range(a + 1))
    assert nodes.tolist() == exp


def _h(L):
    """Farness of L path nodes strictly between two group members."""
    return (L + 1) * (L + 1) // 4


def _path_F(n, S):
    S = sorted(S)
    F = S[0] * (S[0] + 1) // 2  # end segment before the first member
    L = n - 1 - S[-1]
    F += L * (L + 1) // 2
    for a, b in zip(S, S[1:]):
        F += _h(b - a - 1)
    return F


def _cycle_F(n, S):
    S = sorted(S)
    F = 0
    for a, b in zip(S, S[1:] + [S[0] + n]):
        F += _h(b - a - 1)
    return F


def _segment_greedy(n, k, Ffun):
    S = []
    out = []
    for _ in range(k):
        best = None
        for v in range(n):
            if v in S:
                continue
            f = Ffun(n, S + [v])
            if best is None or f < best[0]:
                best = (f, v)
        S.append(best[1])
        out.append(best[0])
    return S, out


@pytest.mark.parametrize("n,k", [(9, 4), (20, 6), (33, 7)])
def test_path_greedy_segment_model(n, k):
    g = graphgen.path(n)
    grp, Fs = oracle.greedy(g, k)
    S, F = _segment_greedy(n, k, _path_F)
    assert grp.tolist() == S
    assert Fs.tolist() == F


@pytest.mark.parametrize("n,k", [(10, 4), (17, 5), (24, 6)])
def test_cycle_greedy_segment_model(n, k):
    g = graphgen.cycle(n)
    grp, Fs = oracle.greedy(g, k)
    S, F = _segment_greedy(n, k, _cycle_F)
    assert grp.tolist() == S
    assert Fs.tolist() == F
    # two members at 0 and v: F = h(v-1) + h(n-v-1)
    for v in range(1, n):
        assert oracle.farness(g, [0, v]) == _h(v - 1) + _h(n - v - 1)


# ------------------------------------------------ brute force on tiny graphs

TINY = [(n, p, s) for n, p, s in [(5, 0.3, 1), (6, 0.4, 2), (7, 0.2, 3), (8, 0.3, 4), (9, 0.25, 5),
                                   (10, 0.2, 6), (11, 0.3, 7), (12, 0.15, 8), (12, 0.4, 9)]]


@pytest.mark.parametrize("n,p,seed", TINY)
def test_bfs_and_farness_vs_floyd_warshall(n, p, seed):
    g = graphgen.gnp_connected(n, p, seed)
    D = small.floyd_warshall(g)
    for v in range(n):
        assert np.array_equal(oracle.bfs(g, v), D[v])
    rng = np.random.default_rng(seed)
    for _ in range(20):
        k = int(rng.integers(1, n + 1))
        S = rng.choice(n, size=k, replace=False).tolist()
        assert oracle.farness(g, S) == small.farness(D, S)
        assert np.array_equal(oracle.group_dist(g, S), D[S].min(axis=0))


@pytest.mark.parametrize("n,p,seed", TINY)
def test_topk_closeness_vs_floyd_warshall(n, p, seed):
    g = graphgen.gnp_connected(n, p, seed)
    D = small.floyd_warshall(g)
    F = D.sum(axis=1)
    exp = sorted(range(n), key=lambda v: (int(F[v]), v))
    for k in (1, 3, n):
        nodes, Fk = oracle.topk_closeness(g, k)
        assert nodes.tolist() == exp[:k]
        assert Fk.tolist() == [int(F[v]) for v in exp[:k]]
    grp, _ = oracle.greedy(g, 1)
    assert int(grp[0]) == exp[0]


@pytest.mark.parametrize("n,p,seed", TINY)
def test_greedy_vs_matrix_form_and_optimum(n, p, seed):
    g = graphgen.gnp_connected(n, p, seed)
    D = small.floyd_warshall(g)
    for k in range(1, n + 1):
        grp, Fs = oracle.greedy(g, k)
        S, F = small.greedy_matrix(D, k)
        assert grp.tolist() == S
        assert Fs.tolist() == F
        if k <= 5:
            opt, _ = small.brute_force_opt(D, k)
            assert opt <= int(Fs[-1])
            if k == 1:
                assert opt == int(Fs[0])


@pytest.mark.parametrize("n,p,seed", TINY)
def test_gains_theorem_identity(n, p, seed):
    g = graphgen.gnp_connected(n, p, seed)
    D = small.floyd_warshall(g)
    bits = small.bit_vectors(g, n)
    rng = np.random.default_rng(100 + seed)
    for _ in range(6):
        k = int(rng.integers(1, n))
        S = rng.choice(n, size=k, replace=False).tolist()
        dS = oracle.group_dist(g, S)
        for u in range(n):
            gu = oracle.gain(g, dS, u)
            assert gu == small.gain_def(D, S, u)
            assert gu == small.theorem_gain(bits, S, u)
            gp, _, _ = oracle.pruned_stats(g, dS, [u])
            assert int(gp[0]) == gu


@pytest.mark.parametrize("n,p,seed", [(6, 0.3, 11), (7, 0.35, 12), (7, 0.2, 13)])
def test_supermodularity_exhaustive(n, p, seed):
    """g(v,S) >= g(v,T) for all S subset T, v notin T (Section 3.2 lemma)."""
    g = graphgen.gnp_connected(n, p, seed)
    subsets = [list(c) for r in range(1, n) for c in itertools.combinations(range(n), r)]
    gain = {}
    for S in subsets:
        dS = oracle.group_dist(g, S)
        gs = oracle.gains(g, dS, np.arange(n, dtype=np.int32))
        for v in range(n):
            gain[(tuple(S), v)] = int(gs[v])
    for T in subsets:
        Tset = set(T)
        for r in range(1, len(T) + 1):
            for S in itertools.combinations(T, r):
                for v in range(n):
                    if v in Tset:
                        continue
                    assert gain[(tuple(S), v)] >= gain[(tuple(T), v)]


@pytest.mark.parametrize("n,p,seed", TINY[:5])
def test_tier_a_gain_rows(n, p, seed):
    g = graphgen.gnp_connected(n, p, seed)
    D = small.floyd_warshall(g)
    k = min(n, 5)
    grp, Fs, G = oracle.greedy(g, k, with_gains=True)
    for r in range(k - 1):
        S = grp[: r + 1].tolist()
        for v in range(n):
            if v in S:
                assert G[r, v] == -1
            else:
                assert G[r, v] == small.gain_def(D, S, v)


# -------------------------------------------------------- tier B vs tier A

TIERB = [lambda: graphgen.ba(400, 3, 21), lambda: graphgen.ba(300, 1, 22),
         lambda: graphgen.grid(12, 15, 23), lambda: graphgen.path(40), lambda: graphgen.cycle(33),
         lambda: graphgen.gnp_connected(60, 0.05, 24), lambda: graphgen.star(30),
         lambda: graphgen.complete_bipartite(4, 9)]


@pytest.mark.parametrize("mk", TIERB)
@pytest.mark.parametrize("block,growth", [(1, 1), (7, 1), (64, 1), (1, 2), (5, 3)])
def test_tier_b_equals_tier_a(mk, block, growth):
    g = mk()
    k = min(g.n, 12)
    grp_a, F_a = oracle.greedy(g, k)
    grp_b, F_b, ev, ed = oracle.greedypp(g, k, block=block, growth=growth)
    assert grp_b.tolist() == grp_a.tolist()
    assert F_b.tolist() == F_a.tolist()
    if k > 1:
        assert ev[1] == g.n - 1          # no bounds in the first round after s_1
        assert np.all(ev[2:] <= g.n - np.arange(2, k))


def test_tier_b_batch_schedule():
    """Batch sizes only move evaluation counts: every schedule gives the same
    picks and farness; a batch as large as the graph skips nothing, so every
    round evaluates all n - r candidates outside S."""
    g = graphgen.ba(500, 2, 31)
    k = 15
    runs = [oracle.greedypp(g, k, block=b, growth=gr) for b, gr in [(1, 1), (4, 1), (4, 2), (16, 4)]]
    for grp, F, ev, ed in runs[1:]:
        assert grp.tolist() == runs[0][0].tolist() and F.tolist() == runs[0][1].tolist()
        assert np.all(ev[1:] <= g.n - np.arange(1, k))
    grp, F, ev, ed = oracle.greedypp(g, k, block=g.n)
    assert grp.tolist() == runs[0][0].tolist()
    assert ev[1:].tolist() == (g.n - np.arange(1, k)).tolist()


def test_tier_b_equals_tier_a_ba2000():
    g = graphgen.workload("ba2000")
    grp_a, F_a = oracle.greedy(g, 10)
    grp_b, F_b, _, _ = oracle.greedypp(g, 10)
    assert grp_a.tolist() == grp_b.tolist()
    assert F_a.tolist() == F_b.tolist()


# ------------------------------------- gains and pruned-BFS statistics, pinned

GAIN_PIN = [lambda s=s: graphgen.gnp_connected(n, p, s) for n, p, s in TINY] + [
    lambda: graphgen.ba(150, 2, 41), lambda: graphgen.grid(9, 11, 42), lambda: graphgen.path(23),
    lambda: graphgen.star(17)]


@pytest.mark.parametrize("mk", GAIN_PIN)
def test_gains_vs_definition(mk):
    """or_gains (the checker of the GPU gain tests) equals g(v,S) = F(S) - F(S u {v})
    from Floyd-Warshall distances (Section 2), for every node -- members of S
    included (gain 0) -- and for random S of every size."""
    g = mk()
    n = g.n
    D = small.floyd_warshall(g)
    rng = np.random.default_rng(7 * n + 1)
    for k in sorted({1, 2, max(1, n // 4), n - 1}):
        S = rng.choice(n, size=k, replace=False).tolist()
        dS = oracle.group_dist(g, S)
        cand = np.concatenate([np.arange(n), rng.integers(0, n, size=5)]).astype(np.int32)
        got = oracle.gains(g, dS, cand)
        FS = small.farness(D, S)
        exp = [FS - small.farness(D, S + [int(v)]) for v in cand]
        assert got.tolist() == exp, (k, S)


@pytest.mark.parametrize("mk", GAIN_PIN)
def test_pruned_stats_vs_definition(mk):
    """or_pruned_stats: the pruned BFS of Section 4.1 visits exactly
    V(v) = {w : d(v,w) < d(S,w)} (a shortest path to such a w stays inside the
    set, by the triangle inequality), so |V(v)| and sum_{w in V(v)} deg(w)
    are fixed by Floyd-Warshall distances, and the gain is the definition."""
    g = mk()
    n = g.n
    D = small.floyd_warshall(g)
    deg = np.diff(g.row_ptr).astype(np.int64)
    rng = np.random.default_rng(11 * n + 3)
    for k in sorted({1, max(1, n // 3), n - 1}):
        S = rng.choice(n, size=k, replace=False).tolist()
        dS = D[S].min(axis=0)
        cand = np.arange(n, dtype=np.int32)
        gg, vv, ee = oracle.pruned_stats(g, dS.astype(np.int32), cand)
        inV = D < dS[None, :]              # row v: membership of every w in V(v)
        assert vv.tolist() == inV.sum(axis=1).tolist()
        assert ee.tolist() == (inV * deg[None, :]).sum(axis=1).tolist()
        FS = int(dS.sum())
        assert gg.tolist() == [FS - small.farness(D, S + [v]) for v in range(n)]
        for v in S:
            assert vv[v] == 0 and ee[v] == 0 and gg[v] == 0


def _malformed():
    """CSR contract violations (Section 2: connected, undirected, simple)."""
    G = graphgen.Graph
    rp = np.array([0, 2, 3, 4], np.int32)
    return {
        "missing reverse edge": G("x", 3, np.array([0, 2, 4, 5], np.int32),
                                  np.array([1, 2, 0, 2, 0], np.int32)),
        "self-loop": G("x", 3, np.array([0, 3, 5, 7], np.int32),
                       np.array([0, 1, 2, 0, 2, 0, 1], np.int32)),
        "duplicate": G("x", 3, np.array([0, 3, 5, 6], np.int32),
                       np.array([1, 1, 2, 0, 0, 0], np.int32)),
        "unsorted row": G("x", 3, rp, np.array([2, 1, 0, 0], np.int32)),
        "id out of range": G("x", 3, rp, np.array([1, 3, 0, 0], np.int32)),
        "disconnected": G("x", 4, np.array([0, 1, 2, 3, 4], np.int32),
                          np.array([1, 0, 3, 2], np.int32)),
        "row_ptr decreases": G("x", 3, np.array([0, 2, 1, 4], np.int32),
                               np.array([1, 2, 0, 0], np.int32)),
        "row_ptr[n] != nnz": G("x", 3, rp, np.array([1, 2, 0, 0, 0], np.int32)),
    }


@pytest.mark.parametrize("case", sorted(_malformed()))
def test_oracle_rejects_malformed_csr(case):
    g = _malformed()[case]
    with pytest.raises(oracle.OracleError):
        oracle.validate(g)
    with pytest.raises(oracle.OracleError):
        oracle.greedy(g, 1)
    with pytest.raises(oracle.OracleError):
        oracle.greedypp(g, 1)


def test_oracle_accepts_valid_csr():
    for g in (graphgen.path(1), graphgen.path(2), graphgen.ba(50, 2, 3), graphgen.grid(5, 6, 4)):
        oracle.validate(g)


# ------------------------------------------- early exit (BFScut-style bound)

@pytest.mark.parametrize("mk", GAIN_PIN)
def test_early_exit_bound_vs_definition(mk):
    """The early-exit search stops only when its bound cannot beat the
    threshold, and the bound it keeps is never below the gain of the
    definition (Floyd-Warshall); a search that runs to the end returns the
    gain itself."""
    g = mk()
    n = g.n
    D = small.floyd_warshall(g)
    rng = np.random.default_rng(13 * n + 5)
    for k in sorted({1, 2, max(1, n // 5)}):
        S = rng.choice(n, size=k, replace=False).tolist()
        dS = D[S].min(axis=0).astype(np.int32)
        FS = int(dS.sum())
        exact = [FS - small.farness(D, S + [v]) for v in range(n)]
        for thr in sorted({0, 1, int(np.median(exact)), max(exact), max(exact) + 5}):
            thr_id = int(rng.integers(0, n))
            val, cut = oracle.gains_cut(g, dS, np.arange(n, dtype=np.int32), thr, thr_id)
            for v in range(n):
                if cut[v]:
                    assert val[v] >= exact[v]
                    assert val[v] < thr or (val[v] == thr and v > thr_id)
                else:
                    assert val[v] == exact[v]


@pytest.mark.parametrize("mk", TIERB)
@pytest.mark.parametrize("mode,seed,block,growth", [(1, 1, 1, 1), (1, 5, 7, 2), (1, 1024, 64, 2),
                                                    (2, 3, 4, 1), (2, 64, 64, 2)])
def test_tier_b_early_exit_equals_tier_a(mk, mode, seed, block, growth):
    """Greedy++ with the early exit (first round, or every round) picks
    exactly the plain greedy's group; the first round still evaluates every
    candidate once."""
    g = mk()
    k = min(g.n, 12)
    grp_a, F_a = oracle.greedy(g, k)
    grp, F, ev, ed, cuts = oracle.greedypp_cut(g, k, block=block, growth=growth, mode=mode, seed=seed)
    assert grp.tolist() == grp_a.tolist()
    assert F.tolist() == F_a.tolist()
    if k > 1:
        assert ev[1] == g.n - 1
        assert np.all(cuts <= ev)
        if mode == 1:
            assert np.all(cuts[2:] == 0)


def test_early_exit_cuts_the_first_round():
    """On a 2,000-node Barabasi-Albert graph the first round's searches stop
    early for most candidates and scan fewer adjacency entries."""
    g = graphgen.workload("ba2000")
    _, _, ev0, ed0 = oracle.greedypp(g, 10, block=64, growth=2)
    _, _, ev1, ed1, cuts = oracle.greedypp_cut(g, 10, block=64, growth=2, mode=1, seed=64)
    assert cuts[1] > g.n // 4
    assert ed1[1] < ed0[1]


# ------------------------------------------------------------ directed graphs
# Section 2 also admits strongly connected directed graphs: d(S, w) is then
# the length of a shortest path from S to w along the arcs.

def _dcycle_F(n, S):
    """Directed cycle: the nodes after a member up to the next one form a gap
    of L nodes at distances 1..L."""
    S = sorted(S)
    F = 0
    for a, b in zip(S, S[1:] + [S[0] + n]):
        L = b - a - 1
        F += L * (L + 1) // 2
    return F


@pytest.mark.parametrize("n,k", [(5, 3), (12, 4), (21, 6)])
def test_directed_cycle_closed_forms(n, k):
    g = graphgen.directed_cycle(n)
    assert np.all(oracle.farness_all(g) == n * (n - 1) // 2)
    grp, Fs = oracle.greedy(g, k)
    S, F = _segment_greedy(n, k, _dcycle_F)
    assert grp.tolist() == S and Fs.tolist() == F
    grp_b, F_b, _, _ = oracle.greedypp(g, k, block=3, growth=2)
    assert grp_b.tolist() == S and F_b.tolist() == F


DIRECTED = [(6, 0.2, 1), (9, 0.15, 2), (12, 0.1, 3), (12, 0.3, 4), (30, 0.06, 5)]


@pytest.mark.parametrize("n,p,seed", DIRECTED)
def test_directed_against_floyd_warshall(n, p, seed):
    """BFS along arcs, farness, gains, pruned-BFS statistics, greedy (against
    the matrix form and, for n <= 12, the brute-force optimum) and Greedy++
    (with and without the early exit) on random strongly connected digraphs."""
    g = graphgen.gnp_directed(n, p, seed)
    oracle.validate(g)
    D = small.floyd_warshall(g)
    assert np.all(D < small.INF)  # strongly connected
    for v in range(g.n):
        assert np.array_equal(oracle.bfs(g, v), D[v])
    rng = np.random.default_rng(seed)
    deg = np.diff(g.row_ptr).astype(np.int64)
    for _ in range(5):
        S = rng.choice(g.n, size=int(rng.integers(1, g.n)), replace=False).tolist()
        dS = D[S].min(axis=0).astype(np.int32)
        assert np.array_equal(oracle.group_dist(g, S), dS)
        gains = oracle.gains(g, dS, np.arange(g.n, dtype=np.int32))
        assert gains.tolist() == [small.gain_def(D, S, v) for v in range(g.n)]
        gg, vv, ee = oracle.pruned_stats(g, dS, np.arange(g.n, dtype=np.int32))
        inV = D < dS[None, :]
        assert gg.tolist() == gains.tolist()
        assert vv.tolist() == inV.sum(axis=1).tolist()
        assert ee.tolist() == (inV * deg[None, :]).sum(axis=1).tolist()
    for k in range(1, min(g.n, 7) + 1):
        grp, Fs = oracle.greedy(g, k)
        S, F = small.greedy_matrix(D, k)
        assert grp.tolist() == S and Fs.tolist() == F
        if g.n <= 12 and k <= 4:
            opt, _ = small.brute_force_opt(D, k)
            assert opt <= int(Fs[-1])
        grp_b, F_b, _, _ = oracle.greedypp(g, k, block=2, growth=2)
        assert grp_b.tolist() == S and F_b.tolist() == F
        grp_c, F_c, _, _, _ = oracle.greedypp_cut(g, k, block=2, growth=2, mode=2, seed=2)
        assert grp_c.tolist() == S and F_c.tolist() == F


def test_directed_validation():
    """A directed path is not strongly connected; read as undirected, a
    one-way arc has no reverse edge."""
    G = graphgen.Graph
    dpath = G("x", 3, np.array([0, 1, 2, 2], np.int32), np.array([1, 2], np.int32))
    dpath.directed = True
    with pytest.raises(oracle.OracleError, match="disconnected"):
        oracle.validate(dpath)
    with pytest.raises(oracle.OracleError):
        oracle.greedy(dpath, 1)
    undirected = G("x", 3, np.array([0, 1, 2, 3], np.int32), np.array([1, 2, 0], np.int32))
    with pytest.raises(oracle.OracleError, match="symmetric"):
        oracle.validate(undirected)
    undirected.directed = True
    oracle.validate(undirected)  # the directed 3-cycle
    oracle.validate(graphgen.rmat_directed(10, 8, 3))


# ------------------------------------------------------------ weighted graphs
# Section 2 defines distances through SSSP, of which BFS is the unit-length
# case; the oracle's weighted path is Dijkstra with a binary heap.

def _star_weighted():
    """Star with centre 0 and leaves 1..4; edge 0-1 has length 10, the rest 1."""
    g = graphgen.star(5)
    w = np.ones(g.nnz, dtype=np.uint8)
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            if {u, int(g.col_idx[e])} == {0, 1}:
                w[e] = 10
    return graphgen.with_weight_array(g, w)


def test_weighted_star_by_hand():
    """Worked by hand: F({0}) = 10+1+1+1 = 13, F({1}) = 10+3*11 = 43,
    F({2}) = 1+11+2+2 = 16 (and so for leaves 3, 4); from {0}, leaf 1 gains
    10 and every other leaf 1, so the group grows 0, 1, 2, 3, 4 with
    F = 13, 3, 2, 1, 0."""
    g = _star_weighted()
    oracle.validate(g)
    assert oracle.sssp(g, 0).tolist() == [0, 10, 1, 1, 1]
    assert oracle.sssp(g, 2).tolist() == [1, 11, 0, 2, 2]
    assert oracle.farness_all(g).tolist() == [13, 43, 16, 16, 16]
    for tier in (lambda k: oracle.greedy(g, k), lambda k: oracle.greedypp(g, k, block=1)[:2]):
        grp, F = tier(5)
        assert grp.tolist() == [0, 1, 2, 3, 4]
        assert F.tolist() == [13, 3, 2, 1, 0]


@pytest.mark.parametrize("n,seed", [(2, 1), (7, 2), (30, 3)])
def test_weighted_path_prefix_sums(n, seed):
    """On a path, d(u, v) is the difference of prefix sums of the lengths."""
    g = graphgen.with_weights(graphgen.path(n), 9, seed)
    lens = [int(g.weight[int(g.row_ptr[i]) + (1 if i > 0 else 0)]) for i in range(n - 1)]
    pre = np.concatenate([[0], np.cumsum(lens)])
    for u in range(n):
        assert oracle.sssp(g, u).tolist() == np.abs(pre - pre[u]).tolist()


@pytest.mark.parametrize("mk", [lambda: graphgen.ba(300, 3, 5), lambda: graphgen.grid(12, 14, 3),
                                lambda: graphgen.rmat_directed(8, 8, 4)])
@pytest.mark.parametrize("c", [1, 3, 255])
def test_weighted_uniform_lengths_scale(mk, c):
    """Every edge of length c multiplies every distance by c: the greedy
    picks the same group and every F is c times the unweighted one."""
    g = mk()
    gw = graphgen.with_weight_array(g, np.full(g.nnz, c, np.uint8))
    for v in (0, g.n // 2, g.n - 1):
        assert np.array_equal(oracle.sssp(gw, v), c * oracle.bfs(g, v))
    grp, F = oracle.greedy(g, 6)
    grp_w, F_w = oracle.greedy(gw, 6)
    assert grp_w.tolist() == grp.tolist() and F_w.tolist() == (c * F).tolist()
    grp_b, F_b, ev, _ = oracle.greedypp(gw, 6, block=4, growth=2)
    assert grp_b.tolist() == grp.tolist() and F_b.tolist() == (c * F).tolist()


WTINY = [(n, p, s, wmax) for (n, p, s), wmax in zip(TINY, [2, 3, 5, 9, 17, 40, 100, 255, 7])]


@pytest.mark.parametrize("n,p,seed,wmax", WTINY)
def test_weighted_against_floyd_warshall(n, p, seed, wmax):
    """SSSP, group distances, farness, gains, pruned-search statistics, the
    greedy (against the matrix form and, for small k, the brute-force
    optimum) and Greedy++ on tiny weighted graphs."""
    g = graphgen.with_weights(graphgen.gnp_connected(n, p, seed), wmax, seed + 50)
    oracle.validate(g)
    D = small.floyd_warshall(g)
    deg = np.diff(g.row_ptr).astype(np.int64)
    for v in range(n):
        assert np.array_equal(oracle.sssp(g, v), D[v])
    assert oracle.farness_all(g).tolist() == D.sum(axis=1).tolist()
    rng = np.random.default_rng(seed)
    for _ in range(6):
        S = rng.choice(n, size=int(rng.integers(1, n)), replace=False).tolist()
        dS = D[S].min(axis=0).astype(np.int32)
        assert np.array_equal(oracle.group_dist(g, S), dS)
        assert oracle.farness(g, S) == small.farness(D, S)
        cand = np.arange(n, dtype=np.int32)
        gains = oracle.gains(g, dS, cand)
        assert gains.tolist() == [small.gain_def(D, S, v) for v in range(n)]
        gg, vv, ee = oracle.pruned_stats(g, dS, cand)
        inV = D < dS[None, :]
        assert gg.tolist() == gains.tolist()
        assert vv.tolist() == inV.sum(axis=1).tolist()
        assert ee.tolist() == (inV * deg[None, :]).sum(axis=1).tolist()
    for k in range(1, n + 1):
        grp, Fs = oracle.greedy(g, k)
        S, F = small.greedy_matrix(D, k)
        assert grp.tolist() == S and Fs.tolist() == F
        if k <= 4:
            opt, _ = small.brute_force_opt(D, k)
            assert opt <= int(Fs[-1])
            if k == 1:
                assert opt == int(Fs[0])
        for block, growth in ((1, 1), (3, 2)):
            grp_b, F_b, _, _ = oracle.greedypp(g, k, block=block, growth=growth)
            assert grp_b.tolist() == S and F_b.tolist() == F


@pytest.mark.parametrize("n,p,seed", DIRECTED)
def test_weighted_directed_against_floyd_warshall(n, p, seed):
    g = graphgen.with_weights(graphgen.gnp_directed(n, p, seed), 20, seed)
    oracle.validate(g)
    D = small.floyd_warshall(g)
    for v in range(g.n):
        assert np.array_equal(oracle.sssp(g, v), D[v])
    for k in range(1, min(g.n, 6) + 1):
        grp, Fs = oracle.greedy(g, k)
        S, F = small.greedy_matrix(D, k)
        assert grp.tolist() == S and Fs.tolist() == F
        grp_b, F_b, _, _ = oracle.greedypp(g, k, block=2, growth=2)
        assert grp_b.tolist() == S and F_b.tolist() == F


@pytest.mark.parametrize("mk", [lambda: graphgen.ba(700, 4, 1), lambda: graphgen.rmat(10, 8, 9),
                                lambda: graphgen.grid(24, 30, 2)])
@pytest.mark.parametrize("wmax", [4, 255])
def test_weighted_tier_b_equals_tier_a(mk, wmax):
    g = graphgen.with_weights(mk(), wmax, 17)
    grp, F = oracle.greedy(g, 6)
    for block, growth in ((1, 1), (64, 2)):
        grp_b, F_b, ev, ed = oracle.greedypp(g, 6, block=block, growth=growth)
        assert grp_b.tolist() == grp.tolist() and F_b.tolist() == F.tolist()
        assert ev[0] == 0 and np.all(ev[1:] >= 1)
    # the pruned update matches group distances from scratch
    dS = oracle.group_dist(g, grp)
    assert int(dS.astype(np.int64).sum()) == int(F[-1])


def test_weighted_validation():
    g = _star_weighted()
    bad = g.weight.copy()
    bad[0] = 0
    with pytest.raises(oracle.OracleError, match="malformed|invalid"):
        oracle.validate(graphgen.with_weight_array(g, bad))
    asym = g.weight.copy()
    asym[0] = 7  # row 0's edge to 1 keeps 10 in row 1
    with pytest.raises(oracle.OracleError, match="symmetric"):
        oracle.validate(graphgen.with_weight_array(g, asym))
    with pytest.raises(oracle.OracleError):
        oracle.greedy(graphgen.with_weight_array(g, asym), 2)
    with pytest.raises(oracle.OracleError, match="weight"):
        oracle.greedy(graphgen.Graph("x", g.n, g.row_ptr, g.col_idx, weight=g.weight[:-1]), 2)
    d = graphgen.with_weights(graphgen.directed_cycle(5), 9, 1)
    d.weight[0] = 3
    oracle.validate(d)  # a directed arc's length need not match any other
    with pytest.raises(oracle.OracleError):
        oracle.bfs(g, 0)
    with pytest.raises(oracle.OracleError):
        oracle.greedypp_cut(g, 2)
