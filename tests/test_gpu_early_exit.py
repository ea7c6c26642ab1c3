"""GPU parity of the early exit inside the first gain round's pruned BFSs
(gc_opts.early_exit) against the CPU Greedy++ with the same early exit (tier
B, greedypp_cut): the same group and F(S_i), the same evaluations and scanned
adjacency entries in every round, the same number of stopped searches; the
picks equal the plain greedy (tier A) or the plain GPU run."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[case] " + msg, flush=True)


def _check(gclib, g, k, block, growth, seed, exact=None, engine_env=None):
    G = gclib.Graph.from_graphgen(g)
    grp_b, F_b, ev_b, ed_b, cuts_b = oracle.greedypp_cut(g, k, block=block, growth=growth, mode=1, seed=seed)
    if exact is not None:
        assert grp_b.tolist() == exact[0] and F_b.tolist() == exact[1]
    _note("%s k=%d block %d growth %d seed %d, early exit" % (g.name, k, block, growth, seed))
    grp, F, st = G.greedy_group(k, order="plain", block=block, block_growth=growth, early_exit=1,
                                early_exit_seed=seed)
    assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
    assert st["evals_per_round"].tolist() == ev_b.tolist()
    assert st["edges_alg"] == int(ed_b.sum())
    assert st["cut_evals"] == int(cuts_b.sum())
    for order in ("celf",):
        _note("%s k=%d %s, early exit" % (g.name, k, order))
        grp_c, F_c, st_c = G.greedy_group(k, order=order, block=block, block_growth=growth, early_exit=1,
                                          early_exit_seed=seed)
        assert grp_c.tolist() == grp_b.tolist() and F_c.tolist() == F_b.tolist()
    return st, cuts_b


SMALL = [lambda: graphgen.path(7), lambda: graphgen.path(300), lambda: graphgen.star(12),
         lambda: graphgen.gnp_connected(40, 0.08, 6), lambda: graphgen.ba(300, 2, 11),
         lambda: graphgen.grid(17, 13, 3), lambda: graphgen.complete_bipartite(3, 5)]


@pytest.mark.parametrize("mk", SMALL)
@pytest.mark.parametrize("seed", [1, 16])
def test_early_exit_small(gclib, mk, seed):
    g = mk()
    k = min(g.n, 8)
    grp_a, F_a = oracle.greedy(g, k)
    _check(gclib, g, k, 4, 2, seed, exact=(grp_a.tolist(), F_a.tolist()))


def test_early_exit_ba2000(gclib):
    g = graphgen.workload("ba2000")
    grp_a, F_a = oracle.greedy(g, 10)
    st, cuts = _check(gclib, g, 10, 64, 2, 64, exact=(grp_a.tolist(), F_a.tolist()))
    assert cuts[1] > 0 and st["cut_evals"] > 0


@pytest.mark.parametrize("seed", [64, 1024])
def test_early_exit_rmat16(gclib, seed):
    g = graphgen.workload("rmat16")
    st, cuts = _check(gclib, g, 50, 64, 2, seed)
    assert cuts[1] > g.n // 2  # most first-round searches stop early


def test_early_exit_grid_u16(gclib):
    """A 64x64 grid (deep BFS, many levels tested) and a 900x5 strip (16-bit
    distances)."""
    st, cuts = _check(gclib, graphgen.grid(64, 64, 21), 12, 64, 2, 256)
    assert cuts[1] > 0
    st, _ = _check(gclib, graphgen.grid(900, 5, 22, shortcut_frac=0.0), 6, 16, 2, 64)
    assert st["dist_bytes"] == 2


def test_early_exit_fixed_blocks_and_chunked_launches(gclib, monkeypatch):
    """Fixed blocks (growth 1), and first-round launches split into many
    chunks by a small record budget: the threshold of the stopped searches
    is fixed for the round, so the results do not depend on the chunks."""
    g = graphgen.ba(3000, 3, 41)
    _check(gclib, g, 15, 16, 1, 128)
    monkeypatch.setenv("GC_VIS_BUDGET_MB", "1")
    _check(gclib, g, 15, 16, 3, 128)


def test_early_exit_argument_checks(gclib):
    G = gclib.Graph.from_graphgen(graphgen.ba(200, 2, 5))
    for bad in (-1, 2):
        with pytest.raises(gclib.GCError):
            G.greedy_group(3, early_exit=bad)
    with pytest.raises(gclib.GCError):
        G.greedy_group(3, early_exit=1, early_exit_seed=-4)
