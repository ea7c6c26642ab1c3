"""Directed graphs (gc_load_csr with GC_DIRECTED; Section 2 admits strongly
connected directed graphs, with d(S, w) measured along the arcs): the HIP path
against the CPU oracle, bit-exact -- first pick and top-k closeness, d(S,.)
updates, marginal gains, Greedy++ in every order, the early exit and
bitGreedy++, and the contract checks of the load."""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[case] " + msg, flush=True)


SMALL = [lambda: graphgen.directed_cycle(9), lambda: graphgen.directed_cycle(300),
         lambda: graphgen.gnp_directed(12, 0.15, 2), lambda: graphgen.gnp_directed(40, 0.05, 3),
         lambda: graphgen.gnp_directed(60, 0.1, 4), lambda: graphgen.rmat_directed(10, 8, 5)]


@pytest.mark.parametrize("mk", SMALL)
def test_directed_small(gclib, device, mk):
    g = mk()
    assert g.directed
    _note("directed %s n=%d nnz=%d" % (g.name, g.n, g.nnz))
    G = gclib.Graph.from_graphgen(g)
    F1 = oracle.farness_all(g)
    order = np.lexsort((np.arange(g.n), F1))
    node, far = G.closest_node()
    assert (node, far) == (int(order[0]), int(F1[order[0]]))
    kk = min(5, g.n)
    nodes, fars = G.topk_closeness(kk)
    assert nodes.tolist() == order[:kk].tolist() and fars.tolist() == F1[order[:kk]].tolist()
    k = min(g.n, 8)
    grp_a, F_a = oracle.greedy(g, k)
    for o in ("plain", "celf"):
        grp, F, st = G.greedy_group(k, order=o, block=4)
        assert grp.tolist() == grp_a.tolist() and F.tolist() == F_a.tolist(), o
    _, _, ev_b, ed_b = oracle.greedypp(g, k, block=4, growth=2)
    grp, F, st = G.greedy_group(k, order="plain", block=4, block_growth=2)
    assert st["evals_per_round"].tolist() == ev_b.tolist() and st["edges_alg"] == int(ed_b.sum())
    # d(S,.) and every gain for a random S
    rng = np.random.default_rng(g.n)
    S = rng.choice(g.n, size=min(3, g.n - 1), replace=False).tolist()
    db = 2 if g.n > 250 else 1  # distances below n fit uint8 on the smaller graphs
    dist = G.new_dist(db)
    far_t = torch.zeros(1, dtype=torch.int64, device=device)
    for s in S:
        G.update_dist(s, dist, db, far_t)
    dS = oracle.group_dist(g, S)
    got = dist.view(torch.uint8 if db == 1 else torch.int16)[: g.n].cpu().numpy().astype(np.int64)
    if db == 2:
        got = got & 0xFFFF
    assert got.tolist() == dS.tolist()
    assert int(far_t.item()) == int(dS.sum())
    cand = torch.arange(g.n, dtype=torch.int32, device=device)
    gains = G.marginal_gains(dist, db, cand)
    assert gains.cpu().numpy().tolist() == oracle.gains(g, dS, np.arange(g.n, dtype=np.int32)).tolist()


def test_directed_rmat14(gclib):
    """A directed R-MAT graph (scale 14, largest strongly connected
    component): Greedy++ against tier B (group, F, evaluations and scanned
    arcs per round) and tier A, CELF and the early exit."""
    g = graphgen.rmat_directed(14, 16, 7)
    _note("directed rmat14 n=%d nnz=%d" % (g.n, g.nnz))
    G = gclib.Graph.from_graphgen(g)
    k = 20
    grp_a, F_a = oracle.greedy(g, k)
    grp_b, F_b, ev_b, ed_b = oracle.greedypp(g, k, block=64, growth=2)
    assert grp_b.tolist() == grp_a.tolist() and F_b.tolist() == F_a.tolist()
    grp, F, st = G.greedy_group(k, order="plain", block=64)
    assert grp.tolist() == grp_a.tolist() and F.tolist() == F_a.tolist()
    assert st["evals_per_round"].tolist() == ev_b.tolist() and st["edges_alg"] == int(ed_b.sum())
    grp, F, _ = G.greedy_group(k, order="celf", block=64)
    assert grp.tolist() == grp_a.tolist() and F.tolist() == F_a.tolist()
    grp_c, F_c, ev_c, ed_c, cuts = oracle.greedypp_cut(g, k, block=64, growth=2, mode=1, seed=256)
    grp, F, st = G.greedy_group(k, order="plain", block=64, early_exit=1, early_exit_seed=256)
    assert grp.tolist() == grp_a.tolist() and F.tolist() == F_a.tolist()
    assert st["evals_per_round"].tolist() == ev_c.tolist() and st["cut_evals"] == int(cuts.sum())


def test_directed_bitgreedy(gclib):
    g = graphgen.rmat_directed(11, 8, 8)
    G = gclib.Graph.from_graphgen(g)
    k = 10
    grp_a, F_a = oracle.greedy(g, k)
    G.bits_prepare(64)
    grp, F, _ = G.greedy_group(k, order="plain", bits=True)
    assert grp.tolist() == grp_a.tolist() and F.tolist() == F_a.tolist()


def test_directed_load_contract(gclib):
    dpath_rp = np.array([0, 1, 2, 2], np.int32)
    dpath_ci = np.array([1, 2], np.int32)
    with pytest.raises(gclib.GCError) as e:
        gclib.Graph(dpath_rp, dpath_ci, directed=True)
    assert e.value.code == gclib.GC_EDISCONNECTED
    cyc_rp = np.array([0, 1, 2, 3], np.int32)
    cyc_ci = np.array([1, 2, 0], np.int32)
    with pytest.raises(gclib.GCError) as e:
        gclib.Graph(cyc_rp, cyc_ci)
    assert e.value.code == gclib.GC_ENOTSYM
    G = gclib.Graph(cyc_rp, cyc_ci, directed=True)
    grp, F, _ = G.greedy_group(2)
    assert grp.tolist() == [0, 1] and F.tolist() == [3, 1]
