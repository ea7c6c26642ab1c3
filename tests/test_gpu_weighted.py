"""Weighted graphs (gc_load_csr_weighted; Section 2 defines distances through
SSSP, BFS being the unit-length case): the HIP path against the CPU oracle
(Dijkstra), bit-exact -- first pick and top-k closeness, d(S,.) updates,
marginal gains with their pruned-search statistics, Greedy++ in plain and
CELF order (evaluation counts too), a resumed prefix, every launch shape the
environment can set, unit lengths against the unweighted engine, and the
contract checks of the load and of the calls that have no weighted form."""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[case] " + msg, flush=True)


def _star():
    g = graphgen.star(5)
    w = np.ones(g.nnz, dtype=np.uint8)
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            if {u, int(g.col_idx[e])} == {0, 1}:
                w[e] = 10
    return graphgen.with_weight_array(g, w)


def _w(mk, wmax, seed=9):
    return lambda: graphgen.with_weights(mk(), wmax, seed)


SMALL = [_star,
         _w(lambda: graphgen.path(40), 9),
         _w(lambda: graphgen.gnp_connected(12, 0.3, 1), 20),
         _w(lambda: graphgen.ba(600, 3, 1), 255),
         _w(lambda: graphgen.grid(30, 30, 2), 7),
         _w(lambda: graphgen.rmat(10, 8, 3), 100),
         _w(lambda: graphgen.gnp_directed(40, 0.08, 2), 50),
         _w(lambda: graphgen.rmat_directed(9, 8, 3), 30)]


def _dist_np(dist, n):
    return dist[:n].cpu().numpy().astype(np.int64)


def _check_ops(gclib, device, g, G, seed):
    """d(S,.) by updates from S = {}, then every node's gain, |V(v)| and
    adjacency entries against the oracle's pruned Dijkstra."""
    rng = np.random.default_rng(seed)
    S = rng.choice(g.n, size=min(3, g.n - 1), replace=False).tolist()
    dist = G.new_dist(4)
    far_t = torch.zeros(1, dtype=torch.int64, device=device)
    for i, s in enumerate(S):
        G.update_dist(s, dist, 4, far_t)
        dS = oracle.group_dist(g, S[: i + 1])
        assert _dist_np(dist, g.n).tolist() == dS.tolist()
        assert int(far_t.item()) == int(dS.astype(np.int64).sum())
    cand = torch.arange(g.n, dtype=torch.int32, device=device)
    gain, edges, vis = G.marginal_gains(dist, 4, cand, stats=True)
    gg, vv, ee = oracle.pruned_stats(g, dS, np.arange(g.n, dtype=np.int32))
    assert gain.cpu().numpy().tolist() == gg.tolist()
    assert vis.cpu().numpy().tolist() == vv.tolist()
    assert edges.cpu().numpy().tolist() == ee.tolist()
    # duplicates, members of S and a reversed order
    cand2 = torch.tensor(list(reversed(S)) + [S[0]] * 3 + list(range(g.n - 1, -1, -7)), dtype=torch.int32,
                         device=device)
    exp = oracle.gains(g, dS, cand2.cpu().numpy())
    assert G.marginal_gains(dist, 4, cand2).cpu().numpy().tolist() == exp.tolist()


@pytest.mark.parametrize("mk", SMALL)
def test_weighted_small(gclib, device, mk):
    g = mk()
    _note("weighted %s n=%d nnz=%d" % (g.name, g.n, g.nnz))
    G = gclib.Graph.from_graphgen(g)
    assert G.weighted
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
        assert st["dist_bytes"] == 4
    _, _, ev_b, ed_b = oracle.greedypp(g, k, block=4, growth=2)
    grp, F, st = G.greedy_group(k, order="plain", block=4, block_growth=2, debug=True)
    assert st["evals_per_round"].tolist() == ev_b.tolist() and st["edges_alg"] == int(ed_b.sum())
    if k > 3:
        grp_p, F_p, _ = G.greedy_group(k, prefix=grp_a[:3])
        assert grp_p.tolist() == grp_a.tolist() and F_p.tolist() == F_a.tolist()
    if g.n > 1:
        _check_ops(gclib, device, g, G, g.n)


MEDIUM = [(lambda: graphgen.ba(5000, 4, 3), 255), (lambda: graphgen.grid(80, 80, 5), 255),
          (lambda: graphgen.rmat(12, 8, 7), 255), (lambda: graphgen.rmat(11, 16, 3), 3),
          (lambda: graphgen.rmat_directed(12, 8, 5), 60)]


@pytest.mark.parametrize("mk,wmax", MEDIUM)
def test_weighted_medium(gclib, device, mk, wmax):
    """Near lists of many 256-node tiles with ragged tails, hubs whose rows
    span the whole workgroup, and more candidates than search slots."""
    g = graphgen.with_weights(mk(), wmax, 11)
    _note("weighted %s n=%d nnz=%d" % (g.name, g.n, g.nnz))
    G = gclib.Graph.from_graphgen(g)
    k = 12
    grp_b, F_b, ev_b, ed_b = oracle.greedypp(g, k, block=64, growth=2)
    for o in ("plain", "celf"):
        grp, F, st = G.greedy_group(k, order=o)
        assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist(), o
        if o == "plain":
            assert st["evals_per_round"].tolist() == ev_b.tolist()
            assert st["edges_alg"] == int(ed_b.sum())
    nodes, fars = G.topk_closeness(3)
    F1 = oracle.farness_all(g)
    order = np.lexsort((np.arange(g.n), F1))
    assert nodes.tolist() == order[:3].tolist() and fars.tolist() == F1[order[:3]].tolist()
    _check_ops(gclib, device, g, G, 5)


ENVS = [{"GC_WSLOTS": "1"}, {"GC_WSLOTS": "3"}, {"GC_WDELTA": "1"}, {"GC_WDELTA": "5000"},
        {"GC_WDELTA_CLOSE": "1"}, {"GC_WDELTA_CLOSE": "4000"}, {"GC_VIS_BUDGET_MB": "1"},
        {"GC_WCLOSE_THREADS": "256"}, {"GC_WCLOSE_SLOTS": "1"}, {"GC_WCLOSE_SLOTS": "5", "GC_WSLOTS": "2"}]


@pytest.mark.parametrize("env", ENVS, ids=lambda e: ",".join("%s=%s" % kv for kv in e.items()))
def test_weighted_launch_shapes(gclib, device, monkeypatch, env):
    """Slot counts and bucket widths change only how the work is spread."""
    for key, val in env.items():
        monkeypatch.setenv(key, val)
    for mk in (lambda: graphgen.ba(1500, 3, 4), lambda: graphgen.grid(25, 40, 6)):
        g = graphgen.with_weights(mk(), 255, 13)
        _note("weighted env %s %s" % (env, g.name))
        G = gclib.Graph.from_graphgen(g)
        grp_b, F_b, ev_b, _ = oracle.greedypp(g, 10, block=8, growth=2)
        grp, F, st = G.greedy_group(10, block=8)
        assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
        assert st["evals_per_round"].tolist() == ev_b.tolist()
        F1 = oracle.farness_all(g)
        order = np.lexsort((np.arange(g.n), F1))
        assert G.closest_node() == (int(order[0]), int(F1[order[0]]))


@pytest.mark.parametrize("mk", [lambda: graphgen.ba(3000, 4, 8), lambda: graphgen.rmat(12, 16, 2),
                                lambda: graphgen.rmat_directed(11, 8, 6)])
def test_unit_lengths_match_unweighted_engine(gclib, device, mk):
    """Every length 1: the weighted searches and the bit-parallel pruned BFS
    must pick the same group with the same farness."""
    g = mk()
    gw = graphgen.with_weight_array(g, np.ones(g.nnz, np.uint8))
    _note("unit lengths %s" % g.name)
    Gu = gclib.Graph.from_graphgen(g)
    Gw = gclib.Graph.from_graphgen(gw)
    grp_u, F_u, _ = Gu.greedy_group(20)
    grp_w, F_w, _ = Gw.greedy_group(20, order="celf")
    assert grp_w.tolist() == grp_u.tolist() and F_w.tolist() == F_u.tolist()
    assert Gw.topk_closeness(4)[0].tolist() == Gu.topk_closeness(4)[0].tolist()


def test_weighted_load_contract(gclib, device):
    g = _star()
    bad = g.weight.copy()
    bad[0] = 0
    with pytest.raises(gclib.GCError) as ei:
        gclib.Graph(g.row_ptr, g.col_idx, weight=bad)
    assert ei.value.code == gclib.GC_EINVAL
    asym = g.weight.copy()
    asym[0] = 7
    with pytest.raises(gclib.GCError) as ei:
        gclib.Graph(g.row_ptr, g.col_idx, weight=asym)
    assert ei.value.code == gclib.GC_ENOTSYM
    with pytest.raises(ValueError):
        gclib.Graph(g.row_ptr, g.col_idx, weight=g.weight[:-1])
    # directed: any lengths
    d = graphgen.with_weights(graphgen.directed_cycle(6), 9, 1)
    d.weight[0] = 200
    Gd = gclib.Graph.from_graphgen(d)
    assert Gd.closest_node()[1] == int(oracle.farness_all(d).min())
    # n >= 2^23 is refused before anything is read
    n = 1 << 23
    rp = torch.zeros(n + 1, dtype=torch.int32, device=device)
    ci = torch.zeros(0, dtype=torch.int32, device=device)
    with pytest.raises(gclib.GCError) as ei:
        gclib.Graph(rp, ci, weight=torch.zeros(0, dtype=torch.uint8), validate=False, workspace=False)
    assert ei.value.code == gclib.GC_ERANGE


def test_weighted_calls_without_a_weighted_form(gclib, device):
    g = graphgen.with_weights(graphgen.ba(300, 3, 2), 50, 3)
    G = gclib.Graph.from_graphgen(g)
    dist = G.new_dist(4)
    far_t = torch.zeros(1, dtype=torch.int64, device=device)
    G.update_dist(0, dist, 4, far_t)
    cand = torch.arange(10, dtype=torch.int32, device=device)

    def code(f):
        with pytest.raises(gclib.GCError) as ei:
            f()
        return ei.value.code

    assert code(lambda: G.update_dist(1, dist, 2, far_t)) == gclib.GC_EINVAL
    assert code(lambda: G.marginal_gains(dist, 1, cand)) == gclib.GC_EINVAL
    assert code(lambda: G.greedy_group(5, early_exit=1)) == gclib.GC_EINVAL
    assert code(lambda: G.greedy_group(5, order="learned")) == gclib.GC_EINVAL
    assert code(lambda: G.greedy_group(5, log_capacity=10)) == gclib.GC_EINVAL
    assert code(lambda: G.bits_prepare(4)) == gclib.GC_EINVAL
    assert code(lambda: G.gain_words()) == gclib.GC_EINVAL
    gain = torch.zeros(10, dtype=torch.int64, device=device)
    assert code(lambda: G.marginal_gains_noalloc(dist, 4, cand, gain)) == gclib.GC_EINVAL
    # an id outside [0, n) is rejected by the binding; at the C ABI it gets 0
    lib = gclib.load_library()
    bad = torch.tensor([-1, g.n, 5], dtype=torch.int32, device=device)
    out = torch.full((3,), 77, dtype=torch.int64, device=device)
    gclib._check(lib.gc_marginal_gains(G.handle, gclib._ptr(dist), 4, gclib._ptr(bad), 3, gclib._ptr(out),
                                       None, None, gclib._ptr(G.ws), G.ws_bytes, gclib._stream()))
    exp5 = int(oracle.gains(g, oracle.group_dist(g, [0]), [5])[0])
    assert out.cpu().tolist() == [0, 0, exp5]
