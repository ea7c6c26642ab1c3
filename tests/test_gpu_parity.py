"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every result is integer, so the bar is bit-exact: the group, its order (ties
to the smallest id), every F(S_i), every evaluated gain and d(S,.) itself.
"""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[case] " + msg, flush=True)


def _graph(gclib, g):
    _note("load %s n=%d nnz=%d" % (g.name, g.n, g.nnz))
    return gclib.Graph.from_graphgen(g)


SMALL = [
    lambda: graphgen.path(1),            # one node, no edges: k = n = 1
    lambda: graphgen.path(2),
    lambda: graphgen.path(7),
    lambda: graphgen.path(300),          # eccentricity > 254: 16-bit distances
    lambda: graphgen.cycle(9),
    lambda: graphgen.star(12),
    lambda: graphgen.complete(6),
    lambda: graphgen.complete_bipartite(3, 5),
    lambda: graphgen.gnp_connected(12, 0.2, 5),
    lambda: graphgen.gnp_connected(40, 0.08, 6),
    lambda: graphgen.ba(300, 2, 11),
    lambda: graphgen.grid(17, 13, 3),
]


@pytest.mark.parametrize("mk", SMALL, ids=lambda f: "small")
def test_closest_node_small(gclib, mk):
    g = mk()
    G = _graph(gclib, g)
    F = oracle.farness_all(g)
    s_ref = int(np.argmin(F))
    _note("closest_node %s" % g.name)
    s, f = G.closest_node()
    assert (s, f) == (s_ref, int(F[s_ref]))


@pytest.mark.parametrize("mk", SMALL + [lambda: graphgen.rmat(12, 16, 7), lambda: graphgen.grid(64, 64, 4)],
                         ids=lambda f: "topk")
def test_topk_closeness(gclib, mk):
    """Top-k closeness for several k, including k = n on the small graphs:
    nodes and farness equal the definition's ranking."""
    g = mk()
    G = _graph(gclib, g)
    for k in sorted({1, min(3, g.n), min(25, g.n)} | ({g.n} if g.n <= 300 else set())):
        _note("topk %s k=%d" % (g.name, k))
        nodes, F = G.topk_closeness(k)
        nodes_ref, F_ref = oracle.topk_closeness(g, k)
        assert nodes.tolist() == nodes_ref.tolist() and F.tolist() == F_ref.tolist()
    for bad in (0, g.n + 1):
        with pytest.raises(gclib.GCError):
            G.topk_closeness(bad)
    assert G.closest_node() == (int(nodes_ref[0]), int(F_ref[0]))


@pytest.mark.parametrize("mk", SMALL, ids=lambda f: "small")
def test_greedy_small(gclib, mk):
    g = mk()
    k = min(g.n, 6)
    grp_ref, F_ref = oracle.greedy(g, k)
    G = _graph(gclib, g)
    for order in ("plain", "celf"):
        _note("greedy %s k=%d %s" % (g.name, k, order))
        grp, F, st = G.greedy_group(k, order=order)
        assert grp.tolist() == grp_ref.tolist()
        assert F.tolist() == F_ref.tolist()


def test_update_dist_and_gains_ba2000(gclib, device):
    g = graphgen.workload("ba2000")
    G = _graph(gclib, g)
    grp_ref, F_ref, gains_ref = oracle.greedy(g, 4, with_gains=True)
    dist = G.new_dist(1)
    far = torch.zeros(1, dtype=torch.int64, device=device)
    S = []
    for i, s in enumerate(grp_ref[:3]):
        _note("update_dist ba2000 pick %d" % i)
        G.update_dist(int(s), dist, 1, far)
        S.append(int(s))
        torch.cuda.synchronize()
        ref = oracle.group_dist(g, S)
        got = dist[: g.n].cpu().numpy().astype(np.int32)
        assert np.array_equal(got, ref)
        assert int(far.item()) == int(F_ref[i])
        _note("marginal_gains ba2000 round %d" % (i + 1))
        cand = torch.arange(g.n, dtype=torch.int32)
        gain, edges, vis = G.marginal_gains(dist, 1, cand, stats=True)
        gain = gain.cpu().numpy()
        exp = gains_ref[i].copy()
        exp[np.array(S)] = 0
        assert np.array_equal(gain, exp)
        # per-candidate work counters equal the oracle's pruned BFS
        dS = oracle.group_dist(g, S)
        gg, vv, ee = oracle.pruned_stats(g, dS, np.arange(g.n, dtype=np.int32))
        assert np.array_equal(gain, gg)
        assert np.array_equal(edges.cpu().numpy(), ee)
        assert np.array_equal(vis.cpu().numpy().astype(np.int64), vv)


def _expansions(g, dS, dv):
    """Per node w of the pruned BFS territory of v (d(v,w) < d(S,w)): the
    neighbours z that a BFS level can still claim from w, d(S,z) >= d(v,w) + 2
    (Section 4.1: a node is expanded only toward nodes it is closer to)."""
    rp, ci = g.row_ptr, g.col_idx
    src = np.repeat(np.arange(g.n), np.diff(rp))
    ok = dS[ci] >= dv[src] + 2
    return np.bincount(src[ok], minlength=g.n)


def test_word_counters_ba2000(gclib, device):
    """The engine's word-level counters.  One candidate per call: a frontier
    entry is a node of the territory with something to expand, and the
    adjacency entries expanded are exactly its neighbours that can still be
    claimed.  A launch over all candidates shares words between sources."""
    g = graphgen.workload("ba2000")
    G = _graph(gclib, g)
    s1 = int(oracle.greedy(g, 1)[0][0])
    dist = G.new_dist(1)
    far = torch.zeros(1, dtype=torch.int64, device=device)
    G.update_dist(s1, dist, 1, far)
    dS = oracle.group_dist(g, [s1]).astype(np.int64)
    rng = np.random.default_rng(4)
    _note("word counters, single candidates")
    for v in rng.choice(g.n, 12, replace=False).tolist() + [s1]:
        gain, edges, vis = G.marginal_gains(dist, 1, torch.tensor([v], dtype=torch.int32), stats=True)
        w = G.gain_words()
        gg, vv, ee = oracle.pruned_stats(g, dS, np.array([v], dtype=np.int32))
        assert int(vis.item()) == int(vv[0]) and int(edges.item()) == int(ee[0])
        dv = oracle.bfs(g, v).astype(np.int64)
        terr = dv < dS
        cnt = _expansions(g, dS, dv)
        assert w["entries"] == int(np.count_nonzero(terr & (cnt > 0)))
        assert w["edges"] + w["edges_last"] == int(cnt[terr].sum())
        assert w["entries_root"] == int(v != s1 and cnt[v] > 0)
        assert w["touched"] == int(vv[0])
    _note("word counters, one launch over all candidates")
    cand = torch.arange(g.n, dtype=torch.int32)
    gain, edges, vis = G.marginal_gains(dist, 1, cand, stats=True)
    w = G.gain_words()
    tv = int(vis.to(torch.int64).sum().item())
    te = int(edges.sum().item())
    roots = _expansions(g, dS, np.zeros(g.n, dtype=np.int64))
    assert w["entries_root"] == int(np.count_nonzero(roots[np.arange(g.n) != s1] > 0))
    assert tv >= w["entries"] >= w["entries_root"]
    assert tv >= w["touched"] >= -(-tv // 64)
    assert te >= w["edges"] + w["edges_last"]


def test_greedy_ba2000_k10(gclib):
    g = graphgen.workload("ba2000")
    grp_ref, F_ref = oracle.greedy(g, 10)
    G = _graph(gclib, g)
    for order in ("plain", "celf"):
        _note("greedy ba2000 k=10 %s" % order)
        grp, F, st = G.greedy_group(10, order=order)
        assert grp.tolist() == grp_ref.tolist()
        assert F.tolist() == F_ref.tolist()
        assert st["evals_round1"] == g.n - 1


@pytest.mark.parametrize("block", [64, 256])
def test_greedy_rmat16(gclib, block):
    g = graphgen.workload("rmat16")
    G = _graph(gclib, g)
    grp_b, F_b, ev_b, ed_b = oracle.greedypp(g, 50, block=block, growth=2)
    _note("greedy rmat16 k=50 plain block %d" % block)
    grp, F, st = G.greedy_group(50, order="plain", block=block, debug=True)
    assert grp.tolist() == grp_b.tolist()
    assert F.tolist() == F_b.tolist()
    # same scan order and batch schedule (the plain order doubles its block
    # per launch of a round): the same evaluations as the CPU Greedy++
    assert st["evals_per_round"].tolist() == ev_b.tolist()
    assert st["edges_alg"] == int(ed_b.sum())
    _note("greedy rmat16 k=50 plain fixed block %d" % block)
    _, _, ev_1, ed_1 = oracle.greedypp(g, 50, block=block, growth=1)
    grp1, F1, st1 = G.greedy_group(50, order="plain", block=block, block_growth=1)
    assert grp1.tolist() == grp_b.tolist() and F1.tolist() == F_b.tolist()
    assert st1["evals_per_round"].tolist() == ev_1.tolist()
    assert st1["edges_alg"] == int(ed_1.sum())
    # F(S) against the definition
    assert int(F[-1]) == oracle.farness(g, grp)
    _note("greedy rmat16 k=50 celf block %d" % block)
    grp_c, F_c, st_c = G.greedy_group(50, order="celf", block=block)
    assert grp_c.tolist() == grp_b.tolist() and F_c.tolist() == F_b.tolist()


@pytest.mark.parametrize("block", [255, 256, 257, 1024, 1025])
def test_greedy_launch_sizes(gclib, block):
    """Later-round launches of 255..1025 candidates: the roots and level 0
    of launches of at most 1024 candidates run as one kernel (ids as a kernel
    argument up to 256 of them, read from the candidate list beyond), larger
    ones as roots plus level kernels.  Picks, F(S_i), evaluations and the
    scanned adjacency entries equal the CPU Greedy++'s."""
    g = graphgen.ba(1100, 3, 17)
    G = _graph(gclib, g)
    grp_b, F_b, ev_b, ed_b = oracle.greedypp(g, 8, block=block, growth=1)
    _note("greedy ba1100 k=8 plain block %d" % block)
    grp, F, st = G.greedy_group(8, order="plain", block=block, block_growth=1, debug=True)
    assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
    assert st["evals_per_round"].tolist() == ev_b.tolist()
    assert st["edges_alg"] == int(ed_b.sum())


def test_greedy_fused_launch_overflow(gclib, monkeypatch):
    """Later-round launches of 1024 candidates on a 48x48 grid, whose
    frontier levels (about 11,000 entries over the 16 batches at the widest)
    overflow a ring of 4,096 entries: each launch is redone with fewer
    batches until it fits, the level-0 sums of the overflowed ones are
    dropped, and every result still equals the CPU Greedy++'s."""
    monkeypatch.setenv("GC_LOG_ENTRIES", "3000")
    g = graphgen.grid(48, 48, 5)
    G = _graph(gclib, g)
    grp_b, F_b, ev_b, ed_b = oracle.greedypp(g, 5, block=1024, growth=1)
    for order in ("plain", "celf"):
        _note("greedy grid48x48 k=5 %s block 1024, small ring" % order)
        grp, F, st = G.greedy_group(5, order=order, block=1024, block_growth=1, debug=True)
        assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
        if order == "plain":
            assert st["evals_per_round"].tolist() == ev_b.tolist()
            assert st["edges_alg"] == int(ed_b.sum())


def test_greedy_block_growth(gclib):
    """Every batch schedule gives the same group; the CELF order with a
    growing block matches the CPU Greedy++ picks; out-of-range factors are
    rejected before any work."""
    g = graphgen.ba(3000, 3, 41)
    G = _graph(gclib, g)
    grp_b, F_b, _, _ = oracle.greedypp(g, 15, block=16, growth=1)
    for order in ("plain", "celf"):
        for gr in (1, 3, 8):
            _note("greedy ba3000 k=15 %s block 16 growth %d" % (order, gr))
            grp, F, st = G.greedy_group(15, order=order, block=16, block_growth=gr)
            assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
            if order == "plain":
                _, _, ev, _ = oracle.greedypp(g, 15, block=16, growth=gr)
                assert st["evals_per_round"].tolist() == ev.tolist()
    for bad in (-1, 9):
        with pytest.raises(gclib.GCError):
            G.greedy_group(5, block_growth=bad)


ENGINE_ENVS = [{}, {"GC_VIS_BUDGET_MB": "1"}, {"GC_LOG_ENTRIES": "3000"}, {"GC_TOUCH_ENTRIES": "3000"},
               {"GC_BALLS": "0"}]


@pytest.mark.parametrize("env", ENGINE_ENVS,
                         ids=["default", "chunked", "log-overflow", "touch-overflow", "id-order"])
def test_engine_configurations(gclib, device, monkeypatch, env):
    """Launch chunking, overflow retries of the frontier ring and of the
    clean-up list and the source order all give the
    oracle's gains and greedy picks."""
    for key, v in env.items():
        monkeypatch.setenv(key, v)
    g = graphgen.rmat(12, 16, 7)
    G = _graph(gclib, g)
    grp_ref, F_ref, gains_ref = oracle.greedy(g, 4, with_gains=True)
    dist = G.new_dist(1)
    far = torch.zeros(1, dtype=torch.int64, device=device)
    S = []
    for i, s in enumerate(grp_ref[:3]):
        _note("engine %s update %d" % (env, i))
        G.update_dist(int(s), dist, 1, far)
        S.append(int(s))
        _note("engine %s gains round %d" % (env, i + 1))
        cand = torch.arange(g.n, dtype=torch.int32)
        gain = G.marginal_gains(dist, 1, cand).cpu().numpy()
        exp = gains_ref[i].copy()
        exp[np.array(S)] = 0
        assert np.array_equal(gain, exp)
    _note("engine %s greedy" % env)
    grp, F, st = G.greedy_group(4)
    assert grp.tolist() == grp_ref.tolist() and F.tolist() == F_ref.tolist()


def test_marginal_gains_u16_and_duplicates(gclib, device):
    """16-bit distances (eccentricity > 254), duplicate and member candidates."""
    g = graphgen.path(600)
    G = _graph(gclib, g)
    dist = G.new_dist(2)
    far = torch.zeros(1, dtype=torch.int64, device=device)
    S = [17, 444]
    for s in S:
        G.update_dist(s, dist, 2, far)
    torch.cuda.synchronize()
    assert np.array_equal(dist[: g.n].cpu().numpy().astype(np.int64) & 0xFFFF,
                          oracle.group_dist(g, S))
    assert int(far.item()) == oracle.farness(g, S)
    rng = np.random.default_rng(3)
    cand = np.concatenate([rng.integers(0, g.n, 150), [17, 17, 444, 5, 5, 5]]).astype(np.int32)
    _note("gains u16 path600")
    gain = G.marginal_gains(dist, 2, torch.from_numpy(cand)).cpu().numpy()
    dS = oracle.group_dist(g, S)
    assert np.array_equal(gain, oracle.gains(g, dS, cand))


def test_greedy_grid_u16(gclib):
    """High-diameter perturbed grid (16-bit distances when ecc > 254)."""
    g = graphgen.grid(900, 5, 9, shortcut_frac=0.0)
    G = _graph(gclib, g)
    grp_b, F_b, ev_b, ed_b = oracle.greedypp(g, 12, block=64, growth=2)
    for order in ("plain", "celf"):
        _note("greedy grid900x5 k=12 %s" % order)
        grp, F, st = G.greedy_group(12, order=order, debug=True)
        assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
        if order == "plain":
            assert st["evals_per_round"].tolist() == ev_b.tolist()
    assert st["dist_bytes"] == 2


@pytest.mark.parametrize("side", [64, 128])
def test_greedy_grid_square(gclib, side):
    g = graphgen.grid(side, side, 10 + side)
    G = _graph(gclib, g)
    grp_b, F_b, ev_b, ed_b = oracle.greedypp(g, 20, block=64, growth=2)
    _note("greedy grid%d k=20" % side)
    grp, F, st = G.greedy_group(20, debug=True)
    assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
    assert st["evals_per_round"].tolist() == ev_b.tolist()
    assert st["edges_alg"] == int(ed_b.sum())


def test_greedy_rmat20_k100_full_size(gclib):
    """R-MAT scale 20, k = 100: the whole group, every F(S_i) and the
    evaluation counts per round against the CPU Greedy++ at full size."""
    g = graphgen.workload("rmat20")
    G = _graph(gclib, g)
    _note("greedy rmat20 k=100 (GPU)")
    grp, F, st = G.greedy_group(100, order="plain")
    _note("greedy rmat20 k=100 (CPU oracle, tier B)")
    grp_b, F_b, ev_b, ed_b = oracle.greedypp(g, 100, block=64, growth=2)
    assert grp.tolist() == grp_b.tolist()
    assert F.tolist() == F_b.tolist()
    assert st["evals_per_round"].tolist() == ev_b.tolist()
    assert st["edges_alg"] == int(ed_b.sum())
    # F(S_k) from the definition, one BFS per member
    assert int(F[-1]) == oracle.farness(g, grp)
    # sampled gains of the second pick, one by one by full BFS
    dS = oracle.group_dist(g, grp[:1])
    rng = np.random.default_rng(5)
    cand = rng.choice(g.n, 40, replace=False).astype(np.int32)
    dist = G.new_dist(st["dist_bytes"])
    import torch
    far = torch.zeros(1, dtype=torch.int64, device=G.row_ptr.device)
    G.update_dist(int(grp[0]), dist, st["dist_bytes"], far)
    got = G.marginal_gains(dist, st["dist_bytes"], torch.from_numpy(cand)).cpu().numpy()
    assert np.array_equal(got, oracle.gains(g, dS, cand))


def test_batched_ba_sample(gclib):
    """The batched Barabasi-Albert workload (256 graphs, n in [1000, 50000],
    m in [2, 8], k in [5, 50], seeds from SplitMix64 of 3): the three smallest
    and the largest graph, each with its own k, give the CPU Greedy++ group,
    farness, evaluation counts and scanned edges; the smallest also matches the
    plain greedy of the definition."""
    params = graphgen.batch_ba_params(3, 256)
    order = sorted(range(len(params)), key=lambda i: params[i][1])
    for idx in order[:3] + order[-1:]:
        sg, n_g, m_g, k_g = params[idx]
        g = graphgen.ba(n_g, m_g, sg)
        G = _graph(gclib, g)
        grp_b, F_b, ev_b, ed_b = oracle.greedypp(g, k_g, block=64, growth=2)
        for ordr in ("plain", "celf"):
            _note("batched BA graph %d (n=%d m=%d) k=%d %s" % (idx, g.n, m_g, k_g, ordr))
            grp, F, st = G.greedy_group(k_g, order=ordr, block=64)
            assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
            if ordr == "plain":
                assert st["evals_per_round"].tolist() == ev_b.tolist()
                assert st["edges_alg"] == int(ed_b.sum())
        if idx == order[0]:
            grp_a, F_a = oracle.greedy(g, k_g)
            assert grp_b.tolist() == grp_a.tolist() and F_b.tolist() == F_a.tolist()


@pytest.mark.parametrize("workers", [1, 3])
def test_greedy_many_matches_single_jobs(gclib, workers):
    """gc_greedy_many: jobs of uneven size on several host threads and
    streams give each job the group, farness and evaluation counts it gets
    alone, and the CPU Greedy++ group."""
    specs = [(graphgen.ba(4000, 3, 51), 12), (graphgen.ba(700, 2, 52), 5),
             (graphgen.rmat(12, 16, 53), 20), (graphgen.ba(1500, 5, 54), 9),
             (graphgen.grid(30, 25, 55), 7)]
    Gs = [_graph(gclib, g) for g, _ in specs]
    ks = [k for _, k in specs]
    many = gclib.Many(Gs, workers=workers)
    from paper_1710_01144_amd import learned
    net = gclib.Mlp(learned.init_master(5))
    for order in ("plain", "celf", "learned"):
        _note("greedy_many %d workers, %s" % (workers, order))
        kw = {"mlp_params": net.block} if order == "learned" else {}
        groups, fars, stats = many.run(ks, order=order, **kw)
        for (g, k), G, grp, F, st in zip(specs, Gs, groups, fars, stats):
            grp1, F1, st1 = G.greedy_group(k, order=order, **kw)
            assert grp.tolist() == grp1.tolist() and F.tolist() == F1.tolist()
            assert st["evals_total"] == st1["evals_total"]
            if order == "plain":
                grp_b, F_b, ev_b, _ = oracle.greedypp(g, k, block=64, growth=2)
                assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
                assert st["evals_total"] == int(ev_b.sum())


def test_tuning_shapes_do_not_change_results(gclib):
    """Every launch shape (gc_set_tuning) and the autotuner's pick give the
    oracle's group, farness and evaluation counts; bad shapes are rejected."""
    from paper_1710_01144_amd import tune
    g = graphgen.rmat(12, 16, 7)
    G = _graph(gclib, g)
    k = 8
    grp_b, F_b, ev_b, _ = oracle.greedypp(g, k, block=64, growth=2)
    default = G.get_tuning()
    shapes = [dict(unroll=16, unroll_small=8), dict(min_edges=16, min_edges_small=16),
              dict(min_edges=1 << 20, min_edges_small=1 << 20, level_wgs_per_cu=1), dict(level_wgs_per_cu=16)]
    for shape in shapes:
        G.set_tuning(**dict(default, **shape))
        for order in ("plain", "celf"):
            _note("tuning %s %s" % (shape, order))
            grp, F, st = G.greedy_group(k, order=order)
            assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
            if order == "plain":
                assert st["evals_per_round"].tolist() == ev_b.tolist()
    G.set_tuning(**default)
    for bad in (dict(unroll=5), dict(unroll_small=16), dict(min_edges=8), dict(level_wgs_per_cu=0)):
        with pytest.raises(gclib.GCError):
            G.set_tuning(**bad)
    assert G.get_tuning() == default
    _note("autotune rmat12 k=%d" % k)
    out = tune.autotune(G, k, reps=1, grid={"unroll_small": (4, 8), "level_wgs_per_cu": (2, 4)})
    assert out["shape"] == G.get_tuning() and out["trials"] == 3
    grp, F, _ = G.greedy_group(k)
    assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()


def test_resumed_runs_continue_the_greedy(gclib):
    """A run resumed from a greedy prefix picks what the full run picks; from
    an arbitrary start set it continues the greedy from that set."""
    g = graphgen.ba(300, 2, 11)
    G = _graph(gclib, g)
    k = 8
    grp_ref, F_ref = oracle.greedy(g, k)
    for order in ("plain", "celf"):
        for m in (1, 3, 7):
            _note("resume %s m=%d" % (order, m))
            grp, F, _ = G.greedy_group(k, order=order, prefix=grp_ref[:m])
            assert grp.tolist() == grp_ref.tolist() and F.tolist() == F_ref.tolist()
    start = [5, 77]
    _note("resume from %s" % start)
    grp, F, _ = G.greedy_group(5, prefix=np.array(start, dtype=np.int32))
    S = list(start)
    while len(S) < 5:
        dS = oracle.group_dist(g, S)
        cand = np.array([v for v in range(g.n) if v not in S], dtype=np.int32)
        gains = oracle.gains(g, dS, cand)
        S.append(int(cand[np.lexsort((cand, -gains))[0]]))
    assert grp.tolist() == S
    assert F.tolist() == [oracle.farness(g, S[: i + 1]) for i in range(5)]


def test_repeated_runs_are_identical(gclib):
    """Repeated jobs give the same picks, evaluation counts and word-level
    work counters (the engine's results do not depend on claim races)."""
    g = graphgen.rmat(12, 16, 7)
    G = _graph(gclib, g)
    keys = ("evals_round1", "evals_later", "edges_alg", "entries_word", "edges_word", "touched_word",
            "gain_launches")
    for order in ("plain", "celf"):
        runs = []
        for rep in range(3):
            _note("repeat %s %d" % (order, rep))
            grp, F, st = G.greedy_group(10, order=order)
            runs.append((grp.tolist(), F.tolist(), st["evals_per_round"].tolist(),
                         tuple(int(st[k]) for k in keys)))
        assert runs[0] == runs[1] == runs[2]


def test_schedule_autotuner_keeps_the_picks(gclib):
    """The batch-schedule tuner times every (block, growth) of its grid on a
    3,000-node BA graph; every schedule gives the same group (checked inside),
    and the chosen one reproduces CPU Greedy++'s group and its evaluation
    counts under that schedule."""
    from paper_1710_01144_amd import tune
    g = graphgen.ba(3000, 3, 41)
    G = _graph(gclib, g)
    out = tune.autotune_schedule(G, 15, schedules=[(16, 1), (64, 2), (256, 8)], reps=1)
    grp, F, st = G.greedy_group(15, block=out["block"], block_growth=out["growth"])
    grp_b, F_b, ev_b, _ = oracle.greedypp(g, 15, block=out["block"], growth=out["growth"])
    assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
    assert st["evals_per_round"].tolist() == ev_b.tolist()


def _broom(path_len, hub_at, satellites, seed):
    """A path with a hub on it: `satellites` extra nodes joined to the hub, to
    their next satellite (a ring) and, every tenth, to a random one of the
    path's first 100 nodes, so the hub's row (more than 2048 entries) has
    neighbours nearer, as near and farther than the hub from a group, and the
    rest of the path stays a long tail."""
    rng = np.random.default_rng(seed)
    src = list(range(path_len - 1))
    dst = list(range(1, path_len))
    sat = np.arange(path_len, path_len + satellites)
    src += [hub_at] * satellites
    dst += sat.tolist()
    src += sat.tolist()
    dst += np.roll(sat, 1).tolist()
    tenth = sat[::10]
    src += tenth.tolist()
    dst += rng.integers(0, min(100, path_len), tenth.shape[0]).tolist()
    return graphgen.from_edges("broom%d_%d" % (path_len, satellites), path_len + satellites,
                               np.array(src), np.array(dst))


@pytest.mark.parametrize("path_len,dist_bytes", [(120, 1), (700, 2)])
def test_long_rows_split_by_chunks(gclib, device, path_len, dist_bytes):
    """Rows of more than 1024 entries are split by 2048-entry chunks: every
    gain, |V(v)| and adjacency count of a round matches the oracle with 8- and
    16-bit distances, and the greedy matches CPU Greedy++ round by round."""
    g = _broom(path_len, 40, 5000, 11)
    deg = np.diff(g.row_ptr)
    assert deg.max() > 2 * 2048
    G = _graph(gclib, g)
    dist = G.new_dist(dist_bytes)
    far = torch.zeros(1, dtype=torch.int64, device=device)
    S = [60, path_len - 1]
    for s in S:
        G.update_dist(s, dist, dist_bytes, far)
    torch.cuda.synchronize()
    dS = oracle.group_dist(g, S)
    assert int(dS.max()) > 254 if dist_bytes == 2 else int(dS.max()) <= 254
    cand = np.arange(g.n, dtype=np.int32)
    _note("gains broom%d (%d-byte distances)" % (path_len, dist_bytes))
    gain = G.marginal_gains(dist, dist_bytes, torch.from_numpy(cand)).cpu().numpy()
    assert np.array_equal(gain, oracle.gains(g, dS, cand))
    grp_b, F_b, ev_b, ed_b = oracle.greedypp(g, 8, block=64, growth=2)
    _note("greedy broom%d k=8" % path_len)
    grp, F, st = G.greedy_group(8, debug=True)
    assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
    assert st["evals_per_round"].tolist() == ev_b.tolist()
    assert st["edges_alg"] == int(ed_b.sum())
