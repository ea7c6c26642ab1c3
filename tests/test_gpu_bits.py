"""Bit-vector gains (Section 4.3) through the C ABI against the oracle:
every stored row is the ball of its node (popcount and bits from BFS
distances), the fixed point comes at the diameter, and the gains equal
the pruned-BFS definition for S = {} and for greedy prefixes."""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu

GRAPHS = [
    lambda: graphgen.path(7),
    lambda: graphgen.cycle(9),
    lambda: graphgen.star(12),
    lambda: graphgen.complete_bipartite(3, 5),
    lambda: graphgen.gnp_connected(40, 0.08, 6),
    lambda: graphgen.ba(300, 2, 11),
    lambda: graphgen.grid(17, 13, 3),
    lambda: graphgen.rmat(12, 16, 7),
]


def _note(msg):
    print("[case] " + msg, flush=True)


@pytest.mark.parametrize("mk", GRAPHS, ids=lambda f: "bits")
def test_bits_rows_and_gains(gclib, device, mk):
    g = mk()
    _note("bits load %s n=%d" % (g.name, g.n))
    G = gclib.Graph.from_graphgen(g)
    D = np.stack([oracle.bfs(g, u) for u in range(g.n)]) if g.n <= 400 else None
    grp, _ = oracle.greedy(g, min(3, g.n))
    ecc = max(int(oracle.bfs(g, int(u)).max()) for u in range(g.n)) if D is None else int(D.max())
    levels = G.bits_prepare(min(256, ecc + 3))
    assert levels == ecc + 1
    if D is not None:
        W = (g.n + 63) // 64
        rows = G.bits[: levels * g.n * W * 8].view(torch.int64).cpu().numpy().view(np.uint64)
        rows = rows.reshape(levels, g.n, W)
        bits = np.unpackbits(rows.view(np.uint8), axis=2, bitorder="little")[:, :, : g.n]
        for i in range(levels):
            assert np.array_equal(bits[i].astype(bool), D <= i), "level %d" % i
    dist = G.new_dist(1)
    far = torch.zeros(1, dtype=torch.int64, device=device)
    cand = torch.arange(g.n, dtype=torch.int32)
    S = []
    for step in range(len(grp) + 1):
        _note("bits gains %s |S|=%d" % (g.name, len(S)))
        gain = G.bits_gains(dist, 1, cand).cpu().numpy()
        if S:
            dS = oracle.group_dist(g, S)
            exp = oracle.gains(g, dS, cand.numpy())
        else:
            # S = {}: d(S,.) is INF = 255 everywhere, gain = sum_w (255 - d(v,w))
            exp = np.array([int((255 - oracle.bfs(g, v)).sum()) for v in range(g.n)])
        assert np.array_equal(gain, exp)
        if step < len(grp):
            G.update_dist(int(grp[step]), dist, 1, far)
            S.append(int(grp[step]))
    with pytest.raises(gclib.GCError):
        G.bits_gains(G.new_dist(2), 2, cand)


@pytest.mark.parametrize("mk", GRAPHS + [lambda: graphgen.ba(2000, 4, 1)], ids=lambda f: "bitgreedy")
def test_bitgreedy_matches_greedy(gclib, mk):
    """bitGreedy++ (the lazy loop over bit-vector gains) picks the plain
    greedy's group and evaluates exactly what CPU Greedy++ evaluates."""
    g = mk()
    k = min(g.n, 8)
    G = gclib.Graph.from_graphgen(g)
    G.bits_prepare(256)
    grp_a, F_a = oracle.greedy(g, k)
    grp_b, F_b, ev_b, _ = oracle.greedypp(g, k, block=64, growth=2)
    for order in ("plain", "celf"):
        _note("bitgreedy %s k=%d %s" % (g.name, k, order))
        grp, F, st = G.greedy_group(k, order=order, bits=True)
        assert grp.tolist() == grp_a.tolist() and F.tolist() == F_a.tolist()
        if order == "plain":
            assert st["evals_per_round"].tolist() == ev_b.tolist()
    with pytest.raises(gclib.GCError):
        G.greedy_group(k, order="learned", bits=True, mlp_params=torch.zeros(1, device=G.row_ptr.device))


def test_bitgreedy_rmat16(gclib):
    """The bench's graph: R-MAT scale 16, k = 50, against CPU Greedy++."""
    g = graphgen.workload("rmat16")
    G = gclib.Graph.from_graphgen(g)
    _note("bitgreedy rmat16 prepare")
    levels = G.bits_prepare(32)
    grp_b, F_b, ev_b, _ = oracle.greedypp(g, 50, block=64, growth=2)
    _note("bitgreedy rmat16 k=50 (%d levels)" % levels)
    grp, F, st = G.greedy_group(50, bits=True)
    assert grp.tolist() == grp_b.tolist() and F.tolist() == F_b.tolist()
    assert st["evals_per_round"].tolist() == ev_b.tolist()


def test_bits_errors(gclib, device):
    """Too few levels for the fixed point, a bad level count and bitGreedy++
    without rows are errors; after them the rows and bitGreedy++ still work."""
    G = gclib.Graph.from_graphgen(graphgen.path(9))  # diameter 8: 9 levels and one to confirm
    with pytest.raises(gclib.GCError):
        G.bits_prepare(5)
    with pytest.raises(gclib.GCError):
        G.bits_prepare(1)
    assert G.bits_prepare(10) == 9
    G2 = gclib.Graph.from_graphgen(graphgen.path(300))  # eccentricity > 254: uint16 distances
    with pytest.raises(ValueError):
        G2.greedy_group(3, bits=True)
    grp, F = oracle.greedy(graphgen.path(9), 3)
    g3, F3, _ = G.greedy_group(3, bits=True)
    assert g3.tolist() == grp.tolist() and F3.tolist() == F.tolist()
