"""gc_greedy_batch: the jobs of gc_greedy_many with their later rounds in
lockstep over the disjoint union of the graphs (one gain call per step for
every job).  Picks, farness and plain-order evaluation counts must equal the
CPU oracle's for each job, whatever the mix of sizes, distance widths, k and
direction; unusable inputs are rejected."""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[case] " + msg, flush=True)


def _run(gclib, graphs, ks, order="plain", block=0, growth=0, workers=3):
    Gs = [gclib.Graph.from_graphgen(g, workspace=False) for g in graphs]
    many = gclib.Many(Gs, workers=workers)
    return many.run(ks, order=order, block=block, block_growth=growth, lockstep=True)


MIXES = {
    "tiny": ([lambda: graphgen.path(5), lambda: graphgen.cycle(6), lambda: graphgen.star(4),
              lambda: graphgen.complete(3)], [3, 6, 1, 2]),
    "mixed": ([lambda: graphgen.ba(300, 2, 1), lambda: graphgen.grid(17, 13, 2), lambda: graphgen.path(600),
               lambda: graphgen.gnp_connected(12, 0.3, 4), lambda: graphgen.ba(2000, 4, 1),
               lambda: graphgen.directed_cycle(40), lambda: graphgen.rmat_directed(9, 8, 3),
               lambda: graphgen.ba(50, 3, 9)], [7, 9, 5, 12, 10, 6, 8, 2]),
}


@pytest.mark.parametrize("mix", sorted(MIXES))
@pytest.mark.parametrize("order", ["plain", "celf"])
def test_batch_against_oracle(gclib, device, mix, order):
    mks, ks = MIXES[mix]
    graphs = [mk() for mk in mks]
    _note("batch %s %s: %s" % (mix, order, [g.n for g in graphs]))
    for block, growth in ((4, 2), (0, 0), (2, 1)):
        grps, fars, sts = _run(gclib, graphs, ks, order=order, block=block, growth=growth)
        for g, k, grp, F, st in zip(graphs, ks, grps, fars, sts):
            ga, Fa = oracle.greedy(g, k)
            assert grp.tolist() == ga.tolist() and F.tolist() == Fa.tolist(), (g.name, block, growth)
            if order == "plain":
                _, _, ev, ed = oracle.greedypp(g, k, block=block or 64, growth=growth or 2)
                assert int(st["evals_total"]) == int(ev.sum()), (g.name, block, growth)
                assert int(st["edges_alg"]) == int(ed.sum()), (g.name, block, growth)


def test_batch_equals_many(gclib, device):
    """The same jobs through gc_greedy_many and gc_greedy_batch: the same
    groups, farness and evaluation counts, on 1 and 4 workers."""
    graphs = [graphgen.ba(n, m, s) for n, m, s in ((3000, 2, 1), (1200, 5, 2), (800, 3, 3), (5000, 4, 4))]
    graphs.append(graphgen.rmat(12, 8, 5))
    ks = [20, 15, 40, 25, 30]
    Gs = [gclib.Graph.from_graphgen(g, workspace=False) for g in graphs]
    for workers in (1, 4):
        many = gclib.Many(Gs, workers=workers)
        g1, f1, s1 = many.run(ks, order="plain")
        g2, f2, s2 = many.run(ks, order="plain", lockstep=True)
        for a, b, fa, fb, sa, sb in zip(g1, g2, f1, f2, s1, s2):
            assert a.tolist() == b.tolist() and fa.tolist() == fb.tolist()
            assert sa["evals_total"] == sb["evals_total"] and sa["edges_alg"] == sb["edges_alg"]


def test_batch_rejects(gclib, device):
    lib = gclib.load_library()
    gw = graphgen.with_weights(graphgen.ba(100, 2, 1), 9, 1)
    Gs = [gclib.Graph.from_graphgen(graphgen.ba(100, 2, 1), workspace=False),
          gclib.Graph.from_graphgen(gw, workspace=False)]
    with pytest.raises(gclib.GCError) as ei:
        gclib.Many(Gs[1:], workers=1).run([3], lockstep=True)
    assert ei.value.code == gclib.GC_EINVAL
    many = gclib.Many(Gs[:1], workers=1)
    with pytest.raises(gclib.GCError) as ei:
        many.run([3], order="learned", lockstep=True)
    assert ei.value.code == gclib.GC_EINVAL
    # a union buffer below gc_batch_union_size
    import ctypes
    handles = (ctypes.c_void_p * 1)(Gs[0].handle)
    need = ctypes.c_size_t()
    gclib._check(lib.gc_batch_union_size(1, handles, 0, ctypes.byref(need)))
    small = torch.empty(need.value // 2, dtype=torch.uint8, device=device)
    karr = (ctypes.c_int32 * 1)(3)
    ws = (ctypes.c_void_p * 1)(many.ws[0].data_ptr())
    wsb = (ctypes.c_size_t * 1)(many.ws_bytes)
    st = (ctypes.c_void_p * 1)(many.streams[0].cuda_stream)
    grp = np.zeros(3, np.int32)
    far = np.zeros(3, np.int64)
    rc = lib.gc_greedy_batch(1, handles, karr, None, 1, ws, wsb, st, ctypes.c_void_p(small.data_ptr()),
                             small.numel(), grp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             far.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None)
    assert rc == gclib.GC_EWORKSPACE
