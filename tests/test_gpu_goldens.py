"""Large workloads against stored oracle results (tests/golden/*.json,
written by tests/golden/make_goldens.py from the CPU oracle alone; each
record names the sha256 of the CSR it was computed on)."""
import json
import os

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _gold(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.skip("%s not generated (tests/golden/make_goldens.py)" % name)
    with open(path) as f:
        return json.load(f)


def _note(msg):
    print("[gpu] " + msg, flush=True)


def test_batched_ba_all_graphs(gclib):
    """All 256 batched Barabasi-Albert graphs (each with its own k) through
    gc_greedy_many on 8 host threads: every group and F(S_1..S_k) equals CPU
    Greedy++ (tier B), the evaluations of each job equal tier B's under the
    same schedule, and the 64 graphs of fewest nodes equal the plain greedy of
    the definition (tier A); the CELF order gives the same groups."""
    gold_b = _gold("batchba_tierB.json")
    gold_a = {r["index"]: r for r in _gold("batchba_tierA64.json")["graphs"]}
    items = graphgen.batch_ba(3, 256)
    assert len(items) == len(gold_b["graphs"]) == 256
    for (g, k), r in zip(items, gold_b["graphs"]):
        assert g.sha256() == r["sha256"] and k == r["k"]
    Gs = [gclib.Graph.from_graphgen(g, workspace=False) for g, _ in items]
    many = gclib.Many(Gs, workers=8)
    ks = [k for _, k in items]
    _note("batched BA: 256 jobs, plain order")
    grps, fars, sts = many.run(ks, order="plain", block=64)
    for i, r in enumerate(gold_b["graphs"]):
        assert grps[i].tolist() == r["group"], i
        assert fars[i].tolist() == r["F"], i
        assert int(sts[i]["evals_total"]) == int(np.sum(r["evals"])), i
        if i in gold_a:
            assert r["group"] == gold_a[i]["group"] and r["F"] == gold_a[i]["F"], i
    assert len(gold_a) == 64
    _note("batched BA: 256 jobs, CELF order")
    grps, fars, _ = many.run(ks, order="celf", block=64)
    for i, r in enumerate(gold_b["graphs"]):
        assert grps[i].tolist() == r["group"] and fars[i].tolist() == r["F"], i


def test_batched_ba_lockstep(gclib):
    """All 256 batched graphs through gc_greedy_batch (later rounds in
    lockstep over the union of the graphs): every group, F and (plain) the
    evaluations of each job equal the stored tier-B run."""
    gold_b = _gold("batchba_tierB.json")
    items = graphgen.batch_ba(3, 256)
    Gs = [gclib.Graph.from_graphgen(g, workspace=False) for g, _ in items]
    many = gclib.Many(Gs, workers=8)
    ks = [k for _, k in items]
    for order in ("plain", "celf"):
        _note("batched BA: 256 jobs in lockstep, %s order" % order)
        grps, fars, sts = many.run(ks, order=order, block=64, lockstep=True)
        for i, r in enumerate(gold_b["graphs"]):
            assert grps[i].tolist() == r["group"] and fars[i].tolist() == r["F"], (order, i)
            if order == "plain":
                assert int(sts[i]["evals_total"]) == int(np.sum(r["evals"])), i


def test_rmat20_k100_against_stored_tier_b(gclib):
    """R-MAT scale 20, k = 100: plain and CELF groups, F and (plain) the
    evaluations of every round equal the stored tier-B run."""
    gold = _gold("rmat20_k100_tierB.json")
    g = graphgen.workload("rmat20")
    assert g.sha256() == gold["sha256"]
    G = gclib.Graph.from_graphgen(g)
    for order in ("plain", "celf"):
        _note("rmat20 k=100 %s" % order)
        grp, F, st = G.greedy_group(100, order=order, block=64)
        assert grp.tolist() == gold["group"] and F.tolist() == gold["F"], order
        if order == "plain":
            assert st["evals_per_round"].tolist() == gold["evals"]


def test_rmat16_k50_against_stored_tier_a(gclib):
    """R-MAT scale 16, k = 50: the group and F(S_1..S_50) of the plain greedy
    computed from the definition (tier A, a full BFS per candidate per
    round)."""
    gold = _gold("rmat16_k50_tierA.json")
    g = graphgen.workload("rmat16")
    assert g.sha256() == gold["sha256"]
    G = gclib.Graph.from_graphgen(g)
    for order in ("plain", "celf"):
        _note("rmat16 k=50 %s vs tier A" % order)
        grp, F, _ = G.greedy_group(50, order=order, block=64)
        assert grp.tolist() == gold["group"] and F.tolist() == gold["F"], order


@pytest.mark.parametrize("name,workload,k", [("rmat16w_k50_tierB.json", "rmat16", 50),
                                             ("grid256w_k50_tierB.json", "grid256", 50)])
def test_weighted_against_stored_tier_b(gclib, name, workload, k):
    """Weighted R-MAT scale 16 and 256 x 256 grid (lengths 1..255, seed 21),
    k = 50: plain and CELF groups, F and (plain) the evaluations of every
    round equal the stored tier-B run on Dijkstra."""
    gold = _gold(name)
    g = graphgen.with_weights(graphgen.workload(workload), 255, 21)
    assert g.sha256() == gold["sha256"]
    G = gclib.Graph.from_graphgen(g)
    for order in ("plain", "celf"):
        _note("%s weighted k=%d %s" % (workload, k, order))
        grp, F, st = G.greedy_group(k, order=order, block=64)
        assert grp.tolist() == gold["group"] and F.tolist() == gold["F"], order
        if order == "plain":
            assert st["evals_per_round"].tolist() == gold["evals"]


def test_grid1024_k100_against_stored_tier_b(gclib):
    """The perturbed 1024 x 1024 grid, k = 100 (a job of about 70 s): the
    plain group, F and the evaluations of every round equal the stored
    tier-B run."""
    gold = _gold("grid1024_k100_tierB.json")
    g = graphgen.workload("grid1024")
    assert g.sha256() == gold["sha256"]
    G = gclib.Graph.from_graphgen(g)
    _note("grid1024 k=100 plain")
    grp, F, st = G.greedy_group(100, order="plain", block=64)
    assert grp.tolist() == gold["group"] and F.tolist() == gold["F"]
    assert st["evals_per_round"].tolist() == gold["evals"]
