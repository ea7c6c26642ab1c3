"""Writes the stored expected values of the large-workload GPU tests.

    python tests/golden/make_goldens.py [batchba] [rmat20] [rmat16a] [grid1024] [rmat16w] [grid256w]

Only the CPU oracle (oracle/) and the seeded generators (graphgen/) are
called; nothing here touches the GPU library.  Each record carries the sha256
of the CSR it was computed on, so a test can check that it compares the
same graph.

  batchba_tierB.json   all 256 batched Barabasi-Albert graphs: tier B
                       (CPU Greedy++) group, F(S_1..S_k) and evaluations per
                       round with batches of 64 doubling per batch of a round
                       (the library's default schedule)
  batchba_tierA64.json the 64 graphs of fewest nodes: tier A (plain greedy
                       from the definition) group and F
  rmat20_k100_tierB.json  R-MAT scale 20, k = 100: tier B as above
  rmat16_k50_tierA.json   R-MAT scale 16, k = 50: tier A
  grid1024_k100_tierB.json  the perturbed 1024 x 1024 grid, k = 100: tier B
  rmat16w_k50_tierB.json    R-MAT scale 16 with edge lengths 1..255 (seed 21),
                            k = 50: tier B on Dijkstra (weighted oracle)
  grid256w_k50_tierB.json   the perturbed 256 x 256 grid with lengths 1..255
                            (seed 21), k = 50: tier B on Dijkstra
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402


def _tier_b(g, k):
    grp, F, ev, _ = oracle.greedypp(g, k, block=64, growth=2)
    return {"group": grp.tolist(), "F": F.tolist(), "evals": ev.tolist()}


def _tier_a(g, k):
    grp, F = oracle.greedy(g, k)
    return {"group": grp.tolist(), "F": F.tolist()}


def _write(name, rec):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(rec, f, separators=(",", ":"))
        f.write("\n")
    print("wrote", path, flush=True)


def batchba():
    items = graphgen.batch_ba(3, 256)
    t0 = time.time()
    recs = []
    for i, (g, k) in enumerate(items):
        r = {"index": i, "n": g.n, "nnz": g.nnz, "k": k, "sha256": g.sha256()}
        r.update(_tier_b(g, k))
        recs.append(r)
    _write("batchba_tierB.json", {"workload": "batched BA, master seed 3", "tier": "B",
                                  "block": 64, "growth": 2, "graphs": recs})
    print("tier B, 256 graphs: %.1f s" % (time.time() - t0), flush=True)
    small = sorted(range(len(items)), key=lambda i: (items[i][0].n, i))[:64]
    t0 = time.time()
    recs = []
    for i in small:
        g, k = items[i]
        r = {"index": i, "n": g.n, "nnz": g.nnz, "k": k, "sha256": g.sha256()}
        r.update(_tier_a(g, k))
        recs.append(r)
    _write("batchba_tierA64.json", {"workload": "batched BA, master seed 3, 64 graphs of fewest nodes",
                                    "tier": "A", "graphs": recs})
    print("tier A, 64 graphs: %.1f s" % (time.time() - t0), flush=True)


def rmat20():
    g = graphgen.workload("rmat20")
    t0 = time.time()
    r = {"workload": "rmat20", "n": g.n, "nnz": g.nnz, "k": 100, "sha256": g.sha256(), "tier": "B",
         "block": 64, "growth": 2}
    r.update(_tier_b(g, 100))
    _write("rmat20_k100_tierB.json", r)
    print("rmat20 tier B: %.1f s" % (time.time() - t0), flush=True)


def grid1024():
    g = graphgen.workload("grid1024")
    t0 = time.time()
    r = {"workload": "grid1024", "n": g.n, "nnz": g.nnz, "k": 100, "sha256": g.sha256(), "tier": "B",
         "block": 64, "growth": 2}
    r.update(_tier_b(g, 100))
    _write("grid1024_k100_tierB.json", r)
    print("grid1024 tier B: %.1f s" % (time.time() - t0), flush=True)


def rmat16a():
    g = graphgen.workload("rmat16")
    t0 = time.time()
    r = {"workload": "rmat16", "n": g.n, "nnz": g.nnz, "k": 50, "sha256": g.sha256(), "tier": "A"}
    r.update(_tier_a(g, 50))
    _write("rmat16_k50_tierA.json", r)
    print("rmat16 tier A: %.1f s" % (time.time() - t0), flush=True)


def _weighted(workload, k, fname):
    g = graphgen.with_weights(graphgen.workload(workload), 255, 21)
    t0 = time.time()
    r = {"workload": workload + ", lengths 1..255 seed 21", "n": g.n, "nnz": g.nnz, "k": k,
         "sha256": g.sha256(), "tier": "B", "block": 64, "growth": 2}
    r.update(_tier_b(g, k))
    r["oracle_s"] = round(time.time() - t0, 1)
    _write(fname, r)
    print("%s tier B: %.1f s" % (fname, time.time() - t0), flush=True)


def rmat16w():
    _weighted("rmat16", 50, "rmat16w_k50_tierB.json")


def grid256w():
    _weighted("grid256", 50, "grid256w_k50_tierB.json")


if __name__ == "__main__":
    todo = sys.argv[1:] or ["batchba", "rmat20", "rmat16a", "grid1024", "rmat16w", "grid256w"]
    for name in todo:
        {"batchba": batchba, "rmat20": rmat20, "rmat16a": rmat16a, "grid1024": grid1024,
         "rmat16w": rmat16w, "grid256w": grid256w}[name]()
