"""Seeded input generators: determinism and the input contract of Section 2
(connected, undirected, unweighted; stored as a simple symmetric CSR)."""
import numpy as np
import pytest

import graphgen


def _check_contract(g):
    n, rp, ci = g.n, g.row_ptr, g.col_idx
    assert rp.dtype == np.int32 and ci.dtype == np.int32
    assert rp[0] == 0 and rp[-1] == ci.shape[0]
    assert np.all(np.diff(rp) >= 0)
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(ci >= 0) and np.all(ci < n)
    assert not np.any(ci == rows), "self-loop"
    # strictly ascending inside each row (no duplicates)
    same_row = rows[1:] == rows[:-1]
    assert np.all(ci[1:][same_row] > ci[:-1][same_row])
    # symmetric
    fwd = rows.astype(np.int64) * n + ci
    bwd = ci.astype(np.int64) * n + rows
    assert np.array_equal(np.sort(fwd), np.sort(bwd))
    # connected (numpy BFS)
    seen = np.zeros(n, bool)
    seen[0] = True
    front = np.array([0])
    while front.size:
        nb = np.concatenate([ci[rp[x]:rp[x + 1]] for x in front]) if front.size else np.array([], int)
        nb = np.unique(nb)
        nb = nb[~seen[nb]]
        seen[nb] = True
        front = nb
    assert seen.all(), "disconnected"


@pytest.mark.parametrize("mk", [lambda: graphgen.ba(2000, 4, 1), lambda: graphgen.ba(500, 2, 9),
                                lambda: graphgen.rmat(10, 16, 3), lambda: graphgen.grid(30, 40, 4),
                                lambda: graphgen.gnp_connected(12, 0.3, 1)])
def test_contract_and_determinism(mk):
    a, b = mk(), mk()
    _check_contract(a)
    assert a.sha256() == b.sha256()


def test_ba_sizes():
    g = graphgen.ba(2000, 4, 1)
    assert g.n == 2000 and g.m == 10 + 4 * 1995  # K5 seed clique, then 4 edges per node
    assert graphgen.ba(2000, 4, 2).sha256() != g.sha256()


def test_grid_sizes():
    g = graphgen.grid(1024, 1024, 4)
    lattice = 2 * 1024 * 1023
    kept = lattice - round(0.05 * lattice) + round(0.001 * 1024 * 1024)
    assert g.m <= kept and g.n <= 1024 * 1024
    assert g.n > 1_000_000


def test_rmat_relabel_keeps_lcc():
    g = graphgen.rmat(12, 16, 2)
    _check_contract(g)
    assert np.all(np.diff(g.old_id) > 0)  # ascending relabel


def test_batch_params_ranges():
    ps = graphgen.batch_ba_params(3, 256)
    assert len(ps) == 256
    for (_, n, m, k) in ps:
        assert 1000 <= n <= 50000 and 2 <= m <= 8 and 5 <= k <= 50
