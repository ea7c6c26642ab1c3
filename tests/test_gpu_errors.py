"""C-ABI error paths on the device: CSR contract violations found by the
validating load, and out-of-range arguments of the calls.  Every case is an
error code from the host side; no kernel runs on bad input."""
import numpy as np
import pytest
import torch

import graphgen

pytestmark = pytest.mark.gpu


def _csr(edges, n, sort=True):
    rows = [[] for _ in range(n)]
    for a, b in edges:
        rows[a].append(b)
    if sort:
        rows = [sorted(r) for r in rows]
    rp = np.zeros(n + 1, np.int32)
    for i in range(n):
        rp[i + 1] = rp[i] + len(rows[i])
    ci = np.array([x for r in rows for x in r], np.int32)
    return rp, ci


def _code(gclib, rp, ci):
    with pytest.raises(gclib.GCError) as e:
        gclib.Graph(rp, ci)
    return e.value.code


def test_load_rejects_bad_csr(gclib):
    sym = [(0, 1), (1, 0), (1, 2), (2, 1)]
    assert _code(gclib, *_csr(sym + [(2, 0)], 3)) == gclib.GC_ENOTSYM           # missing reverse edge
    assert _code(gclib, *_csr([(0, 1), (1, 0), (2, 3), (3, 2)], 4)) == gclib.GC_EDISCONNECTED
    assert _code(gclib, *_csr(sym + [(1, 1)], 3)) == gclib.GC_EINVAL            # self-loop
    rp, ci = _csr([(0, 1), (0, 1), (1, 0), (1, 0)], 2)
    assert _code(gclib, rp, ci) == gclib.GC_EINVAL                             # duplicate
    rp, ci = _csr([(0, 2), (0, 1), (1, 0), (2, 0)], 3, sort=False)
    assert _code(gclib, rp, ci) == gclib.GC_EINVAL                             # unsorted row
    rp, ci = _csr(sym, 3)
    bad = ci.copy()
    bad[0] = 7
    assert _code(gclib, rp, bad) == gclib.GC_EINVAL                            # id out of range
    rp2 = rp.copy()
    rp2[1], rp2[2] = rp2[2], rp2[1]
    assert _code(gclib, rp2, ci) == gclib.GC_EINVAL                            # decreasing row_ptr


def test_calls_reject_bad_arguments(gclib, device):
    g = graphgen.gnp_connected(40, 0.1, 3)
    G = gclib.Graph.from_graphgen(g)
    for k in (0, g.n + 1):
        with pytest.raises(gclib.GCError):
            G.greedy_group(k)
    dist = G.new_dist(1)
    far = torch.zeros(1, dtype=torch.int64, device=device)
    for node in (-1, g.n):
        with pytest.raises(gclib.GCError):
            G.update_dist(node, dist, 1, far)
    with pytest.raises(gclib.GCError):
        G.update_dist(0, dist, 3, far)
    with pytest.raises(gclib.GCError):
        G.greedy_group(5, order="learned")  # no network
    with pytest.raises(gclib.GCError):
        G.greedy_group(5, prefix=[3, 7, 3])  # a repeated id is not a group
    full = G.new_dist(1)
    G.update_dist(0, full, 1, far)
    for bad in ([-1, 2], [0, g.n]):
        with pytest.raises(ValueError):
            G.marginal_gains(full, 1, torch.tensor(bad, dtype=torch.int32))
    # the handle still works after the errors
    grp, F, _ = G.greedy_group(3)
    assert len(grp) == 3 and F[0] > F[1] > F[2]


@pytest.mark.gpu
def test_closeness_search_refuses_graphs_above_its_verified_size(gclib, device):
    """The closeness search (first pick) refuses graphs above 2^20 nodes or
    2^25 adjacency entries with GC_ERANGE, before touching the workspace."""
    import ctypes
    n = (1 << 20) + 1
    g = graphgen.path(n)
    G = gclib.Graph.from_graphgen(g, workspace=False)
    lib = gclib.load_library()
    dummy = torch.zeros(256, dtype=torch.uint8, device=device)
    node, far = ctypes.c_int32(-1), ctypes.c_int64(-1)
    rc = lib.gc_closest_node(G.handle, ctypes.c_void_p(dummy.data_ptr()), 256,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                             ctypes.byref(node), ctypes.byref(far))
    assert rc == -4 and node.value == -1 and far.value == -1
    assert "not supported" in lib.gc_last_error().decode()
    grp = (ctypes.c_int32 * 1)()
    fr = (ctypes.c_int64 * 1)()
    rc = lib.gc_greedy_group(G.handle, 1, None, ctypes.c_void_p(dummy.data_ptr()), 256,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), grp, fr, None)
    assert rc == -4


@pytest.mark.gpu
def test_workspace_too_small_and_allocation_failures(gclib, device, monkeypatch):
    """A workspace below gc_workspace_size gives GC_EWORKSPACE before any
    kernel runs; a failed pinned host allocation inside the greedy (injected
    with GC_TEST_FAIL_ALLOC) gives GC_ENOMEM; the handle keeps working after
    both."""
    import ctypes
    g = graphgen.ba(500, 3, 9)
    G = gclib.Graph.from_graphgen(g)
    lib = gclib.load_library()
    small = torch.zeros(G.ws_bytes // 2, dtype=torch.uint8, device=device)
    node, far = ctypes.c_int32(-1), ctypes.c_int64(-1)
    rc = lib.gc_closest_node(G.handle, ctypes.c_void_p(small.data_ptr()), small.numel(),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                             ctypes.byref(node), ctypes.byref(far))
    assert rc == gclib.GC_EWORKSPACE and node.value == -1
    assert b"workspace" in lib.gc_last_error()
    grp_ref, F_ref, _ = G.greedy_group(5)
    for at in (1, 2, 3):
        monkeypatch.setenv("GC_TEST_FAIL_ALLOC", str(at))
        with pytest.raises(gclib.GCError) as e:
            G.greedy_group(5)
        assert e.value.code == gclib.GC_ENOMEM
    monkeypatch.delenv("GC_TEST_FAIL_ALLOC")
    grp, F, _ = G.greedy_group(5)
    assert grp.tolist() == grp_ref.tolist() and F.tolist() == F_ref.tolist()


def test_level_watchdog(gclib, device, monkeypatch):
    """GC_LEVEL_CAP: a BFS that needs more levels fails the call with
    GC_EDEVICE (the kernels already launched end normally); graphs whose
    searches stay under the cap are not affected."""
    monkeypatch.setenv("GC_LEVEL_CAP", "10")
    P = gclib.Graph.from_graphgen(graphgen.path(300))
    for call in (P.closest_node, lambda: P.greedy_group(3, prefix=[150])):
        with pytest.raises(gclib.GCError) as ei:
            call()
        assert ei.value.code == gclib.GC_EDEVICE and "level cap" in str(ei.value)
        P.alloc_workspace()  # a failed call leaves the workspace to be prepared again
    far_t = torch.zeros(1, dtype=torch.int64, device=device)
    dist = P.new_dist(2)
    with pytest.raises(gclib.GCError) as ei:
        P.update_dist(0, dist, 2, far_t)
    assert ei.value.code == gclib.GC_EDEVICE
    g = graphgen.ba(2000, 4, 1)
    G = gclib.Graph.from_graphgen(g)
    grp, F, _ = G.greedy_group(10)
    monkeypatch.delenv("GC_LEVEL_CAP")
    G2 = gclib.Graph.from_graphgen(g)
    grp2, F2, _ = G2.greedy_group(10)
    assert grp.tolist() == grp2.tolist() and F.tolist() == F2.tolist()
    P2 = gclib.Graph.from_graphgen(graphgen.path(300))
    assert P2.closest_node() == (149, 2 * sum(range(1, 150)) + 150)


def test_round_watchdog_weighted(gclib, device, monkeypatch):
    """GC_ROUND_CAP: a weighted search that needs more near-list rounds is
    abandoned and the synchronising calls report GC_EDEVICE."""
    g = graphgen.with_weights(graphgen.path(200), 9, 3)
    monkeypatch.setenv("GC_ROUND_CAP", "3")
    P = gclib.Graph.from_graphgen(g)
    for call in (P.closest_node, lambda: P.topk_closeness(3), lambda: P.greedy_group(3)):
        with pytest.raises(gclib.GCError) as ei:
            call()
        assert ei.value.code == gclib.GC_EDEVICE and "round cap" in str(ei.value)
        P.alloc_workspace()
    monkeypatch.setenv("GC_ROUND_CAP", "100000")
    P2 = gclib.Graph.from_graphgen(g)
    monkeypatch.delenv("GC_ROUND_CAP")
    P3 = gclib.Graph.from_graphgen(g)
    assert P2.greedy_group(4)[0].tolist() == P3.greedy_group(4)[0].tolist()
