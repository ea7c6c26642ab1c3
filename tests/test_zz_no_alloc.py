"""The allocation-free gain entry point (gc_marginal_gains_noalloc) against
gc_marginal_gains with a workspace, through the C ABI, on calls in a row
(the second on a smaller graph with fewer candidates), with uint8 and uint16
distances, plus the oracle's gains and the size limit."""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _dist_of(G, S, dist_bytes):
    dist = G.new_dist(dist_bytes)
    far = torch.zeros(1, dtype=torch.int64, device=G.row_ptr.device)
    for s in S:
        G.update_dist(int(s), dist, dist_bytes, far)
    return dist


def _check(gclib, device, g, seed, ncand, dist_bytes=1):
    print("no-alloc case: n=%d nnz=%d candidates=%d dist_bytes=%d seed=%d"
          % (g.n, g.nnz, ncand, dist_bytes, seed), flush=True)
    G = gclib.Graph.from_graphgen(g)
    rng = np.random.default_rng(seed)
    S = rng.choice(g.n, size=3, replace=False)
    dist = _dist_of(G, S, dist_bytes)
    cand_np = rng.integers(0, g.n, ncand).astype(np.int32)
    cand_np[:3] = S  # members of S get 0
    cand = torch.from_numpy(cand_np).to(device)
    ref_g, ref_e, ref_v = G.marginal_gains(dist, dist_bytes, cand, stats=True)
    gain = torch.full((ncand,), -7, dtype=torch.int64, device=device)
    edges = torch.full((ncand,), -7, dtype=torch.int64, device=device)
    vis = torch.full((ncand,), -7, dtype=torch.int32, device=device)
    G.marginal_gains_noalloc(dist, dist_bytes, cand, gain, edges, vis)
    torch.cuda.synchronize()
    assert torch.equal(gain, ref_g) and torch.equal(edges, ref_e) and torch.equal(vis, ref_v)
    exp = oracle.gains(g, oracle.group_dist(g, S.tolist()), cand_np)
    assert gain.cpu().numpy().tolist() == exp.tolist()
    # gains only (no statistics)
    gain2 = torch.full((ncand,), -7, dtype=torch.int64, device=device)
    G.marginal_gains_noalloc(dist, dist_bytes, cand, gain2)
    torch.cuda.synchronize()
    assert torch.equal(gain2, ref_g)


def test_noalloc_matches_workspace_entry_point(gclib, device):
    _check(gclib, device, graphgen.rmat(13, 16, 61), 1, 3000)
    _check(gclib, device, graphgen.ba(500, 3, 62), 2, 100)          # smaller, after a larger one
    _check(gclib, device, graphgen.path(600), 3, 50, dist_bytes=2)  # uint16 distances
    _check(gclib, device, graphgen.grid(40, 50, 63), 4, 2500)


def test_noalloc_refuses_graphs_beyond_its_scratch(gclib, device):
    import ctypes
    n = 9_000_000  # one batch of per-node records alone is 288 MB
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = 2
    rp[1] = 1
    rp[n] = 1
    rp = np.cumsum(rp).astype(np.int32)
    ci = np.empty(rp[-1], dtype=np.int32)
    idx = np.arange(n, dtype=np.int64)
    ci[rp[1:n - 1]] = idx[1:n - 1] - 1       # rows 1..n-2: left neighbour first,
    ci[rp[1:n - 1] + 1] = idx[1:n - 1] + 1   # then the right one (a path of n nodes)
    ci[0] = 1
    ci[rp[n - 1]] = n - 2
    G = gclib.Graph(rp, ci, workspace=False)
    lib = gclib.load_library()
    dist = torch.zeros(n, dtype=torch.uint8, device=device)
    cand = torch.zeros(1, dtype=torch.int32, device=device)
    gain = torch.full((1,), -7, dtype=torch.int64, device=device)
    rc = lib.gc_marginal_gains_noalloc(G.handle, ctypes.c_void_p(dist.data_ptr()), 1,
                                       ctypes.c_void_p(cand.data_ptr()), 1,
                                       ctypes.c_void_p(gain.data_ptr()), None, None,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == gclib.GC_EWORKSPACE
    assert b"bytes of scratch" in lib.gc_last_error()
    assert int(gain.item()) == -7
