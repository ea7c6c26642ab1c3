"""GPU parity of the learned-order path: features, MLP forward, backward and
Adam against the float64 reference, and the learned order's effect on the
lazy loop (identical picks, fewer exact evaluations than the plain scan)."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[case] " + msg, flush=True)


def _rand_features(rng, n):
    X = np.stack([rng.uniform(0, 12, n), rng.uniform(0, 1, n), rng.uniform(0, 14, n),
                  rng.uniform(0, 16, n), rng.uniform(0, 6, n), rng.integers(0, 3, n),
                  rng.uniform(0, 1, n), rng.uniform(0, 3, n)], axis=1)
    return X.astype(np.float32)


def _bf16_ulp(x):
    return np.maximum(np.abs(x), 1e-30) * 2.0 ** -7


def test_mlp_forward_layerwise(gclib, device):
    rng = np.random.default_rng(1)
    p = M.init_params(11)
    p[M.OFF_B1:M.OFF_W2] = rng.normal(0, 0.2, M.H).astype(np.float32)
    X = _rand_features(rng, 3000)
    _note("mlp forward 3000 samples")
    net = gclib.Mlp(p)
    out, h1, h2 = net.forward(torch.from_numpy(X).to(device), activations=True)
    out, h1, h2 = (t.cpu().numpy().astype(np.float64) for t in (out, h1, h2))
    x, r1, _, _ = M.forward(p, X)
    # layer 1: identical up to a rare one-ulp bf16 flip (float32 vs float64 sums)
    d1 = np.abs(h1 - r1)
    assert np.all(d1 <= _bf16_ulp(r1) * 1.01 + 1e-30)
    assert np.mean(d1 > 0) < 1e-3
    # layer 2 from the GPU's layer 1, output from the GPU's layer 2
    _, _, r2, _ = M.forward(p, X, h1_in=h1)
    d2 = np.abs(h2 - r2)
    assert np.all(d2 <= _bf16_ulp(r2) * 1.01 + 1e-30)
    assert np.mean(d2 > 0) < 1e-3
    _, _, _, ro = M.forward(p, X, h1_in=h1, h2_in=h2)
    assert np.allclose(out, ro, rtol=1e-5, atol=1e-5)


def test_mlp_backward_and_adam(gclib, device):
    rng = np.random.default_rng(2)
    p = M.init_params(12)
    X = _rand_features(rng, 2048)
    y = rng.uniform(0, 10, 2048).astype(np.float32)
    net = gclib.Mlp(p)
    xd = torch.from_numpy(X).to(device)
    yd = torch.from_numpy(y).to(device)
    _note("mlp backward 2048 samples")
    out, h1, h2 = net.forward(xd, activations=True)
    g = net.backward(xd, h1, h2, out, yd).cpu().numpy().astype(np.float64)
    x = M.bf16(X)
    gr = M.backward(p, x, h1.cpu().numpy().astype(np.float64), h2.cpu().numpy().astype(np.float64),
                    out.cpu().numpy().astype(np.float64), y)
    for lo, hi in [(M.OFF_W1, M.OFF_B1), (M.OFF_B1, M.OFF_W2), (M.OFF_W2, M.OFF_B2),
                   (M.OFF_B2, M.OFF_W3), (M.OFF_W3, M.OFF_B3), (M.OFF_B3, M.NPARAM)]:
        err = np.linalg.norm(g[lo:hi] - gr[lo:hi]) / max(np.linalg.norm(gr[lo:hi]), 1e-30)
        assert err <= 1e-4, (lo, hi, err)
    _note("mlp adam step")
    w0 = net.master.cpu().numpy().astype(np.float64)
    net.adam(torch.from_numpy(g.astype(np.float32)).to(device), lr=1e-3)
    w1_ref, m1, v1 = M.adam(w0, np.zeros_like(w0), np.zeros_like(w0), g.astype(np.float32), 1)
    assert np.allclose(net.master.cpu().numpy(), w1_ref, rtol=1e-6, atol=1e-7)
    assert np.allclose(net.m.cpu().numpy(), m1, rtol=1e-6, atol=1e-10)


def test_node_features(gclib, device):
    g = graphgen.ba(500, 3, 5)
    G = gclib.Graph.from_graphgen(g)
    rng = np.random.default_rng(3)
    S = [int(v) for v in rng.choice(g.n, 4, replace=False)]
    dS = oracle.group_dist(g, S)
    dist = torch.from_numpy(np.pad(dS.astype(np.uint8), (0, 4))).to(device)
    ub = rng.integers(0, 5000, g.n).astype(np.int64)
    le = rng.integers(-1, 3, g.n).astype(np.int32)
    dat = (dS + rng.integers(0, 2, g.n)).astype(np.uint16)
    _note("features ba500")
    F = G.node_features(dist, 1, torch.from_numpy(ub).to(device), torch.from_numpy(le).to(device),
                        torch.from_numpy(dat).to(device), 4, 10, int(dS.max())).cpu().numpy()
    Fr = M.features(g.row_ptr, g.col_idx, dS, ub, le, dat, 4, 10, int(dS.max()))
    assert np.allclose(F, Fr, rtol=2e-6, atol=2e-6)


def test_learned_order_picks_and_evaluations(gclib, device, monkeypatch):
    """Train on gains logged from plain runs of the BA-2000 and R-MAT-16
    workloads; on held-out graphs the learned order gives the plain picks
    with fewer exact evaluations in rounds >= 2 (an untrained network still
    gives the plain picks).  The network ranking a wide pool (16 blocks of the
    largest bounds, GC_LEARNED_POOL_PCT=1600) also keeps the picks; its
    evaluation counts against the untrained network and CELF are printed (the
    trained network does not beat either: a measured negative result)."""
    from paper_1710_01144_amd import learned
    train_runs = [(gclib.Graph.from_graphgen(graphgen.workload("ba2000")), 10),
                  (gclib.Graph.from_graphgen(graphgen.workload("rmat16")), 10),
                  (gclib.Graph.from_graphgen(graphgen.workload("rmat16")), 50)]
    _note("collect training data")
    X, Y = learned.collect(train_runs)
    assert X.shape[0] > 5000 and np.all(np.isfinite(X))
    _note("train %d samples" % X.shape[0])
    net, losses = learned.train(X, Y, steps=800)
    assert losses[-1] < 0.5 * losses[0], losses
    untrained = gclib.Mlp(learned.init_master(99))
    for g, k in [(graphgen.rmat(14, 16, 21), 30), (graphgen.ba(6000, 3, 22), 30)]:
        G = gclib.Graph.from_graphgen(g)
        _note("held-out %s k=%d" % (g.name, k))
        gp, Fp, sp = G.greedy_group(k, order="plain")
        gl, Fl, sl = G.greedy_group(k, order="learned", mlp_params=net.block)
        gu, Fu, su = G.greedy_group(k, order="learned", mlp_params=untrained.block)
        assert gl.tolist() == gp.tolist() and Fl.tolist() == Fp.tolist()
        assert gu.tolist() == gp.tolist() and Fu.tolist() == Fp.tolist()
        assert sl["evals_later"] < sp["evals_later"], (sl["evals_later"], sp["evals_later"])
        print("evals later: plain %d learned %d untrained %d" %
              (sp["evals_later"], sl["evals_later"], su["evals_later"]), flush=True)
        monkeypatch.setenv("GC_LEARNED_POOL_PCT", "1600")
        Gw = gclib.Graph.from_graphgen(g)
        monkeypatch.delenv("GC_LEARNED_POOL_PCT")
        _note("held-out %s k=%d, wide pool" % (g.name, k))
        gl, Fl, slw = Gw.greedy_group(k, order="learned", mlp_params=net.block)
        gu, Fu, suw = Gw.greedy_group(k, order="learned", mlp_params=untrained.block)
        gc_, Fc, sc = Gw.greedy_group(k, order="celf")
        assert gl.tolist() == gp.tolist() and gu.tolist() == gp.tolist() and gc_.tolist() == gp.tolist()
        print("wide pool, evals later: learned %d untrained %d celf %d" %
              (slw["evals_later"], suw["evals_later"], sc["evals_later"]), flush=True)



def test_learned_device_first_block_matches_host_ranking(gclib, device):
    """The first block of each learned round is chosen on the device (top-k of
    the scored pool, launched behind the update); with logging on it is ranked
    on the host instead.  Both must evaluate the same candidates: the same
    evaluation counts in every round and the same picks."""
    from paper_1710_01144_amd import learned
    net = gclib.Mlp(learned.init_master(17))
    for g, k in [(graphgen.rmat(13, 16, 31), 25), (graphgen.ba(5000, 3, 32), 20)]:
        G = gclib.Graph.from_graphgen(g)
        _note("learned first block, device vs host, %s k=%d" % (g.name, k))
        gd, Fd, sd = G.greedy_group(k, order="learned", mlp_params=net.block)
        gh, Fh, sh = G.greedy_group(k, order="learned", mlp_params=net.block, log_capacity=1 << 16)
        assert gd.tolist() == gh.tolist() and Fd.tolist() == Fh.tolist()
        assert sd["evals_per_round"].tolist() == sh["evals_per_round"].tolist()
        assert sd["gain_launches"] == sh["gain_launches"]
