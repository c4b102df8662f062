"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

The oracle cannot walk the scale-22/23 graphs in test time, so those are checked on
sampled outputs it computes one by one (per-edge local counts, per-edge gradients) and on
properties that hold at any size; the scale-20 counts are compared whole.

* R-MAT s20, P+ ~ Beta(2,2): exact counts at t in {0.5, 0.7, 0.9}, every method and the
  batched form, against the oracle's counts.
* R-MAT s23, bimodal P+: the pruned count at t = 0.8 equals a third of the sum of the
  per-edge local counts over all edges (each triangle has three edges); 2,000 sampled
  edges' local counts equal the oracle's.
* R-MAT s20, P+ ~ Beta(2,2), vertex sampling at the benchmark's thresholds: the local
  counts of all vertices sum to three times the exact counts; 8 worlds x 1,000 vertices
  replay the oracle's estimates exactly.
* R-MAT s20, P+ ~ Beta(2,2), sign worlds: 32 worlds equal the oracle's counts exactly;
  the mean of 1,024 worlds is within 4 standard errors of the exact expected count.
* R-MAT s22, P+ ~ U(0.05, 0.95): the gradient of 1,000 sampled edges (seed 3) equals the
  oracle's bit for bit and matches central finite differences at h = 1e-6 within 1e-6
  relative (local differences of the exact expected count: E is affine in each P+).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_14084_amd import inputs, utri

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def device_graph(n, lo, hi, p):
    d = torch.device("cuda")
    return utri.Graph(torch.from_numpy(lo).to(d), torch.from_numpy(hi).to(d),
                      torch.from_numpy(np.asarray(p, np.float64)).to(d), n)


def test_rmat_s20_counts_match_oracle():
    n, lo, hi = inputs.rmat_graph(20, seed=1)
    p = inputs.draw_p(lo.shape[0], "beta22", 2)
    say("rmat20 beta22 m_in", lo.shape[0])
    ts = [0.5, 0.7, 0.9]
    og = oracle.load(n, lo, hi, p)
    want = og.count_multi(ts)
    say("oracle", want.tolist())
    g = device_graph(n, lo, hi, p)
    for j, t in enumerate(ts):
        for method in (utri.UTRI_PLAIN, utri.UTRI_PRUNED, utri.UTRI_PRUNED_L3):
            assert g.count(t, method) == tuple(want[j]), (t, method)
    assert np.array_equal(g.count_batch(ts), want)


def test_rmat_s20_vertex_sampling():
    n, lo, hi = inputs.rmat_graph(20, seed=1)
    p = inputs.draw_p(lo.shape[0], "beta22", 2)
    say("rmat20 vertex sampling m_in", lo.shape[0])
    g = device_graph(n, lo, hi, p)
    ts = [0.5 + 0.0075 * j for j in range(0, 64, 9)]
    tot = np.zeros((len(ts), 2), np.int64)
    step = 1 << 18
    for v0 in range(0, n, step):
        vids = torch.arange(v0, min(n, v0 + step), dtype=torch.int64, device="cuda")
        tot += g.vertex_local(ts, vids).sum(dim=0).cpu().numpy()
    want = g.count_batch(ts)
    assert np.array_equal(tot, 3 * want), (tot, want)
    est = g.sample(ts, 1000, 8, 2026, utri.UTRI_SAMPLE_VERTEX).cpu().numpy()
    del g
    torch.cuda.empty_cache()
    say("oracle load")
    og = oracle.load(n, lo, hi, p)
    oest, _ = og.sample_vertices(ts, 1000, 8, 2026)
    assert np.array_equal(est, oest)


def test_rmat_s20_sign_worlds():
    n, lo, hi = inputs.rmat_graph(20, seed=1)
    p = inputs.draw_p(lo.shape[0], "beta22", 2)
    say("rmat20 sign worlds m_in", lo.shape[0])
    g = device_graph(n, lo, hi, p)
    E = g.expected()
    many = g.sign_worlds(1024, 7).cpu().numpy().astype(np.float64)
    assert abs(many.mean() - E) <= 4 * many.std(ddof=1) / np.sqrt(1024), (many.mean(), E)
    few = g.sign_worlds(32, 8).cpu().numpy()
    del g
    torch.cuda.empty_cache()
    say("oracle load")
    og = oracle.load(n, lo, hi, p)
    assert np.array_equal(few, og.sign_worlds(32, 8))


def test_rmat_s23_count_and_sampled_edge_locals():
    n, lo, hi = inputs.rmat_graph(23, seed=1)
    p = inputs.draw_p(lo.shape[0], "bimodal", 2)
    say("rmat23 bimodal m_in", lo.shape[0])
    g = device_graph(n, lo, hi, p)
    m = utri.utri_graph_info(g.handle)["m"]
    bal, unb = g.count(0.8, utri.UTRI_PRUNED)
    say("gpu count", bal, unb)
    # every triangle is counted once by the walk and once at each of its edges
    tot = np.zeros(2, np.int64)
    step = 1 << 24
    for e0 in range(0, m, step):
        eids = torch.arange(e0, min(m, e0 + step), dtype=torch.int64, device="cuda")
        tot += g.edge_local([0.8], eids).sum(dim=0).cpu().numpy().reshape(-1)
    assert tot[0] == 3 * bal and tot[1] == 3 * unb, (tot, bal, unb)
    eids = np.random.default_rng(7).integers(0, m, 2000)
    got = g.edge_local([0.8, 0.6], eids).cpu().numpy()
    del g
    torch.cuda.empty_cache()
    say("oracle load")
    og = oracle.load(n, lo, hi, p)
    assert np.array_equal(got, og.edge_local([0.8, 0.6], eids))


def test_rmat_s22_sampled_gradient_and_finite_differences():
    n, lo, hi = inputs.rmat_graph(22, seed=1)
    p = inputs.draw_p(lo.shape[0], "uniform_05_95", 2)
    say("rmat22 uniform_05_95 m_in", lo.shape[0])
    g = device_graph(n, lo, hi, p)
    grad = g.expected_grad().cpu().numpy()
    m = grad.shape[0]
    eids = np.random.default_rng(3).integers(0, m, 1000)
    del g
    torch.cuda.empty_cache()
    say("oracle load")
    og = oracle.load(n, lo, hi, p)
    want = og.grad(eids)
    assert np.array_equal(grad[eids], want)
    fd = og.local_central_difference(eids, 1e-6)
    scale = np.maximum(np.abs(want), 1e-300)
    rel = np.abs(grad[eids] - fd) / scale
    say("fd max rel", float(rel[np.abs(want) > 0].max(initial=0.0)))
    # edges in no triangle have gradient 0 and a zero difference
    assert np.all(fd[want == 0] == 0)
    assert np.all(rel[want != 0] <= 1e-6)
