"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

Whole-graph results of the scale-20/22/23 workloads come from the CPU oracle through
tests/golden/fullsize.json (written by tests/golden/make_fullsize.py, oracle only); the
rest is checked on sampled outputs the oracle computes one by one and on properties that
hold at any size.

* R-MAT s23, bimodal P+ (the benchmark graph): counts at t in {0.5, 0.8, 0.9, 0.95} for
  every method and every walk order equal the oracle's whole-graph counts; the t = 0.8
  enumeration (3.3e9 triangles), unsorted and sorted, has the oracle's list sizes, its
  order-free digests and its hash-selected spot samples (about 1e5 triangles), and the
  sorted lists are lexicographic.
* R-MAT s22, P+ ~ U(0.05, 0.95): the expected balanced count equals the oracle's bit for
  bit.
* R-MAT s20, P+ ~ Beta(2,2), the batch at the benchmark's shape (64 thresholds, 1,024
  worlds x 10,000 draws, hipGraph replays): exact counts and the first 32 worlds'
  estimates equal the oracle's.

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
import functools
import gzip
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_2602_14084_amd import inputs, utri

pytestmark = pytest.mark.gpu

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(key):
    """Oracle results on the full-size workloads, written by tests/golden/make_fullsize.py
    (CPU oracle only)."""
    with open(os.path.join(GOLDEN_DIR, "fullsize.json")) as f:
        return json.load(f)[key]


@functools.lru_cache(maxsize=1)
def rmat23_inputs():
    n, lo, hi = inputs.rmat_graph(23, seed=1)
    p = inputs.draw_p(lo.shape[0], "bimodal", 2)
    return n, lo, hi, p


def hash_device_triples(tri, bits):
    """Order-free digest (sum, xor) and spot sample of a device int32 [k, 3] list, hashed
    by the oracle's hash_triples on the host in chunks."""
    chunk = 1 << 24
    starts = list(range(0, tri.shape[0], chunk))

    def one(i0):
        part = tri[i0:i0 + chunk].cpu().numpy()
        return oracle.hash_triples(part, bits)

    s = x = 0
    samples = []
    with ThreadPoolExecutor(8) as ex:
        for (sx, samp) in ex.map(one, starts):
            s = (s + int(sx[0])) % (1 << 64)
            x ^= int(sx[1])
            samples.append(samp)
    samp = np.concatenate(samples) if samples else np.zeros((0, 3), np.int32)
    samp = samp[np.lexsort((samp[:, 2], samp[:, 1], samp[:, 0]))]
    return (str(s), str(x)), samp


def lexsorted_on_device(tri):
    """True when the rows of a device int32 [k, 3] list ascend lexicographically."""
    chunk = 1 << 26
    for i0 in range(0, max(tri.shape[0] - 1, 0), chunk):
        a = tri[i0:i0 + chunk + 1]
        x, y = a[:-1].long(), a[1:].long()
        lt = (x[:, 0] < y[:, 0]) | ((x[:, 0] == y[:, 0]) & (
            (x[:, 1] < y[:, 1]) | ((x[:, 1] == y[:, 1]) & (x[:, 2] < y[:, 2]))))
        if not bool(lt.all()):
            return False
    return True


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


def test_rmat_s23_whole_graph_counts_match_oracle():
    """The headline workload whole: counts at four thresholds, every method and both walk
    orders, equal the oracle's counts over all of R-MAT s23."""
    G = golden("rmat_s23_bimodal")
    n, lo, hi, p = rmat23_inputs()
    say("rmat23 whole-graph counts m_in", lo.shape[0])
    g = device_graph(n, lo, hi, p)
    assert g.m == G["m"]
    ts = sorted(float(t) for t in G["counts"])
    want = np.array([G["counts"][str(t)] for t in ts], np.int64)
    for order in (utri.UTRI_ORDER_AUTO, utri.UTRI_ORDER_PLAIN, utri.UTRI_ORDER_SHORTER):
        utri.utri_set_walk_order(g.handle, order)
        for j, t in enumerate(ts):
            for method in (utri.UTRI_PLAIN, utri.UTRI_PRUNED, utri.UTRI_PRUNED_L3):
                got = g.count(t, method)
                say("order", order, "t", t, "method", method, got)
                assert got == tuple(want[j]), (order, t, method)
        assert np.array_equal(g.count_batch(ts), want)


def test_rmat_s23_enumeration_digest_matches_oracle():
    """The t = 0.8 enumeration of R-MAT s23 (3.3e9 triangles) against the oracle's: list
    sizes, the order-free digest of each list and its hash-selected spot sample; then the
    sorted form, which must be lexicographic with the same digests."""
    G = golden("rmat_s23_bimodal")["enumerate_t0.8"]
    bits = G["sample_bits"]
    with gzip.open(os.path.join(GOLDEN_DIR, "rmat_s23_t08_sample.txt.gz"), "rt") as f:
        rows = [ln.split() for ln in f if not ln.startswith("#")]
    want_s = {c: np.array([[int(a), int(b), int(d)] for k, a, b, d in rows if k == c],
                          np.int32).reshape(-1, 3) for c in "BU"}
    n, lo, hi, p = rmat23_inputs()
    g = device_graph(n, lo, hi, p)
    for sorted_ in (False, True):
        say("rmat23 enumerate t=0.8 sorted", sorted_)
        bal, unb = g.enumerate(0.8, utri.UTRI_PRUNED, sorted=sorted_)
        assert [bal.shape[0], unb.shape[0]] == G["counts"]
        for lst, key, c in ((bal, "digest_bal", "B"), (unb, "digest_unbal", "U")):
            if sorted_:
                assert lexsorted_on_device(lst), key
            dig, samp = hash_device_triples(lst, bits)
            say(key, dig, "sample", samp.shape[0])
            assert list(dig) == G[key], (sorted_, key)
            assert np.array_equal(samp, want_s[c]), (sorted_, key)
        del bal, unb
        torch.cuda.empty_cache()


def test_rmat_s23_count_and_sampled_edge_locals():
    n, lo, hi, p = rmat23_inputs()
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
    G = golden("rmat_s22_uniform_05_95")
    E = g.expected()
    say("rmat22 E", E.hex(), "oracle", G["expected"])
    assert E == float.fromhex(G["expected"])  # the whole-graph expected count, bit for bit
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


def test_rmat_s20_batch_at_benchmark_shape_replays_oracle():
    """The batch exactly as the benchmark runs it (R-MAT s20 Beta(2,2), 64 thresholds,
    1,024 worlds x 10,000 draws, seed 2026, hipGraph capture and replays): the exact counts
    equal the oracle's at all 64 thresholds and the first 32 worlds' estimates equal the
    oracle's replay bit for bit."""
    G = golden("rmat_s20_beta22_batch")
    n, lo, hi = inputs.rmat_graph(20, seed=1)
    p = inputs.draw_p(lo.shape[0], "beta22", 2)
    g = device_graph(n, lo, hi, p)
    ts, k, W = G["ts"], G["k"], G["worlds"]
    want_est = np.array([[[float.fromhex(x) for x in row] for row in w] for w in G["est"]])
    side = torch.cuda.Stream()
    ex = torch.empty((64, 2), dtype=torch.int64, device="cuda")
    es = torch.empty((1024, 64, 2), dtype=torch.float64, device="cuda")
    for rep in range(3):
        ex.fill_(-1)
        es.fill_(-1.0)
        say("rmat20 batch graph replay", rep)
        with torch.cuda.stream(side):
            g.batch(ts, k, 1024, G["seed"], use_graph=True, exact=ex, est=es)
        torch.cuda.synchronize()
        assert np.array_equal(ex.cpu().numpy(), np.array(G["exact"], np.int64)), rep
        assert np.array_equal(es[:W].cpu().numpy(), want_est), rep
        g.count(0.7)
