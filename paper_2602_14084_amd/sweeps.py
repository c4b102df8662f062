"""Experiment sweeps of the paper's Section 7 on the synthetic stand-in graphs (needs a GPU).

* Exact counting, baseline against improved, and runtime as t grows (the "exact runtime"
  and "runtime as t increases" figures): R-MAT s20 with P+ ~ Beta(2,2) and R-MAT s23 with
  the bimodal P+, t = 0.50, 0.55, ..., 1.00; UTRI_PLAIN is the baseline (every triangle
  classified), UTRI_PRUNED adds Lemma 2, UTRI_PRUNED_L3 Lemmas 2 and 3.
* The five P+ distributions on one fixed graph (the "edge sign distributions" figure):
  R-MAT s20 re-weighted with Uniform, Normal(0.5, 0.15) clipped to [0, 1], Beta(0.5, 0.5),
  Beta(3, 1) and Beta(1, 3); improved runtime as t grows. The paper does not give the
  Normal's parameters; these are the generator's.
* Sampling queries per second as t grows (the "queries per second" figures): edge and
  vertex sampling with 1,024 independent runs of 10,000 (edge) / 1,000 (vertex) draws,
  with the improved local search and with the baseline one (eBase / vBase: no Lemma 2).
* MAPE against the exact count as the number of samples grows, t = 0.8, averaged over 100
  runs (the "MAPE" figure): edge and vertex sampling, k = 10^2 ... 10^5.

    python -m paper_2602_14084_amd.sweeps [--quick] [--out sweeps.json]

--quick runs every sweep on small graphs (R-MAT s12 / s13) in a few seconds.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import inputs, utri

TS = [round(0.5 + 0.05 * j, 2) for j in range(11)]
DISTS = ["uniform", "normal", "beta0505", "beta31", "beta13"]


def _ms(torch, fn, reps=3):
    """Median wall time of fn() in ms, the device synchronised around each call."""
    out = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t) * 1e3)
    return float(np.median(out))


def _graph(torch, n, lo, hi, p):
    d = torch.device("cuda")
    return utri.Graph(torch.from_numpy(lo).to(d), torch.from_numpy(hi).to(d),
                      torch.from_numpy(np.asarray(p, np.float64)).to(d), n)


def exact_vs_t(torch, g, ts):
    rows = []
    for t in ts:
        r = {"t": t}
        for name, method in (("plain", utri.UTRI_PLAIN), ("pruned", utri.UTRI_PRUNED),
                             ("pruned_l3", utri.UTRI_PRUNED_L3)):
            g.count(t, method)
            r[name + "_ms"] = _ms(torch, lambda: g.count(t, method))
        r["counts"] = list(g.count(t, utri.UTRI_PRUNED))
        rows.append(r)
    return rows


def distributions(torch, n, lo, hi, ts):
    g = None
    out = {}
    for dist in DISTS:
        p = inputs.draw_p(lo.shape[0], dist, 2)
        if g is None:
            g = _graph(torch, n, lo, hi, p)
        else:
            g.set_p(torch.from_numpy(p).to("cuda"))
        rows = []
        for t in ts:
            g.count(t, utri.UTRI_PRUNED)
            rows.append({"t": t, "pruned_ms": _ms(torch, lambda: g.count(t, utri.UTRI_PRUNED)),
                         "counts": list(g.count(t, utri.UTRI_PRUNED))})
        out[dist] = rows
    return out


def sampling_qps(torch, g, ts, worlds, k_edge, k_vertex):
    rows = []
    for t in ts:
        r = {"t": t}
        for name, scheme, k in (("edge", utri.UTRI_SAMPLE_EDGE, k_edge),
                                ("vertex", utri.UTRI_SAMPLE_VERTEX, k_vertex),
                                ("edge_base", utri.UTRI_SAMPLE_EDGE_PLAIN, k_edge),
                                ("vertex_base", utri.UTRI_SAMPLE_VERTEX_PLAIN, k_vertex)):
            g.sample([t], k, worlds, 11, scheme)
            ms = _ms(torch, lambda: g.sample([t], k, worlds, 11, scheme))
            r[name + "_ms"] = ms
            r[name + "_queries_per_s"] = worlds * k / (ms / 1e3)
        rows.append(r)
    return rows


def mape_vs_k(torch, g, t, runs, ks):
    exact = np.array(g.count(t, utri.UTRI_PRUNED), np.float64)
    out = {"t": t, "runs": runs, "exact": exact.tolist(), "edge": [], "vertex": []}
    for name, scheme in (("edge", utri.UTRI_SAMPLE_EDGE), ("vertex", utri.UTRI_SAMPLE_VERTEX)):
        for k in ks:
            est = g.sample([t], k, runs, 2026, scheme).cpu().numpy()[:, 0, :]
            mape = [float(np.mean(np.abs(est[:, c] - exact[c]) / exact[c])) if exact[c] > 0
                    else None for c in range(2)]
            out[name].append({"k": k, "mape_balanced": mape[0], "mape_unbalanced": mape[1]})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available(), "the sweeps need a GPU"
    res = {"thresholds": TS}
    big, small = (13, 12) if args.quick else (23, 20)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)

    n, lo, hi = inputs.rmat_graph(small, seed=1)
    g = _graph(torch, n, lo, hi, inputs.draw_p(lo.shape[0], "beta22", 2))
    log(f"exact vs t, R-MAT s{small} Beta(2,2)")
    res[f"exact_rmat_s{small}_beta22"] = exact_vs_t(torch, g, TS)
    log("sampling queries per second vs t")
    res[f"sampling_qps_rmat_s{small}_beta22"] = sampling_qps(
        torch, g, TS[:-1], 1024, 10000, 1000)
    log("MAPE vs samples at t = 0.8")
    ks = [100, 300, 1000, 3000, 10000, 30000, 100000]
    res[f"mape_rmat_s{small}_beta22"] = mape_vs_k(torch, g, 0.8, 100, ks[:4] if args.quick else ks)
    del g
    torch.cuda.empty_cache()
    log(f"five distributions, R-MAT s{small}")
    res[f"distributions_rmat_s{small}"] = distributions(torch, n, lo, hi, TS)

    n, lo, hi = inputs.rmat_graph(big, seed=1)
    g = _graph(torch, n, lo, hi, inputs.draw_p(lo.shape[0], "bimodal", 2))
    log(f"exact vs t, R-MAT s{big} bimodal")
    res[f"exact_rmat_s{big}_bimodal"] = exact_vs_t(torch, g, TS)
    del g
    torch.cuda.empty_cache()

    text = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()
