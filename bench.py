#!/usr/bin/env python3
"""Benchmark: exact-count TEPS on R-MAT scale 23 (one MI355X).

A step is one exact counting query at t = 0.8 with probability pruning on the R-MAT
scale-23 graph (edge factor 16, P+ ~ 0.5*Beta(0.5,8) + 0.5*Beta(8,0.5)): per-query row
cuts, work items, and the triangle walk, counts read back to the host. TEPS = m / time
per query (the one-time graph load is reported separately, like the paper's
pre-sorting). The graph is resident in HBM before timing starts.

Printed on stdout: one JSON line (the contract fields plus `roofline`,
`cpu_baseline` and `secondary`). Progress goes to stderr.

  python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--no-secondary] [--no-cpu-baseline]
                  [--only-main] [--copy-calibration] [--cpu-full] [--cpu-detail]

The counts are checked against the CPU oracle's whole-graph counts of the same workload
(tests/golden/fullsize.json); the CPU baseline (the oracle) runs after all GPU timing.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_count_traffic.json")
# the autotuner's choice for the benchmark graphs, written by utri_autotune on an MI355X
TUNE_CACHE = os.path.join(ROOT, "profiles", "autotune_cache.jsonl")
# the walk kernel and what fixes its inputs' layout (the row packing is done at ingest)
WALK_SOURCES = ["paper_2602_14084_amd/csrc/walk.hip", "paper_2602_14084_amd/csrc/walk_common.h",
                "paper_2602_14084_amd/csrc/utri_internal.h", "paper_2602_14084_amd/csrc/ingest.hip"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def walk_source_hash() -> str:
    h = hashlib.sha256()
    for f in WALK_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per walk launch from the committed rocprofv3 counter summary, or None
    when the walk kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("walk_source_sha") != walk_source_hash() or rec.get("workload") != workload:
        return None
    return rec.get("traffic_bytes")


def timed(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=23)
    ap.add_argument("--tau", type=float, default=0.8)
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-main", action="store_true", help="main count timing only")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="utri_autotune cache: a line for this graph shape is taken as it is, "
                         "else the autotuner times its candidates and appends one")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 2 GiB device copy (counter calibration)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the oracle's whole count instead of a bounded sample")
    ap.add_argument("--cpu-detail", action="store_true",
                    help="also time the oracle on the small configurations, 1 and all threads")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs the hot path on a single "
              "MI355X; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.only_main:
        args.no_secondary = True
        args.no_cpu_baseline = True

    import torch

    from paper_2602_14084_amd import inputs, utri

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    # ------------------------------------------------------------ main workload
    t0 = time.time()
    n, lo, hi = inputs.rmat_graph(args.scale, seed=1)
    p = inputs.draw_p(lo.shape[0], "bimodal", 2)
    log(f"generated R-MAT s{args.scale}: n={n} m={lo.shape[0]} in {time.time() - t0:.1f}s")
    workload = f"rmat_s{args.scale}_ef16_bimodal_pruned_count_t{args.tau}"

    src = torch.from_numpy(lo).to(dev)
    dst = torch.from_numpy(hi).to(dev)
    pp = torch.from_numpy(p).to(dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    g = utri.Graph(src, dst, pp, n)
    torch.cuda.synchronize()
    load_ms = (time.perf_counter() - t) * 1e3
    del src, dst, pp
    m_edges = g.m
    log(f"ingest {load_ms:.1f} ms, m={g.m}, max_deg={g.max_deg}")

    # launch shape: the library's autotuner, for this graph at this threshold (set-up, not
    # part of the timed region)
    if not args.no_autotune:
        t = time.perf_counter()
        g.autotune(args.tau, args.tune_cache)
        log(f"autotune {(time.perf_counter() - t) * 1e3:.0f} ms: {g.tuning()}")
    tuning = g.tuning()

    method = utri.UTRI_PRUNED
    for _ in range(args.warmup):
        g.count(args.tau, method)
    utri.utri_timing(g.handle, 1)
    step_s, counts = timed(lambda: g.count(args.tau, method), args.steps, torch)
    walk_ms_total, launches = utri.utri_timing(g.handle, 0)
    walk_ms = walk_ms_total / max(1, launches)
    again = g.count(args.tau, method)
    assert again == counts, "counts differ between runs"
    # the oracle's whole-graph counts (tests/golden/fullsize.json, written by the CPU
    # oracle alone) for this exact workload: the benchmarked result must equal them
    want = golden_counts(args.scale, args.tau)
    if want is not None:
        assert tuple(want) == tuple(counts), ("counts differ from the oracle's", counts, want)
        log(f"counts equal the oracle's whole-graph counts {want}")
    teps = g.m / step_s
    stats = utri.utri_walk_stats(g.handle, args.tau, method)
    # staged-table algorithmic bytes: 4 B per streamed row id (each kept edge streams the
    # shorter of its two kept rows once), per kept edge 4 B of staged table id, 8 B of
    # partner ids (it is listed in the symmetric rows of both ends) and 8 B of its d, and
    # 8 B per candidate triangle (the streamed entry's d)
    b_alg = 4 * stats["target_elems"] + 20 * stats["m_c"] + 8 * stats["candidates"]
    achieved = b_alg / (walk_ms / 1e3) / 1e9
    log(f"count {counts} step {step_s * 1e3:.2f} ms, walk kernel {walk_ms:.2f} ms, "
        f"TEPS {teps:.3e}, B_alg {b_alg / 1e9:.1f} GB -> {achieved:.0f} GB/s")

    # top-k search (Section 5) on the same graph: the 1,000 most balanced / unbalanced
    tk = {}
    for name, which in (("balanced", utri.UTRI_BAL), ("unbalanced", utri.UTRI_UNBAL)):
        g.topk(1000, which)
        ms, (tri, sv) = timed(lambda: g.topk(1000, which), 3, torch)
        tk[name] = {"k": 1000, "ms": round(ms * 1e3, 2), "s_first": float(sv[0]),
                    "s_last": float(sv[-1])}
    log(f"top-1000 balanced {tk['balanced']['ms']} ms, unbalanced {tk['unbalanced']['ms']} ms")

    secondary = {
        "topk": tk,
        "ingest_ms": round(load_ms, 2),
        "counts": {"balanced": counts[0], "unbalanced": counts[1]},
        "walk_kernel_ms": round(walk_ms, 3),
        "walk_stats": stats,
        "b_alg_bytes": b_alg,
    }

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float64, device=dev)  # 2 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        secondary["copy_calibration_bytes"] = 2 * a.numel() * 8
        del a, b

    if not args.no_secondary:
        # enumeration at the same threshold (count walk + fill walk, unsorted): one call to
        # warm the output buffers, then the mean of two
        try:
            bal, unb = g.enumerate(args.tau, method, sorted=False)
            del bal, unb
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(2):
                bal, unb = g.enumerate(args.tau, method, sorted=False)
                nb, nu = int(bal.shape[0]), int(unb.shape[0])
                del bal, unb
            torch.cuda.synchronize()
            ems = (time.perf_counter() - t) * 1e3 / 2
            secondary["enumerate_ms"] = round(ems, 2)
            secondary["enumerated"] = [nb, nu]
            secondary["enumerate_triangles_per_s"] = (nb + nu) / (ems * 1e-3)
            secondary["enumerate_out_bytes"] = 12 * (nb + nu)
            assert (nb, nu) == counts
        except Exception as exc:  # noqa: BLE001 -- reported, never hidden
            secondary["enumerate_error"] = repr(exc)
        torch.cuda.empty_cache()
        secondary.update(run_secondary(args, torch, inputs, utri, dev))

    secondary["oracle_counts_equal"] = want is not None

    # ------------------------------------------------------------ CPU baseline (oracle)
    # runs after every GPU measurement, so the host is idle while the GPU is timed
    cpu = None
    if not args.no_cpu_baseline:
        del g
        torch.cuda.empty_cache()
        cpu = cpu_baseline(args, n, lo, hi, p, counts)
        if args.cpu_detail:
            secondary["cpu_detail"] = cpu_detail(inputs)

    traffic = measured_traffic(workload)
    line = {
        "metric": "exact-count TEPS on R-MAT s23",
        "value": teps,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "m": m_edges, "tau": args.tau, "method": "pruned",
                   "graph": f"R-MAT scale {args.scale}, edge factor 16, a=0.57 b=c=0.19, seed 1",
                   "p_dist": "0.5*Beta(0.5,8)+0.5*Beta(8,0.5), seed 2", "tuning": tuning},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_walk<WALK_COUNT>", "kernel_ms": walk_ms,
                     "algorithmic_bytes": b_alg},
        "cpu_baseline": cpu,
        "secondary": secondary,
    }
    print(json.dumps(line), flush=True)


def golden_counts(scale, tau):
    """The CPU oracle's whole-graph counts of this workload, when they are on file."""
    path = os.path.join(ROOT, "tests", "golden", "fullsize.json")
    try:
        with open(path) as f:
            rec = json.load(f)[f"rmat_s{scale}_bimodal"]
        return rec["counts"].get(str(tau))
    except (OSError, ValueError, KeyError):
        return None


def cpu_baseline(args, n, lo, hi, p, gpu_counts):
    """The oracle (node iterator with hash sets, all host threads) on the same query.

    Default: a bounded sample, vertices drawn uniformly (seed 5) until about 15 s of work,
    scaled to the whole graph by the node iterator's pair probes (the sample's share of
    them is computed exactly). --cpu-full times the whole count instead and checks it
    against the GPU's."""
    import oracle
    t = time.time()
    og = oracle.load(n, lo, hi, p)
    load_s = time.time() - t
    threads = oracle.num_threads()
    log(f"oracle load {load_s:.1f}s on {threads} threads")
    if args.cpu_full:
        t = time.time()
        full = og.count(args.tau)
        t_full = time.time() - t
        assert tuple(full) == tuple(gpu_counts), ("oracle and GPU counts differ", full, gpu_counts)
        sample = (f"whole graph, node iterator at t={args.tau}: {t_full:.1f}s, counts equal "
                  f"the GPU's; load {load_s:.0f}s not timed")
    else:
        rng = np.random.default_rng(5)
        k = max(1024, n // 512)
        t = time.time()
        og.count_vertices(args.tau, rng.choice(n, k, replace=False))
        first = time.time() - t
        k2 = int(min(n, max(k, k * 15.0 / max(first, 1e-3))))
        us = rng.choice(n, k2, replace=False)
        t = time.time()
        og.count_vertices(args.tau, us)
        t_sample = time.time() - t
        part, tot = og.probe_work(us)
        t_full = t_sample * tot / max(part, 1)
        sample = (f"node iterator at t={args.tau} over {k2} of {n} vertices drawn uniformly "
                  f"(seed 5): {t_sample:.1f}s for {part / tot:.3f} of the whole graph's "
                  f"{tot:.3e} pair probes, scaled by that share; load {load_s:.0f}s not timed")
    log(f"cpu baseline {og.m / t_full:.3e} edges/s on {threads} threads")
    return {"value": og.m / t_full, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": sample}


def cpu_detail(inputs):
    """Oracle timings on the small configurations, on one thread and on all of them: the
    Chung-Lu count, enumeration and expected count; the R-MAT s20 counts."""
    import oracle
    out = {}
    all_threads = oracle.num_threads()
    n, lo, hi = inputs.chung_lu_graph()
    p = inputs.draw_p(lo.shape[0], "uniform", 1)
    og = oracle.load(n, lo, hi, p)
    n2, lo2, hi2 = inputs.rmat_graph(20, seed=1)
    p2 = inputs.draw_p(lo2.shape[0], "beta22", 2)
    og2 = oracle.load(n2, lo2, hi2, p2)
    for th in (1, all_threads):
        oracle.set_threads(th)
        r = {}
        for name, fn in (("count_t0.6", lambda: og.count(0.6)),
                         ("enumerate_t0.6", lambda: og.enumerate(0.6)),
                         ("expected", lambda: og.expected())):
            t = time.time()
            fn()
            r["chung_lu_" + name + "_ms"] = (time.time() - t) * 1e3
        for tau in (0.5, 0.7, 0.9):
            t = time.time()
            og2.count(tau)
            r[f"rmat_s20_beta22_count_t{tau}_s"] = time.time() - t
            log(f"cpu detail: s20 count at t={tau} on {th} threads {time.time() - t:.1f}s")
        out[f"threads_{th}"] = r
        log(f"cpu detail on {th} threads: {r}")
    oracle.set_threads(all_threads)
    return out


def run_secondary(args, torch, inputs, utri, dev):
    out = {}
    # batch: 64 thresholds + 1,024 sampled worlds in one persistent launch (hipGraph)
    n, lo, hi = inputs.rmat_graph(20, seed=1)
    p = inputs.draw_p(lo.shape[0], "beta22", 2)
    g = utri.Graph(torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev),
                   torch.from_numpy(p).to(dev), n)
    ts = [0.5 + 0.0075 * j for j in range(64)]
    worlds, k, seed = 1024, 10000, 2026
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ex, es = g.batch(ts, k, worlds, seed, use_graph=True)
        side.synchronize()
        bt, _ = timed(lambda: g.batch(ts, k, worlds, seed, use_graph=True, exact=ex, est=es),
                      max(2, args.steps), torch)
    exact = ex.cpu().numpy().astype(np.float64)
    est = es.cpu().numpy()
    mape = np.abs(est - exact[None]) / np.maximum(exact[None], 1)
    mape = np.where(exact > 0, mape.mean(axis=0), np.nan)  # NaN where the exact count is 0
    st, _ = timed(lambda: g.sample(ts, k, worlds, seed), 2, torch)
    seq_counts = time.perf_counter()
    for tt in ts:
        g.count(tt)
    torch.cuda.synchronize()
    seq_counts = time.perf_counter() - seq_counts
    t3 = {}
    for tt in (0.5, 0.7, 0.9):
        t3[str(tt)] = {
            "pruned_ms": timed(lambda: g.count(tt, utri.UTRI_PRUNED), 3, torch)[0] * 1e3,
            "plain_ms": timed(lambda: g.count(tt, utri.UTRI_PLAIN), 3, torch)[0] * 1e3,
            "lemma3_ms": timed(lambda: g.count(tt, utri.UTRI_PRUNED_L3), 3, torch)[0] * 1e3,
            "counts": list(g.count(tt)),
        }
    out["rmat_s20_beta22_counts"] = t3
    out["batch_rmat_s20"] = {
        "worlds": worlds, "samples_per_world": k, "taus": 64,
        "batch_ms": bt * 1e3, "worlds_per_s": worlds / bt, "samples_per_s": worlds * k / bt,
        "sample_only_ms": st * 1e3, "sequential_64_counts_ms": seq_counts * 1e3,
        "mape_bal_by_tau": [float(x) for x in mape[:, 0]],
        "mape_unbal_by_tau": [float(x) for x in mape[:, 1]],
    }
    log(f"batch {bt * 1e3:.1f} ms ({worlds / bt:.0f} worlds/s), 64 sequential counts "
        f"{seq_counts * 1e3:.1f} ms")
    # vertex sampling (Section 6.1): 1,024 worlds x 1,000 vertices at the same thresholds
    kv = 1000
    g.sample(ts, kv, worlds, seed, utri.UTRI_SAMPLE_VERTEX)
    vt, ves = timed(lambda: g.sample(ts, kv, worlds, seed, utri.UTRI_SAMPLE_VERTEX), 2, torch)
    ves = ves.cpu().numpy()
    vmape = np.abs(ves - exact[None]) / np.maximum(exact[None], 1)
    vmape = np.where(exact > 0, vmape.mean(axis=0), np.nan)
    out["vertex_sample_rmat_s20"] = {
        "worlds": worlds, "vertices_per_world": kv, "taus": 64, "ms": vt * 1e3,
        "worlds_per_s": worlds / vt, "vertex_samples_per_s": worlds * kv / vt,
        "mape_bal_by_tau": [float(x) for x in vmape[:, 0]],
        "mape_unbal_by_tau": [float(x) for x in vmape[:, 1]],
    }
    log(f"vertex sampling {vt * 1e3:.1f} ms ({worlds * kv / vt:.3e} vertex samples/s)")
    del g
    torch.cuda.empty_cache()
    # differentiation: expected count forward + edge-centric backward on R-MAT s22
    n, lo, hi = inputs.rmat_graph(22, seed=1)
    p = inputs.draw_p(lo.shape[0], "uniform_05_95", 2)
    g = utri.Graph(torch.from_numpy(lo).to(dev), torch.from_numpy(hi).to(dev),
                   torch.from_numpy(p).to(dev), n)
    g.expected()
    grad = g.expected_grad()
    fwd, E = timed(lambda: g.expected(), max(2, args.steps), torch)
    bwd, _ = timed(lambda: g.expected_grad(grad), max(2, args.steps), torch)
    cnt, _ = timed(lambda: g.count(0.5, utri.UTRI_PLAIN), 2, torch)
    # possible-world sign Monte-Carlo of E: 1,024 worlds
    g.sign_worlds(1024, 7)
    swt, sw = timed(lambda: g.sign_worlds(1024, 7), 2, torch)
    sw = sw.cpu().numpy().astype(np.float64)
    out["sign_worlds_rmat_s22"] = {"worlds": 1024, "ms": swt * 1e3, "worlds_per_s": 1024 / swt,
                                   "mean": float(sw.mean()), "exact_expected": E,
                                   "rel_error_of_mean": float(abs(sw.mean() - E) / E),
                                   "rel_std_error": float(sw.std(ddof=1) / np.sqrt(1024) / E)}
    log(f"s22 sign worlds {swt * 1e3:.1f} ms for 1024 worlds")
    out["diff_rmat_s22"] = {"expected": E, "forward_ms": fwd * 1e3, "backward_ms": bwd * 1e3,
                            "backward_over_forward": bwd / fwd,
                            "plain_count_ms": cnt * 1e3, "m": g.m}
    log(f"s22 forward {fwd * 1e3:.1f} ms backward {bwd * 1e3:.1f} ms")
    del g, grad
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
