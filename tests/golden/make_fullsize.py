"""Write the oracle's results on the full-size workloads to tests/golden/ (CPU only).

The GPU tests compare the library with these values. Every number here comes from the
CPU oracle (oracle/) on the seeded inputs of paper_2602_14084_amd/inputs.py; nothing
is taken from the HIP library. Run on a multi-core host (minutes per graph):

    python tests/golden/make_fullsize.py [s23] [s22] [s20]

Outputs:
  fullsize.json                 counts, digests, expected counts, sampler estimates
  rmat_s23_t08_sample.txt.gz    spot sample of the s23 enumeration at t = 0.8
                                (class, a, b, c per line; a < b < c, original ids)
"""
from __future__ import annotations

import gzip
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2602_14084_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "fullsize.json")
SAMPLE = os.path.join(HERE, "rmat_s23_t08_sample.txt.gz")
S23_TS = [0.5, 0.8, 0.9, 0.95]
SAMPLE_BITS = 15          # one triangle in 32,768 of each list
BATCH_TS = [0.5 + 0.0075 * j for j in range(64)]
BATCH_WORLDS = 32         # the first 32 of the benchmark's 1,024 replicates
BATCH_K, BATCH_SEED = 10000, 2026


def log(*a):
    print("[golden]", *a, flush=True)


def hexf(x: float) -> str:
    return float(x).hex()


def s23(rec):
    n, lo, hi = inputs.rmat_graph(23, seed=1)
    p = inputs.draw_p(lo.shape[0], "bimodal", 2)
    t = time.time()
    og = oracle.load(n, lo, hi, p)
    log(f"s23 load {time.time() - t:.0f}s m={og.m}")
    t = time.time()
    cnt = og.count_multi(S23_TS)
    log(f"s23 counts {cnt.tolist()} in {time.time() - t:.0f}s")
    t = time.time()
    counts, dig, sb, su = og.enumerate_digest(0.8, SAMPLE_BITS)
    log(f"s23 digest {counts.tolist()} samples {sb.shape[0]}/{su.shape[0]} in {time.time() - t:.0f}s")
    rec["rmat_s23_bimodal"] = {
        "graph": "R-MAT scale 23, edge factor 16, seed 1; P+ bimodal seed 2",
        "n": int(og.n), "m": int(og.m), "threads": oracle.num_threads(),
        "counts": {str(t): [int(a), int(b)] for t, (a, b) in zip(S23_TS, cnt)},
        "enumerate_t0.8": {"counts": [int(x) for x in counts],
                           "digest_bal": [str(int(dig[0])), str(int(dig[1]))],
                           "digest_unbal": [str(int(dig[2])), str(int(dig[3]))],
                           "sample_bits": SAMPLE_BITS,
                           "sample_sizes": [int(sb.shape[0]), int(su.shape[0])]},
    }
    with gzip.open(SAMPLE, "wt") as f:
        f.write("# class a b c: triangles of the t = 0.8 lists whose digest hash has its top "
                f"{SAMPLE_BITS} bits zero (oracle, R-MAT s23 bimodal)\n")
        for cls, arr in (("B", sb), ("U", su)):
            for a, b, c in arr:
                f.write(f"{cls} {a} {b} {c}\n")


def s22(rec):
    n, lo, hi = inputs.rmat_graph(22, seed=1)
    p = inputs.draw_p(lo.shape[0], "uniform_05_95", 2)
    t = time.time()
    og = oracle.load(n, lo, hi, p)
    log(f"s22 load {time.time() - t:.0f}s m={og.m}")
    t = time.time()
    E, T, S = og.expected()
    log(f"s22 E={E!r} T={T} in {time.time() - t:.0f}s")
    rec["rmat_s22_uniform_05_95"] = {
        "graph": "R-MAT scale 22, edge factor 16, seed 1; P+ U(0.05,0.95) seed 2",
        "n": int(og.n), "m": int(og.m), "expected": hexf(E), "triangles": int(T),
        "sum_s_fixed62": str(S),
    }


def s20(rec):
    n, lo, hi = inputs.rmat_graph(20, seed=1)
    p = inputs.draw_p(lo.shape[0], "beta22", 2)
    t = time.time()
    og = oracle.load(n, lo, hi, p)
    log(f"s20 load {time.time() - t:.0f}s m={og.m}")
    t = time.time()
    cnt = og.count_multi(BATCH_TS)
    log(f"s20 64 counts in {time.time() - t:.0f}s")
    t = time.time()
    est, sums = og.sample(BATCH_TS, BATCH_K, BATCH_WORLDS, BATCH_SEED)
    log(f"s20 sampler {BATCH_WORLDS} worlds in {time.time() - t:.0f}s")
    rec["rmat_s20_beta22_batch"] = {
        "graph": "R-MAT scale 20, edge factor 16, seed 1; P+ Beta(2,2) seed 2",
        "n": int(og.n), "m": int(og.m), "ts": BATCH_TS, "k": BATCH_K, "seed": BATCH_SEED,
        "worlds": BATCH_WORLDS, "exact": cnt.tolist(),
        "sums": sums.tolist(),
        "est": [[[hexf(x) for x in row] for row in w] for w in est],
    }


def main():
    which = sys.argv[1:] or ["s23", "s22", "s20"]
    rec = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            rec = json.load(f)
    for name in which:
        {"s23": s23, "s22": s22, "s20": s20}[name](rec)
        with open(OUT, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
            f.write("\n")
    log("wrote", OUT)


if __name__ == "__main__":
    main()
