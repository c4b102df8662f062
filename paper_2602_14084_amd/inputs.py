"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws graphs and per-edge P+ values. It holds none of the
balance arithmetic (no d = 1 - 2p, no triangle products, no thresholds), so the
oracle and the HIP path can both consume it without sharing any of the method.

Graph families stand in for the paper's SNAP/Konect datasets (Table 2 of the
paper lists their sizes, degrees and P+ distributions):

* R-MAT (Graph500-style quadrant recursion, a=0.57, b=c=0.19, d=0.05, edge
  factor 16, no noise), relabelled by a seeded vertex permutation, symmetrised,
  self-loops dropped, duplicates merged.
* Chung-Lu power law, weights w_i proportional to (i+1)^(-1/(gamma-1)), rescaled
  so that the expected edge count hits a target, one Bernoulli per vertex pair.

P+ draws follow the distributions of the paper's experiments section: Uniform,
Beta(0.5,0.5), Beta(a,b), plus the mixtures the benchmarks use. P+ is drawn per
unique canonical edge in ascending (lo, hi) order, which is the library's edge-id
order, so a seed fixes the value on every edge.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "rmat_graph", "chung_lu_graph", "draw_p", "random_graph", "dirty_edges",
    "CONFIGS", "make_config",
]


def _canonical_unique(n: int, src: np.ndarray, dst: np.ndarray):
    """Undirected (min, max) pairs, self-loops dropped, duplicates merged, sorted."""
    lo = np.minimum(src, dst).astype(np.int64)
    hi = np.maximum(src, dst).astype(np.int64)
    keep = lo != hi
    key = (lo[keep] << 32) | hi[keep]
    key = np.unique(key)
    return (key >> 32).astype(np.int64), (key & 0xFFFFFFFF).astype(np.int64)


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _rmat_chunk(seed_seq, cnt: int, scale: int, t_a, t_ab, t_abc):
    rng = np.random.Generator(np.random.PCG64(seed_seq))
    src = np.zeros(cnt, dtype=np.uint32)
    dst = np.zeros(cnt, dtype=np.uint32)
    c_or_d = np.empty(cnt, dtype=bool)
    tmp = np.empty(cnt, dtype=bool)
    for _ in range(scale):
        r = rng.integers(0, 1 << 32, cnt, dtype=np.uint32)
        src <<= np.uint32(1)
        dst <<= np.uint32(1)
        # quadrant a = r < t_a, b = [t_a, t_ab), c = [t_ab, t_abc), d = r >= t_abc.
        # src bit is set in c and d; dst bit is set in b and d (parity of the three tests).
        np.greater_equal(r, t_ab, out=c_or_d)
        src |= c_or_d
        np.greater_equal(r, t_a, out=tmp)
        np.logical_xor(tmp, c_or_d, out=tmp)
        np.logical_xor(tmp, r >= t_abc, out=tmp)
        dst |= tmp
    return src, dst


def _sorted_unique_keys(keys: np.ndarray, nbits_hi: int) -> np.ndarray:
    """np.unique over non-negative int64 keys whose high word has nbits_hi bits.

    Keys are split into 16 ranges by their top bits (a stable radix pass on a
    uint8 bucket id) and each range is sorted and deduplicated in a thread.
    """
    nb = 16
    shift = 32 + nbits_hi - 4
    bucket = (keys >> np.int64(shift)).astype(np.uint8)
    order = np.argsort(bucket, kind="stable")
    keys = keys[order]
    del order
    bounds = np.concatenate([[0], np.cumsum(np.bincount(bucket, minlength=nb))])
    del bucket
    parts = [keys[bounds[i]:bounds[i + 1]] for i in range(nb)]
    with ThreadPoolExecutor(_workers()) as ex:
        parts = list(ex.map(np.unique, parts))
    return np.concatenate(parts)


def rmat_graph(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
               c: float = 0.19, seed: int = 1, chunk: int = 1 << 22):
    """R-MAT edge list at 2**scale vertices; returns (n, lo, hi) canonical and unique.

    Each quadrant choice uses 32 random bits (thresholds rounded to 2**-32). Chunk i
    of the raw edge stream draws from its own spawned PCG64 stream, so the graph
    does not depend on how many threads generate it.
    """
    n = 1 << scale
    m_raw = edge_factor * n
    t_a = np.uint32(round(a * 2.0 ** 32))
    t_ab = np.uint32(round((a + b) * 2.0 ** 32))
    t_abc = np.uint32(round((a + b + c) * 2.0 ** 32))
    nchunks = (m_raw + chunk - 1) // chunk
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(nchunks + 1)
    sizes = [min(chunk, m_raw - i * chunk) for i in range(nchunks)]
    with ThreadPoolExecutor(_workers()) as ex:
        outs = list(ex.map(lambda i: _rmat_chunk(children[i], sizes[i], scale, t_a, t_ab, t_abc),
                           range(nchunks)))
    src = np.concatenate([o[0] for o in outs])
    dst = np.concatenate([o[1] for o in outs])
    del outs
    perm = np.random.Generator(np.random.PCG64(children[nchunks])).permutation(n).astype(np.uint32)
    src = perm[src]
    dst = perm[dst]
    lo = np.minimum(src, dst)
    hi = np.maximum(src, dst)
    del src, dst
    keep = lo != hi
    key = (lo[keep].astype(np.int64) << np.int64(32)) | hi[keep].astype(np.int64)
    del lo, hi, keep
    key = _sorted_unique_keys(key, max(scale, 4))
    return n, (key >> np.int64(32)).astype(np.int64), (key & np.int64(0xFFFFFFFF)).astype(np.int64)


def chung_lu_graph(n: int = 2000, gamma: float = 2.5, m_target: float = 20000.0, seed: int = 1):
    """Chung-Lu graph with power-law expected degrees; returns (n, lo, hi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w0 = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    iu, ju = np.triu_indices(n, k=1)

    def expected(scale):
        w = w0 * scale
        return np.minimum(1.0, w[iu] * w[ju] / w.sum()).sum()

    lo_s, hi_s = 1e-3, 1e6
    for _ in range(200):
        mid = np.sqrt(lo_s * hi_s)
        if expected(mid) < m_target:
            lo_s = mid
        else:
            hi_s = mid
    w = w0 * np.sqrt(lo_s * hi_s)
    prob = np.minimum(1.0, w[iu] * w[ju] / w.sum())
    take = rng.random(prob.shape[0]) < prob
    return n, iu[take].astype(np.int64), ju[take].astype(np.int64)


def random_graph(n: int, density: float, seed: int):
    """Erdos-Renyi style tiny graph for brute-force checks; returns (n, lo, hi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, k=1)
    take = rng.random(iu.shape[0]) < density
    return n, iu[take].astype(np.int64), ju[take].astype(np.int64)


def draw_p(m: int, dist: str, seed: int) -> np.ndarray:
    """Per-edge P+ in edge-id order.

    dist: 'uniform' U(0,1); 'uniform_05_95' U(0.05,0.95); 'beta22' Beta(2,2);
    'beta0505' Beta(0.5,0.5); 'beta31' / 'beta13'; 'normal' N(0.5,0.15) clipped;
    'bimodal' 0.5*Beta(0.5,8)+0.5*Beta(8,0.5); 'dyadic16' k/16 for k in 0..16;
    'certain' {0,1}; 'tri' {0, 0.5, 1}; 'half' all 0.5.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if dist == "uniform":
        return rng.random(m)
    if dist == "uniform_05_95":
        return 0.05 + 0.9 * rng.random(m)
    if dist == "beta22":
        return rng.beta(2.0, 2.0, m)
    if dist == "beta0505":
        return rng.beta(0.5, 0.5, m)
    if dist == "beta31":
        return rng.beta(3.0, 1.0, m)
    if dist == "beta13":
        return rng.beta(1.0, 3.0, m)
    if dist == "normal":
        return np.clip(rng.normal(0.5, 0.15, m), 0.0, 1.0)
    if dist == "bimodal":
        pick = rng.random(m) < 0.5
        lo = rng.beta(0.5, 8.0, m)
        hi = rng.beta(8.0, 0.5, m)
        return np.where(pick, lo, hi)
    if dist == "dyadic16":
        return rng.integers(0, 17, m).astype(np.float64) / 16.0
    if dist == "certain":
        return rng.integers(0, 2, m).astype(np.float64)
    if dist == "tri":
        return rng.integers(0, 3, m).astype(np.float64) / 2.0
    if dist == "half":
        return np.full(m, 0.5)
    raise ValueError(f"unknown P+ distribution {dist!r}")


def dirty_edges(lo: np.ndarray, hi: np.ndarray, p: np.ndarray, seed: int,
                dup_frac: float = 0.1, self_loops: int = 5, n: int | None = None):
    """Raw input with shuffled order, random orientation, exact duplicates and self-loops.

    Loading it must give back the canonical (lo, hi, p) graph.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    m = lo.shape[0]
    k = int(m * dup_frac)
    dup = rng.integers(0, m, k) if m else np.zeros(0, dtype=np.int64)
    src = np.concatenate([lo, lo[dup]])
    dst = np.concatenate([hi, hi[dup]])
    pp = np.concatenate([p, p[dup]])
    if n is None:
        n = int(max(hi.max() if m else 0, 0)) + 1
    if self_loops:
        v = rng.integers(0, n, self_loops)
        src = np.concatenate([src, v])
        dst = np.concatenate([dst, v])
        pp = np.concatenate([pp, rng.random(self_loops)])
    flip = rng.random(src.shape[0]) < 0.5
    s2 = np.where(flip, dst, src)
    d2 = np.where(flip, src, dst)
    order = rng.permutation(src.shape[0])
    return s2[order].astype(np.int64), d2[order].astype(np.int64), pp[order].astype(np.float64)


# Workload recipes. 'query' fields describe what is run on them.
CONFIGS = {
    "chunglu_n2000": dict(kind="chunglu", n=2000, gamma=2.5, m_target=20000.0, gseed=1,
                          dist="uniform", pseed=1, taus=(0.6,)),
    "rmat_s20_beta22": dict(kind="rmat", scale=20, gseed=1, dist="beta22", pseed=2,
                            taus=(0.5, 0.7, 0.9)),
    "rmat_s23_bimodal": dict(kind="rmat", scale=23, gseed=1, dist="bimodal", pseed=2,
                             taus=(0.8,)),
    "rmat_s20_batch": dict(kind="rmat", scale=20, gseed=1, dist="beta22", pseed=2,
                           taus=tuple(0.5 + 0.0075 * j for j in range(64))),
    "rmat_s22_uniform": dict(kind="rmat", scale=22, gseed=1, dist="uniform_05_95", pseed=2,
                             taus=()),
}


def make_config(name: str, scale_override: int | None = None):
    """Build a named workload: returns dict(n, lo, hi, p, taus)."""
    cfg = dict(CONFIGS[name])
    if cfg["kind"] == "chunglu":
        n, lo, hi = chung_lu_graph(cfg["n"], cfg["gamma"], cfg["m_target"], cfg["gseed"])
    else:
        scale = scale_override if scale_override is not None else cfg["scale"]
        n, lo, hi = rmat_graph(scale, seed=cfg["gseed"])
    p = draw_p(lo.shape[0], cfg["dist"], cfg["pseed"])
    return dict(n=n, lo=lo, hi=hi, p=p, taus=cfg["taus"], name=name)
