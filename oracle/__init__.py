"""ctypes front end of the CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline import this package; the library's product path never does. The
oracle shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OK, E_INVALID, E_CONFLICT, E_CAPACITY, E_NOMEM, E_RANGE = 0, -1, -2, -3, -4, -6

_lib = None

_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)
_u64p = C.POINTER(C.c_uint64)
_u32p = C.POINTER(C.c_uint32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.orc_load.argtypes = [C.c_int64, C.c_int64, _i64p, _i64p, _f64p, C.POINTER(vp)]
    lib.orc_free.argtypes = [vp]
    lib.orc_info.argtypes = [vp, _i64p, _i64p, _i64p, _i64p, _i64p]
    lib.orc_edges.argtypes = [vp, _i32p, _i32p, _f64p]
    lib.orc_count.argtypes = [vp, C.c_double, _i64p]
    lib.orc_count_multi.argtypes = [vp, _f64p, C.c_int, _i64p]
    lib.orc_count_vertices.argtypes = [vp, C.c_double, _i64p, C.c_int64, _i64p]
    lib.orc_enumerate.argtypes = [vp, C.c_double, _i32p, C.c_int64, _i32p, C.c_int64, _i64p]
    lib.orc_expected.argtypes = [vp, _f64p, _i64p, _u64p, _i64p]
    lib.orc_grad.argtypes = [vp, _i64p, C.c_int64, _f64p]
    lib.orc_edge_local.argtypes = [vp, _f64p, C.c_int, _i64p, C.c_int64, _i64p]
    lib.orc_local_expected.argtypes = [vp, _i64p, _f64p, C.c_int64, _i64p, _u64p]
    lib.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.orc_sample_edge.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int64]
    lib.orc_sample_edge.restype = C.c_int64
    lib.orc_sample.argtypes = [vp, _f64p, C.c_int, C.c_int64, C.c_int32, C.c_uint64, _f64p, _i64p]
    lib.orc_vertex_local.argtypes = [vp, _f64p, C.c_int, _i64p, C.c_int64, _i64p]
    lib.orc_sample_vertex.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int64]
    lib.orc_sample_vertex.restype = C.c_int64
    lib.orc_sample_vertices.argtypes = [vp, _f64p, C.c_int, C.c_int64, C.c_int32, C.c_uint64,
                                        _f64p, _i64p]
    lib.orc_topk.argtypes = [vp, C.c_int64, C.c_int, _i32p, _f64p, _i64p]
    lib.orc_sign_negative.argtypes = [C.c_uint64, C.c_int64, C.c_int32, C.c_double]
    lib.orc_sign_negative.restype = C.c_int
    lib.orc_sign_worlds.argtypes = [vp, C.c_int32, C.c_uint64, _i64p]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_set_threads.restype = C.c_int
    lib.orc_probe_work.argtypes = [vp, _i64p, C.c_int64, _i64p]
    lib.orc_hash_triples.argtypes = [_i32p, C.c_int64, C.c_int, _u64p, _i32p, C.c_int64, _i64p]
    lib.orc_enumerate_digest.argtypes = [vp, C.c_double, C.c_int, _i64p, _u64p, _i32p,
                                         C.c_int64, _i32p, C.c_int64, _i64p]
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(t)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def num_threads() -> int:
    return _load().orc_num_threads()


def set_threads(n: int) -> int:
    """Run later oracle calls on n OpenMP threads; returns the count in effect."""
    return _load().orc_set_threads(int(n))


class OracleGraph:
    """Canonical uncertain signed graph held by the oracle."""

    def __init__(self, n, src, dst, p):
        lib = _load()
        src = np.ascontiguousarray(src, dtype=np.int64)
        dst = np.ascontiguousarray(dst, dtype=np.int64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        h = C.c_void_p()
        rc = lib.orc_load(int(n), int(src.shape[0]), _p(src, _i64p), _p(dst, _i64p),
                          _p(p, _f64p), C.byref(h))
        if rc != OK:
            raise OracleError(rc, "load")
        self._h = h
        self._lib = lib
        vals = [C.c_int64() for _ in range(5)]
        lib.orc_info(h, *[C.byref(v) for v in vals])
        self.n, self.m, self.self_loops, self.dups, self.max_deg = [v.value for v in vals]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.orc_free(h)
            self._h = None

    def edges(self):
        lo = np.empty(self.m, np.int32)
        hi = np.empty(self.m, np.int32)
        p = np.empty(self.m, np.float64)
        self._lib.orc_edges(self._h, _p(lo, _i32p), _p(hi, _i32p), _p(p, _f64p))
        return lo, hi, p

    def count(self, t):
        out = np.zeros(2, np.int64)
        rc = self._lib.orc_count(self._h, float(t), _p(out, _i64p))
        if rc != OK:
            raise OracleError(rc, "count")
        return int(out[0]), int(out[1])

    def count_vertices(self, t, us):
        """Counts of the triangles whose lowest-ranked vertex is in `us`."""
        us = np.ascontiguousarray(us, dtype=np.int64)
        out = np.zeros(2, np.int64)
        rc = self._lib.orc_count_vertices(self._h, float(t), _p(us, _i64p), int(us.shape[0]),
                                          _p(out, _i64p))
        if rc != OK:
            raise OracleError(rc, "count_vertices")
        return int(out[0]), int(out[1])

    def probe_work(self, us):
        """(probes of the node iterator over the vertices `us`, probes over all vertices)."""
        us = np.ascontiguousarray(us, dtype=np.int64)
        out = np.zeros(2, np.int64)
        rc = self._lib.orc_probe_work(self._h, _p(us, _i64p), int(us.shape[0]), _p(out, _i64p))
        if rc != OK:
            raise OracleError(rc, "probe_work")
        return int(out[0]), int(out[1])

    def count_multi(self, ts):
        ts = np.ascontiguousarray(ts, dtype=np.float64)
        out = np.zeros((ts.shape[0], 2), np.int64)
        rc = self._lib.orc_count_multi(self._h, _p(ts, _f64p), int(ts.shape[0]), _p(out, _i64p))
        if rc != OK:
            raise OracleError(rc, "count_multi")
        return out

    def enumerate(self, t, cap=None):
        """(balanced, unbalanced) as int32 [k,3] arrays, rows sorted within and across."""
        counts = np.zeros(2, np.int64)
        if cap is None:
            nb, nu = self.count(t)
            cap = (nb, nu)
        bal = np.empty((max(cap[0], 1), 3), np.int32)
        unb = np.empty((max(cap[1], 1), 3), np.int32)
        rc = self._lib.orc_enumerate(self._h, float(t), _p(bal, _i32p), int(cap[0]),
                                     _p(unb, _i32p), int(cap[1]), _p(counts, _i64p))
        if rc != OK:
            raise OracleError(rc, "enumerate")
        return bal[:counts[0]].copy(), unb[:counts[1]].copy()

    def enumerate_digest(self, t, sample_bits=15, cap=1 << 20):
        """The enumeration at t reduced to an order-free digest: (counts [2], digest [4] =
        (sum, xor) of the balanced list then of the unbalanced one, sample_b, sample_u), the
        samples being the triangles of each list whose hash has its top `sample_bits` bits
        zero, sorted (see hash_triples)."""
        counts = np.zeros(2, np.int64)
        dig = np.zeros(4, np.uint64)
        sb = np.zeros((cap, 3), np.int32)
        su = np.zeros((cap, 3), np.int32)
        ns = np.zeros(2, np.int64)
        rc = self._lib.orc_enumerate_digest(self._h, float(t), int(sample_bits), _p(counts, _i64p),
                                            _p(dig, _u64p), _p(sb, _i32p), int(cap), _p(su, _i32p),
                                            int(cap), _p(ns, _i64p))
        if rc != OK:
            raise OracleError(rc, "enumerate_digest")
        if ns[0] > cap or ns[1] > cap:
            raise OracleError(E_CAPACITY, "enumerate_digest sample")
        return counts, dig, sb[:ns[0]].copy(), su[:ns[1]].copy()

    def expected(self):
        """(E, T, S) with S the exact fixed-point sum of s as a Python int."""
        E = C.c_double()
        T = C.c_int64()
        lo = C.c_uint64()
        hi = C.c_int64()
        rc = self._lib.orc_expected(self._h, C.byref(E), C.byref(T), C.byref(lo), C.byref(hi))
        if rc != OK:
            raise OracleError(rc, "expected")
        return E.value, T.value, (hi.value << 64) + lo.value

    def grad(self, eids=None):
        eids = np.arange(self.m, dtype=np.int64) if eids is None else np.ascontiguousarray(eids, np.int64)
        out = np.empty(eids.shape[0], np.float64)
        rc = self._lib.orc_grad(self._h, _p(eids, _i64p), int(eids.shape[0]), _p(out, _f64p))
        if rc != OK:
            raise OracleError(rc, "grad")
        return out

    def local_expected_fixed(self, eids, q):
        """Exact N_e(q) (Python ints) with L_e(q) = N * 2^-63 = sum over triangles through e
        of P_bal with P+(e) replaced by q."""
        eids = np.ascontiguousarray(eids, np.int64)
        q = np.ascontiguousarray(np.broadcast_to(np.asarray(q, np.float64), eids.shape))
        hi = np.zeros(eids.shape[0], np.int64)
        lo = np.zeros(eids.shape[0], np.uint64)
        rc = self._lib.orc_local_expected(self._h, _p(eids, _i64p), _p(q, _f64p),
                                          int(eids.shape[0]), _p(hi, _i64p), _p(lo, _u64p))
        if rc != OK:
            raise OracleError(rc, "local_expected")
        return [(int(h) << 64) + int(l) for h, l in zip(hi, lo)]

    def local_central_difference(self, eids, h):
        """(L_e(fl(p+h)) - L_e(fl(p-h))) / (fl(p+h) - fl(p-h)) per edge, exact up to the
        2^-63 rounding of each term (E is affine in p_e, so this equals dE/dp_e)."""
        _, _, p = self.edges()
        eids = np.ascontiguousarray(eids, np.int64)
        qp = np.minimum(p[eids] + h, 1.0)
        qm = np.maximum(p[eids] - h, 0.0)
        Np = self.local_expected_fixed(eids, qp)
        Nm = self.local_expected_fixed(eids, qm)
        from fractions import Fraction
        return np.array([float(Fraction(a - b, 2 ** 63) / (Fraction(float(x)) - Fraction(float(y))))
                         for a, b, x, y in zip(Np, Nm, qp, qm)])

    def edge_local(self, ts, eids=None):
        ts = np.atleast_1d(np.ascontiguousarray(ts, dtype=np.float64))
        eids = np.arange(self.m, dtype=np.int64) if eids is None else np.ascontiguousarray(eids, np.int64)
        out = np.zeros((eids.shape[0], ts.shape[0], 2), np.int64)
        rc = self._lib.orc_edge_local(self._h, _p(ts, _f64p), int(ts.shape[0]), _p(eids, _i64p),
                                      int(eids.shape[0]), _p(out, _i64p))
        if rc != OK:
            raise OracleError(rc, "edge_local")
        return out

    def sample(self, ts, k, worlds, seed):
        ts = np.atleast_1d(np.ascontiguousarray(ts, dtype=np.float64))
        est = np.zeros((worlds, ts.shape[0], 2), np.float64)
        sums = np.zeros((worlds, ts.shape[0], 2), np.int64)
        rc = self._lib.orc_sample(self._h, _p(ts, _f64p), int(ts.shape[0]), int(k), int(worlds),
                                  C.c_uint64(seed), _p(est, _f64p), _p(sums, _i64p))
        if rc != OK:
            raise OracleError(rc, "sample")
        return est, sums


    def vertex_local(self, ts, vs=None):
        """Local counts at each listed vertex (all vertices by default): [k][nt][2]."""
        ts = np.atleast_1d(np.ascontiguousarray(ts, dtype=np.float64))
        vs = np.arange(self.n, dtype=np.int64) if vs is None else np.ascontiguousarray(vs, np.int64)
        out = np.zeros((vs.shape[0], ts.shape[0], 2), np.int64)
        rc = self._lib.orc_vertex_local(self._h, _p(ts, _f64p), int(ts.shape[0]), _p(vs, _i64p),
                                        int(vs.shape[0]), _p(out, _i64p))
        if rc != OK:
            raise OracleError(rc, "vertex_local")
        return out

    def sample_vertices(self, ts, k, worlds, seed):
        ts = np.atleast_1d(np.ascontiguousarray(ts, dtype=np.float64))
        est = np.zeros((worlds, ts.shape[0], 2), np.float64)
        sums = np.zeros((worlds, ts.shape[0], 2), np.int64)
        rc = self._lib.orc_sample_vertices(self._h, _p(ts, _f64p), int(ts.shape[0]), int(k),
                                           int(worlds), C.c_uint64(seed), _p(est, _f64p),
                                           _p(sums, _i64p))
        if rc != OK:
            raise OracleError(rc, "sample_vertices")
        return est, sums


    def topk(self, k, which):
        """(triples [r][3] int32 sorted within, s [r] f64), r = min(k, #qualifying); which is
        1 for the most balanced (smallest s, s <= 0) or 2 for the most unbalanced (largest
        s, s > 0); ties in s by the triple, lexicographically."""
        tri = np.zeros((max(k, 1), 3), np.int32)
        sv = np.zeros(max(k, 1), np.float64)
        cnt = np.zeros(1, np.int64)
        rc = self._lib.orc_topk(self._h, int(k), int(which), _p(tri, _i32p), _p(sv, _f64p),
                                _p(cnt, _i64p))
        if rc != OK:
            raise OracleError(rc, "topk")
        r = int(cnt[0])
        return tri[:r].copy(), sv[:r].copy()


    def sign_worlds(self, worlds, seed):
        """Balanced triangles in each of `worlds` sampled sign worlds: int64 [worlds]."""
        out = np.zeros(worlds, np.int64)
        rc = self._lib.orc_sign_worlds(self._h, int(worlds), C.c_uint64(seed), _p(out, _i64p))
        if rc != OK:
            raise OracleError(rc, "sign_worlds")
        return out


def load(n, src, dst, p) -> OracleGraph:
    return OracleGraph(n, src, dst, p)


def hash_triples(tri, sample_bits=15, cap=1 << 20):
    """Order-free digest (sum mod 2^64, xor) of a list of triangles, int32 [k,3] with each
    row sorted ascending, h(a, b, c) = splitmix64(splitmix64((a << 32) | b) + c), and the
    spot sample: the rows whose h has its top `sample_bits` bits zero, in list order."""
    tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(2, np.uint64)
    samp = np.zeros((cap, 3), np.int32)
    ns = np.zeros(1, np.int64)
    rc = _load().orc_hash_triples(_p(tri, _i32p), int(tri.shape[0]), int(sample_bits),
                                  _p(out, _u64p), _p(samp, _i32p), int(cap), _p(ns, _i64p))
    if rc != OK:
        raise OracleError(rc, "hash_triples")
    if ns[0] > cap:
        raise OracleError(E_CAPACITY, "hash_triples sample")
    return out, samp[:ns[0]].copy()


def philox4x32_10(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib.orc_philox4x32_10(_p(c, _u32p), _p(k, _u32p), _p(out, _u32p))
    return out


def sample_edge(seed, world, i, m) -> int:
    return int(_load().orc_sample_edge(C.c_uint64(seed), C.c_uint32(world), C.c_uint64(i), int(m)))


def sample_vertex(seed, world, i, n) -> int:
    return int(_load().orc_sample_vertex(C.c_uint64(seed), C.c_uint32(world), C.c_uint64(i), int(n)))


def sign_negative(seed, e, w, p) -> int:
    return int(_load().orc_sign_negative(C.c_uint64(seed), int(e), int(w), float(p)))
