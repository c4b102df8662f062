"""Thin ctypes binding of libutri (include/utri.h): argument marshalling only.

Every step of every query runs in the HIP kernels of libutri.so; this module only
passes pointers, sizes and the current torch stream. It raises if the library has
not been built -- there is no fallback path.

Functions carry the names of the C entry points. Tensors may live on the GPU
(passed as device pointers) or on the host (numpy arrays or CPU tensors, passed as
host pointers where the C call accepts them). Results that the C call writes to
device memory are returned as CUDA tensors on the current device.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libutri.so")

UTRI_OK = 0
UTRI_E_INVALID = -1
UTRI_E_CONFLICT = -2
UTRI_E_CAPACITY = -3
UTRI_E_NOMEM = -4
UTRI_E_HIP = -5
UTRI_E_RANGE = -6
UTRI_PLAIN, UTRI_PRUNED, UTRI_PRUNED_L3 = 0, 1, 2
UTRI_BAL, UTRI_UNBAL, UTRI_BOTH = 1, 2, 3
UTRI_HOST_PTR, UTRI_DEVICE_PTR = 0, 1
UTRI_SAMPLE_EDGE, UTRI_SAMPLE_VERTEX, UTRI_SAMPLE_EDGE_PLAIN, UTRI_SAMPLE_VERTEX_PLAIN = 0, 1, 2, 3
UTRI_ORDER_AUTO, UTRI_ORDER_PLAIN, UTRI_ORDER_SHORTER = 0, 1, 2

ABI_FUNCTIONS = [
    "utri_graph_load", "utri_graph_free", "utri_graph_info", "utri_graph_edges",
    "utri_graph_set_p", "utri_count", "utri_count_batch", "utri_enumerate", "utri_expected",
    "utri_expected_grad", "utri_edge_local", "utri_vertex_local", "utri_topk", "utri_sign_worlds", "utri_sample", "utri_batch", "utri_autotune", "utri_set_walk_order",
    "utri_walk_stats", "utri_timing", "utri_strerror", "utri_count_noalloc",
    "utri_get_tuning", "utri_set_tuning",
]

# launch parameters, in the order of utri_get_tuning / utri_set_tuning
TUNE_NAMES = ["walk_blocks_per_cu", "sample_chunk", "walk_partners", "walk_light_cap",
              "walk_chunk", "walk_unroll", "walk_shorter_min"]

_lib = None


class UtriError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = _lib.utri_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what} failed: {msg} ({code})")
        self.code = code


def lib():
    """Load libutri.so (raises if it is missing: build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, f64, u64 = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_uint64
    P = C.POINTER
    L.utri_graph_load.argtypes = [vp, vp, vp, i64, i64, C.c_int, vp, P(vp)]
    L.utri_graph_free.argtypes = [vp]
    L.utri_graph_info.argtypes = [vp, P(i64), P(i64), P(i64), P(i64), P(i64)]
    L.utri_graph_edges.argtypes = [vp, vp, vp, vp, C.c_int, vp]
    L.utri_graph_set_p.argtypes = [vp, vp, C.c_int, vp]
    L.utri_count.argtypes = [vp, f64, C.c_int, C.c_int, P(i64), vp]
    L.utri_count_noalloc.argtypes = [vp, f64, C.c_int, C.c_int, P(i64), vp]
    L.utri_count_batch.argtypes = [vp, P(f64), C.c_int, C.c_int, P(i64), vp]
    L.utri_enumerate.argtypes = [vp, f64, C.c_int, C.c_int, vp, i64, vp, i64, P(i64), C.c_int, vp]
    L.utri_expected.argtypes = [vp, P(f64), vp]
    L.utri_expected_grad.argtypes = [vp, vp, vp]
    L.utri_edge_local.argtypes = [vp, P(f64), C.c_int, vp, i64, vp, vp]
    L.utri_vertex_local.argtypes = [vp, P(f64), C.c_int, vp, i64, vp, vp]
    L.utri_topk.argtypes = [vp, i64, C.c_int, vp, vp, P(i64), vp]
    L.utri_sign_worlds.argtypes = [vp, i32, u64, vp, vp]
    L.utri_sample.argtypes = [vp, P(f64), C.c_int, i64, i32, u64, C.c_int, vp, vp]
    L.utri_batch.argtypes = [vp, P(f64), C.c_int, i64, i32, u64, vp, vp, C.c_int, vp]
    L.utri_autotune.argtypes = [vp, f64, C.c_char_p, vp]
    L.utri_set_walk_order.argtypes = [vp, C.c_int]
    L.utri_get_tuning.argtypes = [vp, P(i64)]
    L.utri_set_tuning.argtypes = [vp, P(i64)]
    L.utri_walk_stats.argtypes = [vp, f64, C.c_int, P(i64), vp]
    L.utri_timing.argtypes = [vp, C.c_int, P(f64), P(i64)]
    L.utri_strerror.argtypes = [C.c_int]
    L.utri_strerror.restype = C.c_char_p
    for name in ABI_FUNCTIONS:
        if name != "utri_strerror":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != UTRI_OK:
        raise UtriError(rc, what)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _as_input(x, dtype):
    """(pointer, keepalive, ptr_kind) for an input array on either side."""
    torch = _torch()
    if isinstance(x, torch.Tensor):
        tdt = {np.int64: torch.int64, np.float64: torch.float64}[dtype]
        x = x.to(tdt).contiguous()
        kind = UTRI_DEVICE_PTR if x.is_cuda else UTRI_HOST_PTR
        return C.c_void_p(x.data_ptr()), x, kind
    a = np.ascontiguousarray(x, dtype=dtype)
    return C.c_void_p(a.ctypes.data), a, UTRI_HOST_PTR


def _f64_array(ts):
    a = np.ascontiguousarray(np.atleast_1d(np.asarray(ts, dtype=np.float64)))
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


# ---------------------------------------------------------------- C entry points

def utri_graph_load(src, dst, p, n, stream=None):
    """Handle (c_void_p) of the canonical graph built from (src, dst, p) with n vertices."""
    L = lib()
    ps, ks, kind_s = _as_input(src, np.int64)
    pd, kd, kind_d = _as_input(dst, np.int64)
    pp, kp, kind_p = _as_input(p, np.float64)
    if len({kind_s, kind_d, kind_p}) != 1:
        raise ValueError("src, dst and p must all be on the host or all on the device")
    m_in = int(ks.shape[0])
    h = C.c_void_p()
    rc = L.utri_graph_load(ps, pd, pp, m_in, int(n), kind_s, _stream(stream), C.byref(h))
    _check(rc, "utri_graph_load")
    return h


def utri_graph_free(h):
    return lib().utri_graph_free(h)


def utri_graph_info(h):
    vals = [C.c_int64() for _ in range(5)]
    _check(lib().utri_graph_info(h, *[C.byref(v) for v in vals]), "utri_graph_info")
    keys = ["n", "m", "self_loops_dropped", "dups_merged", "max_deg"]
    return {k: v.value for k, v in zip(keys, vals)}


def utri_graph_edges(h, device=False, stream=None):
    torch = _torch()
    m = utri_graph_info(h)["m"]
    dev = torch.device("cuda") if device else torch.device("cpu")
    lo = torch.empty(m, dtype=torch.int32, device=dev)
    hi = torch.empty(m, dtype=torch.int32, device=dev)
    p = torch.empty(m, dtype=torch.float64, device=dev)
    kind = UTRI_DEVICE_PTR if device else UTRI_HOST_PTR
    rc = lib().utri_graph_edges(h, C.c_void_p(lo.data_ptr()), C.c_void_p(hi.data_ptr()),
                                C.c_void_p(p.data_ptr()), kind, _stream(stream))
    _check(rc, "utri_graph_edges")
    return lo, hi, p


def utri_graph_set_p(h, p, stream=None):
    pp, keep, kind = _as_input(p, np.float64)
    _check(lib().utri_graph_set_p(h, pp, kind, _stream(stream)), "utri_graph_set_p")
    del keep


def utri_count(h, t, method=UTRI_PRUNED, which=UTRI_BOTH, stream=None):
    out = (C.c_int64 * 2)()
    _check(lib().utri_count(h, float(t), method, which, out, _stream(stream)), "utri_count")
    return int(out[0]), int(out[1])


def utri_count_noalloc(h, t, method=UTRI_PRUNED, which=UTRI_BOTH, stream=None):
    """utri_count on the library's static device scratch (no allocation)."""
    out = (C.c_int64 * 2)()
    _check(lib().utri_count_noalloc(h, float(t), method, which, out, _stream(stream)),
           "utri_count_noalloc")
    return int(out[0]), int(out[1])


def utri_count_batch(h, ts, method=UTRI_PRUNED, stream=None):
    a, pa = _f64_array(ts)
    out = np.zeros((a.shape[0], 2), np.int64)
    rc = lib().utri_count_batch(h, pa, int(a.shape[0]), method,
                                out.ctypes.data_as(C.POINTER(C.c_int64)), _stream(stream))
    _check(rc, "utri_count_batch")
    return out


def utri_enumerate(h, t, method=UTRI_PRUNED, which=UTRI_BOTH, sorted=True, cap=None,
                   stream=None):
    """(balanced, unbalanced) CUDA int32 tensors of shape [k, 3] (original vertex ids).

    Without `cap` the library is probed with capacities 0 first: it counts, reports the
    sizes, and the call at those sizes fills from the counts it kept."""
    torch = _torch()
    cb, cu = (0, 0) if cap is None else (int(cap[0]), int(cap[1]))
    bal = torch.empty((max(cb, 1), 3), dtype=torch.int32, device="cuda")
    unb = torch.empty((max(cu, 1), 3), dtype=torch.int32, device="cuda")
    counts = (C.c_int64 * 2)()
    rc = lib().utri_enumerate(h, float(t), method, which, C.c_void_p(bal.data_ptr()), cb,
                              C.c_void_p(unb.data_ptr()), cu, counts, 1 if sorted else 0,
                              _stream(stream))
    if rc == UTRI_E_CAPACITY:
        if cap is not None and counts[0] <= cb and counts[1] <= cu:
            _check(rc, "utri_enumerate")
        return utri_enumerate(h, t, method, which, sorted, (counts[0], counts[1]), stream)
    _check(rc, "utri_enumerate")
    return bal[:counts[0]], unb[:counts[1]]


def utri_expected(h, stream=None):
    E = C.c_double()
    _check(lib().utri_expected(h, C.byref(E), _stream(stream)), "utri_expected")
    return E.value


def utri_expected_grad(h, out=None, stream=None):
    torch = _torch()
    m = utri_graph_info(h)["m"]
    if out is None:
        out = torch.empty(m, dtype=torch.float64, device="cuda")
    _check(lib().utri_expected_grad(h, C.c_void_p(out.data_ptr()), _stream(stream)),
           "utri_expected_grad")
    return out


def utri_edge_local(h, ts, eids, stream=None):
    torch = _torch()
    a, pa = _f64_array(ts)
    e = torch.as_tensor(eids, dtype=torch.int64).to("cuda").contiguous()
    out = torch.zeros((e.shape[0], a.shape[0], 2), dtype=torch.int64, device="cuda")
    rc = lib().utri_edge_local(h, pa, int(a.shape[0]), C.c_void_p(e.data_ptr()),
                               int(e.shape[0]), C.c_void_p(out.data_ptr()), _stream(stream))
    _check(rc, "utri_edge_local")
    return out


def utri_vertex_local(h, ts, vids, stream=None):
    torch = _torch()
    a, pa = _f64_array(ts)
    v = torch.as_tensor(vids, dtype=torch.int64).to("cuda").contiguous()
    out = torch.zeros((v.shape[0], a.shape[0], 2), dtype=torch.int64, device="cuda")
    rc = lib().utri_vertex_local(h, pa, int(a.shape[0]), C.c_void_p(v.data_ptr()),
                                 int(v.shape[0]), C.c_void_p(out.data_ptr()), _stream(stream))
    _check(rc, "utri_vertex_local")
    return out


def utri_sign_worlds(h, worlds, seed, stream=None):
    """Balanced triangles in each sampled sign world: int64 CUDA tensor [worlds]."""
    torch = _torch()
    out = torch.empty(int(worlds), dtype=torch.int64, device="cuda")
    rc = lib().utri_sign_worlds(h, int(worlds), C.c_uint64(seed), C.c_void_p(out.data_ptr()),
                                _stream(stream))
    _check(rc, "utri_sign_worlds")
    return out


def utri_topk(h, k, which, stream=None):
    """(triples [r,3] int32, s [r] f64) CUDA tensors of the top-k search, r <= k."""
    torch = _torch()
    tri = torch.empty((max(int(k), 1), 3), dtype=torch.int32, device="cuda")
    sv = torch.empty(max(int(k), 1), dtype=torch.float64, device="cuda")
    cnt = C.c_int64(0)
    rc = lib().utri_topk(h, int(k), int(which), C.c_void_p(tri.data_ptr()),
                         C.c_void_p(sv.data_ptr()), C.byref(cnt), _stream(stream))
    _check(rc, "utri_topk")
    r = int(cnt.value)
    return tri[:r], sv[:r]


def utri_sample(h, ts, k, worlds, seed, scheme=UTRI_SAMPLE_EDGE, stream=None):
    torch = _torch()
    a, pa = _f64_array(ts)
    est = torch.empty((int(worlds), a.shape[0], 2), dtype=torch.float64, device="cuda")
    rc = lib().utri_sample(h, pa, int(a.shape[0]), int(k), int(worlds), C.c_uint64(seed),
                           int(scheme), C.c_void_p(est.data_ptr()), _stream(stream))
    _check(rc, "utri_sample")
    return est


def utri_batch(h, ts, k, worlds, seed, use_graph=True, exact=None, est=None, want_exact=True,
               want_est=True, stream=None):
    """(exact [nt,2] int64, est [worlds,nt,2] f64) CUDA tensors from one persistent launch."""
    torch = _torch()
    a, pa = _f64_array(ts)
    nt = a.shape[0]
    if want_exact and exact is None:
        exact = torch.empty((nt, 2), dtype=torch.int64, device="cuda")
    if want_est and est is None:
        est = torch.empty((int(worlds), nt, 2), dtype=torch.float64, device="cuda")
    pe = C.c_void_p(exact.data_ptr()) if want_exact else C.c_void_p()
    ps = C.c_void_p(est.data_ptr()) if want_est else C.c_void_p()
    rc = lib().utri_batch(h, pa, nt, int(k), int(worlds), C.c_uint64(seed), pe, ps,
                          1 if use_graph else 0, _stream(stream))
    _check(rc, "utri_batch")
    return (exact if want_exact else None), (est if want_est else None)


def utri_autotune(h, t, cache_path=None, stream=None):
    cp = cache_path.encode() if cache_path else None
    _check(lib().utri_autotune(h, float(t), cp, _stream(stream)), "utri_autotune")


def utri_set_walk_order(h, order):
    _check(lib().utri_set_walk_order(h, int(order)), "utri_set_walk_order")


def utri_get_tuning(h):
    """dict of the handle's launch parameters (names in TUNE_NAMES)."""
    out = (C.c_int64 * len(TUNE_NAMES))()
    _check(lib().utri_get_tuning(h, out), "utri_get_tuning")
    return dict(zip(TUNE_NAMES, [int(x) for x in out]))


def utri_set_tuning(h, **kw):
    """Set some launch parameters by name; the others keep their current values."""
    cur = utri_get_tuning(h)
    for k, v in kw.items():
        if k not in cur:
            raise KeyError(k)
        cur[k] = int(v)
    arr = (C.c_int64 * len(TUNE_NAMES))(*[cur[k] for k in TUNE_NAMES])
    _check(lib().utri_set_tuning(h, arr), "utri_set_tuning")


def utri_walk_stats(h, t, method=UTRI_PRUNED, stream=None):
    """dict(m_c, target_elems, candidates, streamed, items) of one counting walk at t."""
    out = (C.c_int64 * 5)()
    _check(lib().utri_walk_stats(h, float(t), method, out, _stream(stream)), "utri_walk_stats")
    keys = ["m_c", "target_elems", "candidates", "streamed", "items"]
    return {k: int(v) for k, v in zip(keys, out)}


def utri_timing(h, enable):
    """(ms, launches) of the timed counting-walk kernels; enable 1 resets, 0 stops, 2 reads."""
    ms = C.c_double()
    n = C.c_int64()
    _check(lib().utri_timing(h, int(enable), C.byref(ms), C.byref(n)), "utri_timing")
    return ms.value, n.value


def utri_strerror(code):
    return lib().utri_strerror(int(code)).decode()


# ---------------------------------------------------------------- convenience wrapper

class Graph:
    """Owning wrapper around a utri_graph handle."""

    def __init__(self, src, dst, p, n, stream=None):
        self._h = utri_graph_load(src, dst, p, n, stream)
        info = utri_graph_info(self._h)
        self.n, self.m = info["n"], info["m"]
        self.self_loops, self.dups, self.max_deg = (info["self_loops_dropped"],
                                                    info["dups_merged"], info["max_deg"])
        # P+ bookkeeping for expected_balanced: a counter bumped by every set_p, and the
        # tensor (weakly referenced, with its version) the current P+ was last set from
        self._p_token = 0
        self._p_src = None
        self._p_src_version = None

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            utri_graph_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def edges(self, device=False):
        return utri_graph_edges(self._h, device)

    def set_p(self, p):
        utri_graph_set_p(self._h, p)
        self._p_token += 1
        self._p_src = None
        self._p_src_version = None

    def _set_p_from(self, p):
        """Make p (a tensor) the graph's P+ unless it already is, unchanged since."""
        src = self._p_src() if self._p_src is not None else None
        if src is not p or self._p_src_version != p._version:
            self.set_p(p.detach())
            self._p_src = weakref.ref(p)
            self._p_src_version = p._version

    def count(self, t, method=UTRI_PRUNED, which=UTRI_BOTH):
        return utri_count(self._h, t, method, which)

    def count_batch(self, ts, method=UTRI_PRUNED):
        return utri_count_batch(self._h, ts, method)

    def enumerate(self, t, method=UTRI_PRUNED, which=UTRI_BOTH, sorted=True):
        return utri_enumerate(self._h, t, method, which, sorted)

    def expected(self):
        return utri_expected(self._h)

    def expected_grad(self, out=None):
        return utri_expected_grad(self._h, out)

    def edge_local(self, ts, eids):
        return utri_edge_local(self._h, ts, eids)

    def sign_worlds(self, worlds, seed):
        return utri_sign_worlds(self._h, worlds, seed)

    def topk(self, k, which):
        return utri_topk(self._h, k, which)

    def vertex_local(self, ts, vids):
        return utri_vertex_local(self._h, ts, vids)

    def sample(self, ts, k, worlds, seed, scheme=UTRI_SAMPLE_EDGE):
        return utri_sample(self._h, ts, k, worlds, seed, scheme)

    def batch(self, ts, k, worlds, seed, use_graph=True, **kw):
        return utri_batch(self._h, ts, k, worlds, seed, use_graph, **kw)

    def autotune(self, t, cache_path=None):
        utri_autotune(self._h, t, cache_path)

    def tuning(self):
        return utri_get_tuning(self._h)

    def set_tuning(self, **kw):
        utri_set_tuning(self._h, **kw)


def _make_expected_balanced():
    torch = _torch()

    class ExpectedBalanced(torch.autograd.Function):
        """E(p) = expected number of balanced triangles; backward gives dE/dp per edge.

        forward(p, graph): p is a float64 tensor [m] of P+ in the graph's edge-id order.
        The graph's P+ is replaced by p (rows re-sorted) unless it was last set from this
        same tensor object, unmodified since; then E is computed by the walk. backward
        re-sets the graph's P+ to the forward's p if anything changed it in between
        (another forward, a direct set_p), then multiplies the edge-centric gradient
        kernel's output by the incoming gradient.
        """

        @staticmethod
        def forward(ctx, p, graph):
            graph._set_p_from(p)
            ctx.graph = graph
            ctx.token = graph._p_token
            ctx.save_for_backward(p)  # autograd rejects backward if p is modified in place
            E = graph.expected()
            return torch.tensor(E, dtype=torch.float64, device=p.device)

        @staticmethod
        def backward(ctx, gout):
            (p,) = ctx.saved_tensors
            graph = ctx.graph
            if graph._p_token != ctx.token:
                graph._set_p_from(p)
                ctx.token = graph._p_token
            g = graph.expected_grad()
            return gout.to(g.device) * g, None

    return ExpectedBalanced


_EB = None


def expected_balanced(p, graph):
    """Differentiable expected balanced-triangle count (torch.autograd.Function)."""
    global _EB
    if _EB is None:
        _EB = _make_expected_balanced()
    return _EB.apply(p, graph)
