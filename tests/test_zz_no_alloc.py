"""The no-allocation count entry point against utri_count (through the C ABI).

utri_count_noalloc runs utri_count's kernels on the library's file-scope device scratch
array instead of hipMalloc'd buffers. Results must equal utri_count's on consecutive
calls, the second on a smaller graph (the array keeps the last call's contents), and a
graph whose query needs more than the array holds is refused before any work.
"""
import ctypes as C

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
    return utri.Graph(torch.from_numpy(np.asarray(lo)).to(d), torch.from_numpy(np.asarray(hi)).to(d),
                      torch.from_numpy(np.asarray(p, np.float64)).to(d), n)


def raw_noalloc(g, t, method, which):
    out = (C.c_int64 * 2)()
    rc = utri.lib().utri_count_noalloc(g.handle, float(t), method, which, out,
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, (int(out[0]), int(out[1]))


def check_same(g, og=None):
    for t in (0.5, 0.6, 0.75, 0.9):
        for method in (utri.UTRI_PLAIN, utri.UTRI_PRUNED, utri.UTRI_PRUNED_L3):
            for which in (utri.UTRI_BOTH, utri.UTRI_BAL, utri.UTRI_UNBAL):
                rc, got = raw_noalloc(g, t, method, which)
                assert rc == utri.UTRI_OK, (t, method, which, rc)
                want = g.count(t, method, which)
                assert got == want, (t, method, which, got, want)
        if og is not None:
            assert raw_noalloc(g, t, utri.UTRI_PRUNED, utri.UTRI_BOTH)[1] == og.count(t)


def test_noalloc_count_equals_count_on_consecutive_calls():
    n1, lo1, hi1 = inputs.rmat_graph(16, seed=3)
    p1 = inputs.draw_p(lo1.shape[0], "bimodal", 5)
    n2, lo2, hi2 = inputs.chung_lu_graph()
    p2 = inputs.draw_p(lo2.shape[0], "dyadic16", 6)
    g1 = device_graph(n1, lo1, hi1, p1)
    g2 = device_graph(n2, lo2, hi2, p2)
    say("noalloc rmat16")
    check_same(g1, oracle.load(n1, lo1, hi1, p1))
    say("noalloc chung-lu 2000 (smaller, right after)")
    check_same(g2, oracle.load(n2, lo2, hi2, p2))
    say("noalloc rmat16 again")
    check_same(g1)


def test_noalloc_rejects_what_does_not_fit():
    # 3 M vertices need more than the array's 64 MiB of row prefixes and item counts
    n = 3_000_000
    lo = np.array([0, 0, 1, 5], np.int64)
    hi = np.array([1, 2, 2, n - 1], np.int64)
    g = device_graph(n, lo, hi, np.array([0.1, 0.2, 0.9, 0.5]))
    say("noalloc capacity")
    rc, _ = raw_noalloc(g, 0.6, utri.UTRI_PRUNED, utri.UTRI_BOTH)
    assert rc == utri.UTRI_E_CAPACITY
    assert g.count(0.6) == (0, 1) or g.count(0.6) == (1, 0) or g.count(0.6) == (0, 0)
    rc, _ = raw_noalloc(g, 0.3, utri.UTRI_PRUNED, utri.UTRI_BOTH)
    assert rc == utri.UTRI_E_INVALID
    # a graph that fits still works after the refusal
    n2, lo2, hi2 = inputs.rmat_graph(12, seed=3)
    p2 = inputs.draw_p(lo2.shape[0], "uniform", 1)
    g2 = device_graph(n2, lo2, hi2, p2)
    check_same(g2)
