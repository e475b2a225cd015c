"""The allocation-free Enforce HSE (mp_enforce_hse_noalloc, static device
scratch) against the context entry point mp_enforce_hse, called through the
C ABI: the same kernels, so p0 and the cutoff index must be equal bit for
bit, on calls in a row of decreasing size (the static scratch keeps the
previous call's values), and within rounding of the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1908_03634_amd import mproj
from tests.gpu_util import N, T, say

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    re = np.concatenate([[0.0], np.cumsum(rng.uniform(0.5, 1.5, n))]) / n
    rc = 0.5 * (re[:-1] + re[1:])
    rho0 = np.exp(-3.0 * rc) * (1 + 0.1 * rng.standard_normal(n))
    g = rng.uniform(0.5, 2.0, n + 1)
    return rc, rho0, g


def _noalloc(lib, rc, rho0, g, p0_base, cut, p0, jc):
    stream = torch.cuda.current_stream()
    return lib.mp_enforce_hse_noalloc(ctypes.c_void_p(stream.cuda_stream), int(rc.shape[0]),
                                      ctypes.c_void_p(rc.data_ptr()), ctypes.c_void_p(rho0.data_ptr()),
                                      ctypes.c_void_p(g.data_ptr()), p0_base, cut, ctypes.c_void_p(p0.data_ptr()),
                                      ctypes.c_void_p(jc.data_ptr()))


def test_noalloc_enforce_hse_equals_the_context_entry_point():
    lib = mproj.load_library()
    ctx = mproj.Context(16, 16, 16, bc=(1, 1, 1), precision="fp64")
    # the largest size the static scratch takes, then smaller inputs (tile
    # counts 4096, 245, 6): each call must not depend on what the last left
    for n, cut, seed in ((1 << 24, 0.02, 1), (1000003, 0.2, 2), (24385, 0.5, 3)):
        say("noalloc hse", n, cut)
        rc, rho0, g = _inputs(n, seed)
        trc, trho, tg = T(rc), T(rho0), T(g)
        ref, jref = ctx.enforce_hse(trc, trho, tg, 3.0, cut)
        p0 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        jc = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
        assert _noalloc(lib, trc, trho, tg, 3.0, cut, p0, jc) == 0
        torch.cuda.synchronize()
        assert int(jc.item()) == jref
        assert torch.equal(p0, ref)
        p_or, j_or = oracle.enforce_hse(rc, rho0, g, 3.0, cut)
        assert j_or == jref
        assert np.abs(N(p0) - p_or).max() <= 1e-12 * 3.0
        if jref < n:
            assert bool((p0[jref:] == p0[jref]).all())
    ctx.close()


def test_noalloc_enforce_hse_rejects_inputs_beyond_the_scratch():
    lib = mproj.load_library()
    n = (1 << 24) + 1
    x = torch.ones(n + 1, dtype=torch.float64, device="cuda:0")
    p0 = torch.full((n,), 5.0, dtype=torch.float64, device="cuda:0")
    jc = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
    assert _noalloc(lib, x[:n], x[:n], x, 1.0, 0.0, p0, jc) == 1
    assert b"16777216" in lib.mp_last_error(None)
    torch.cuda.synchronize()
    assert bool((p0 == 5.0).all()) and int(jc.item()) == -1
    # the binding raises with that text
    with pytest.raises(mproj.MprojError):
        mproj.enforce_hse_noalloc(x[:n], x[:n], x, 1.0, 0.0, p0, jc)
    # a valid call after the rejected one
    rc, rho0, g = _inputs(4097, 4)
    q = torch.empty(4097, dtype=torch.float64, device="cuda:0")
    mproj.enforce_hse_noalloc(T(rc), T(rho0), T(g), 2.0, 0.3, q, jc)
    torch.cuda.synchronize()
    p_or, j_or = oracle.enforce_hse(rc, rho0, g, 2.0, 0.3)
    assert int(jc.item()) == j_or and np.abs(N(q) - p_or).max() <= 1e-12 * 2.0
