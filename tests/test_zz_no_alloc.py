"""spt_execute_noalloc (the workspace in the library's static device array)
against spt_execute, through the C ABI: the same kernels, so the same bits,
on two calls in a row (the second with fewer right-hand sides and a smaller
plan), and its refusals (workspace beyond the array, plans it does not run)."""

import ctypes

import numpy as np
import pytest

import workloads
from tests.helpers import say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2004_11610_amd as m
    return m


def noalloc(spt, plan, X, Y, prec):
    import torch
    lib = spt._lib.load()
    R = X.shape[0]
    st = lib.spt_execute_noalloc(plan.handle, ctypes.c_void_p(X.data_ptr()),
                                 ctypes.c_void_p(Y.data_ptr()), ctypes.c_int64(R),
                                 ctypes.c_int32(prec),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "split_bf16"])
def test_noalloc_matches_execute(spt, prec):
    import torch
    dt = torch.float64 if prec == spt.F64 else torch.float32
    cases = [("legendre", 16384, 64, 71), ("hermite_fn", 3000, 5, 72)]
    plans = {}
    for fam, N, R, seed in cases:
        say("noalloc", fam, N, R, "prec", prec)
        if (fam, N) not in plans:
            plans[fam, N] = spt.Plan(fam, N, 1e-7).precompute()
        p = plans[fam, N]
        X = to_dev(workloads.rhs("normal", R, N, seed), dt)
        ref = to_host(p.execute(X, prec=prec))
        Y = torch.full_like(X, float("nan"))
        assert noalloc(spt, p, X, Y, prec) == 0, spt._lib.load().spt_last_error()
        y = to_host(Y)
        assert np.array_equal(y, ref), float(np.nanmax(np.abs(y - ref)))


def test_noalloc_refusals(spt):
    import torch
    lib = spt._lib.load()
    say("noalloc refusals")
    p = spt.Plan("legendre", 16384, 1e-7, precisions=1 << spt.F64).precompute()
    info = p.info()
    # half spectra of every block, complex float64, per right-hand side
    per_rhs = 16 * sum(L // 2 + 1 for L, _, _, _ in p.blocks())
    R = spt._lib.NOALLOC_MAX_BYTES // per_rhs + 1
    X = torch.zeros((R, 16384), dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    assert noalloc(spt, p, X, Y, spt.F64) == -1
    assert b"SPT_NOALLOC_MAX_BYTES" in lib.spt_last_error()
    q = spt.Plan("legendre", 2048, 1e-7, executor=spt.EXECUTOR_PERSISTENT).precompute()
    x = torch.zeros((2, 2048), dtype=torch.float64, device="cuda")
    assert noalloc(spt, q, x, torch.empty_like(x), spt.F64) == -5
    # first block L = 37500 (P = 18750): its forward FFT runs as work-list items
    big = spt.Plan("legendre", 30000, 1e-7, precisions=1 << spt.F64).precompute()
    xb = torch.zeros((1, 30000), dtype=torch.float64, device="cuda")
    assert noalloc(spt, big, xb, torch.empty_like(xb), spt.F64) == -5
    assert info["N"] == 16384
