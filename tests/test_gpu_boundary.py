"""Boundary behaviour of the C ABI on the device: the allocator hook
(spt_set_allocator) owning every device buffer, and the out-of-memory path
leaving the plan valid."""

import numpy as np
import pytest

import workloads
from tests.helpers import oracle_compressed, rel_rows, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2004_11610_amd as m
    return m


def test_allocator_hook_owns_memory_and_oom_keeps_plan(spt):
    """Every buffer of a plan comes from the hook (here PyTorch's caching
    allocator) and goes back to it; a hook that returns NULL makes the
    execute that needs a larger workspace fail with SPT_E_OOM, and the same
    plan then executes correctly once memory is available again."""
    import torch
    live, calls, fail = {}, {"alloc": 0, "free": 0}, {"on": False}

    def alloc(n, stream):
        if fail["on"]:
            return 0
        ptr = torch.cuda.caching_allocator_alloc(n, stream=stream)
        calls["alloc"] += 1
        live[ptr] = n
        return ptr

    def free(ptr, stream):
        calls["free"] += 1
        live.pop(ptr)
        torch.cuda.caching_allocator_delete(ptr)

    N, eps = 2048, 1e-7
    ref = oracle_compressed("legendre", N, eps)
    spt.set_allocator(alloc, free)
    try:
        say("allocator hook: precompute", N)
        p = spt.Plan("legendre", N, eps, precisions=1 << spt.F64).precompute()
        assert calls["alloc"] > 0 and live
        X1 = workloads.rhs("normal", 3, N, 51)
        y1 = to_host(p.execute(to_dev(X1, torch.float64), prec=spt.F64))
        assert rel_rows(y1, ref.execute(X1)) <= 1e-12
        X2 = workloads.rhs("normal", 200, N, 52)
        x2 = to_dev(X2, torch.float64)
        Y2 = torch.empty_like(x2)
        fail["on"] = True
        say("allocator hook: NULL for the larger workspace")
        with pytest.raises(spt.SptError) as e:
            p.execute(x2, Y2, prec=spt.F64)
        assert e.value.code == -4
        fail["on"] = False
        y2 = to_host(p.execute(x2, Y2, prec=spt.F64))
        assert rel_rows(y2, ref.execute(X2)) <= 1e-12
        torch.cuda.synchronize()
        p.close()
        assert not live and calls["free"] == calls["alloc"]
    finally:
        spt.set_allocator()


def test_precompute_oom_keeps_plan(spt):
    """A hook out of memory during the precomputation: SPT_E_OOM, the plan is
    not precomputed but valid, and precomputes once memory returns."""
    import torch
    fail = {"on": True}

    def alloc(n, stream):
        return 0 if fail["on"] else torch.cuda.caching_allocator_alloc(n, stream=stream)

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    spt.set_allocator(alloc, free)
    try:
        say("allocator hook: precompute out of memory")
        p = spt.Plan("legendre", 1024, 1e-7, precisions=1 << spt.F64)
        with pytest.raises(spt.SptError) as e:
            p.precompute()
        assert e.value.code == -4 and p.info()["precomputed"] == 0
        fail["on"] = False
        p.precompute()
        X = workloads.rhs("normal", 2, 1024, 53)
        y = to_host(p.execute(to_dev(X, torch.float64), prec=spt.F64))
        assert rel_rows(y, oracle_compressed("legendre", 1024, 1e-7).execute(X)) <= 1e-12
        p.close()
    finally:
        spt.set_allocator()
