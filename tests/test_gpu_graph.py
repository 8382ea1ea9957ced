"""The staged execute replayed from a captured HIP graph.  spt_execute_noalloc
allocates nothing and its launches record no memory operations, so a caller
can capture it on a stream (here with torch.cuda.graph) and replay it: every
replay equals the eager execute, with eager work and synchronisations between
the replays."""

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


@pytest.mark.parametrize("prec", [0, 2], ids=["f64", "split_bf16"])
def test_noalloc_execute_replays_from_a_graph(spt, prec):
    import torch
    dt = torch.float64 if prec == spt.F64 else torch.float32
    N, R = 8192, 24
    say("graph replay, prec", prec)
    p = spt.Plan("legendre", N, 1e-7).precompute()
    X = to_dev(workloads.rhs("normal", R, N, 80), dt)
    Y = torch.empty_like(X)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        p.execute_noalloc(X, Y, prec=prec)  # the first call looks up the array's address
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        p.execute_noalloc(X, Y, prec=prec)
    torch.cuda.synchronize()
    for i in range(4):
        X.copy_(to_dev(workloads.rhs("normal", R, N, 81 + i), dt))
        Y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = to_host(Y)
        ref = to_host(p.execute(X, prec=prec))
        say("  replay %d" % i)
        assert np.array_equal(got, ref), i
    del g
    p.close()
