"""The staged executes replayed from captured HIP graphs.  spt_execute_noalloc
allocates nothing and its launches record no memory operations, so a caller
can capture it on a stream (here with torch.cuda.graph) and replay it; a
staged batch of plans (spt_execute_batched) is captured the same way once a
first call has built its work lists.  Every replay equals the eager result,
with eager work and synchronisations between the replays."""

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


@pytest.mark.parametrize("prec", [0, 2], ids=["f64", "split_bf16"])
def test_batch_replays_from_a_graph(spt, prec):
    import torch
    dt = torch.float64 if prec == spt.F64 else torch.float32
    specs = [("legendre", 4096, 8), ("chebyshev_t", 3000, 5), ("laguerre_fn", 2000, 3)]
    say("batched graph replay, prec", prec)
    plans = [spt.Plan(f, n, 1e-7).precompute() for f, n, _ in specs]
    Xs = [to_dev(workloads.rhs("normal", r, n, 90 + i), dt) for i, (_, n, r) in enumerate(specs)]
    Ys = [torch.empty_like(x) for x in Xs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    spt.execute_batched(plans, Xs, Ys, prec=prec, stream=s)  # builds the batch's work lists
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        spt.execute_batched(plans, Xs, Ys, prec=prec, stream=s)
    torch.cuda.synchronize()
    for k in range(4):
        for i, (x, (_, n, r)) in enumerate(zip(Xs, specs)):
            x.copy_(to_dev(workloads.rhs("normal", r, n, 100 + 10 * k + i), dt))
        for y in Ys:
            y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [to_host(y) for y in Ys]
        refs = [torch.empty_like(y) for y in Ys]
        spt.execute_batched(plans, Xs, refs, prec=prec)
        torch.cuda.synchronize()
        say("  replay %d" % k)
        for a, b in zip(got, refs):
            assert np.array_equal(a, to_host(b)), k
    del g
    for p in plans:
        p.close()
