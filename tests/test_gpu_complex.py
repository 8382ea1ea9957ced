"""The complex generators on the device (through the C ABI) against the oracle:
exp(i m theta_j) at the Chebyshev-Gauss angles (sec. 2) and the
spectral-domain Laguerre matrix C (sec. 4.1, eq. lag_matrix), Algorithm 1
(y = A x) and Algorithm 2 (the Laguerre coefficients V = C^T F).

Bars: float64 against the oracle's compressed method on the same plan (the
oracle's row phases passed to the library for C) at 1e-12 per right-hand
side, and against the direct product within the oracle's own compression
error + 1e-12; float32 (transforms in float64 arithmetic) against float64 at
1e-6."""

import numpy as np
import pytest

from oracle import compressed, direct, matrix, transposed
from tests.helpers import REDUCED_TOL, rel_rows, say

pytestmark = pytest.mark.gpu

CASES = [("cexp", 256, 1e-12, {}), ("cexp", 1000, 1e-10, {}), ("cexp", 3000, 1e-7, {}),
         ("laguerre_spectral", 501, 1e-10, dict(eta=2500.0, period=4.0)),
         ("laguerre_spectral", 1200, 1e-7, dict(eta=100.0, period=4.0)),
         ("laguerre_spectral", 2048, 1e-7, dict(eta=100.0, period=4.0)),
         ("laguerre_spectral", 40, 1e-12, dict(eta=1.0, period=30.0))]
FAM = {"cexp": matrix.CEXP, "laguerre_spectral": matrix.LAGUERRE_SPECTRAL}


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2004_11610_amd as m
    return m


def crhs(R, N, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal((R, N)) + 1j * g.standard_normal((R, N))


def dev(X, dt):
    import torch
    return torch.as_tensor(np.ascontiguousarray(X)).to(dtype=dt, device="cuda")


def host(Y):
    import torch
    torch.cuda.synchronize()
    return Y.to(torch.complex128).cpu().numpy()


@pytest.mark.parametrize("R", [1, 5, 33])
@pytest.mark.parametrize("fam,N,eps,kw", CASES)
def test_complex_vs_oracle(spt, fam, N, eps, kw, R):
    import torch
    say("complex", fam, N, eps, kw, "R =", R)
    ofam = matrix.MatrixFamily(FAM[fam], N, eta=kw.get("eta", 1.0), period=kw.get("period", 1.0))
    nodes = ofam.nodes() if fam == "laguerre_spectral" else None
    p = spt.Plan(fam, N, eps, nodes=nodes, **kw).precompute()
    info = p.info()
    assert info["is_complex"] == 1 and info["n_blocks"] == 1 and info["tail"] == 0
    comp = compressed.Compressed(compressed.Plan(ofam, eps, 1e-2))
    assert [b.as_tuple() for b in comp.plan.blocks] == p.blocks()
    X = crhs(R, N, 100 + R)
    Yc, Ft_c = comp.execute(X), transposed.execute(comp, X)
    Yd, Ftd = direct.matvec(ofam, X), direct.matvec_transposed(ofam, X)
    e_cd, e_tcd = rel_rows(Yc, Yd), rel_rows(Ft_c, Ftd)
    Y = host(p.execute(dev(X, torch.complex128), prec=spt.F64))
    Ft = host(p.execute_transposed(dev(X, torch.complex128), prec=spt.F64))
    e, et = rel_rows(Y, Yc), rel_rows(Ft, Ft_c)
    say("  F64 vs oracle-C %.2e (transposed %.2e); oracle-C vs direct %.2e / %.2e; nnz/row %.1f"
        % (e, et, e_cd, e_tcd, info["nnz"] / N))
    assert e <= 1e-12 and et <= 1e-12
    assert rel_rows(Y, Yd) <= e_cd + 1e-12
    assert rel_rows(Ft, Ftd) <= e_tcd + 1e-12
    Y32 = host(p.execute(dev(X, torch.complex64), prec=spt.F32))
    F32 = host(p.execute_transposed(dev(X, torch.complex64), prec=spt.F32))
    e32, et32 = rel_rows(Y32, Y), rel_rows(F32, Ft)
    say("  F32 vs F64 %.2e (transposed %.2e)" % (e32, et32))
    assert e32 <= REDUCED_TOL and et32 <= REDUCED_TOL


def test_complex_refusals(spt):
    import torch
    say("complex refusals")
    p = spt.Plan("cexp", 300, 1e-8).precompute()
    x = torch.zeros((1, 300), dtype=torch.complex64, device="cuda")
    with pytest.raises(spt.SptError) as e:
        p.execute(x, torch.empty_like(x), prec=spt.SPLIT_BF16)
    assert e.value.code in (-5, -1)
    with pytest.raises(spt.SptError) as e:
        spt.execute_batched([p], [x], [torch.empty_like(x)], prec=spt.F32)
    assert e.value.code == -5
    big = spt.Plan("cexp", 9000, 1e-7)
    with pytest.raises(spt.SptError) as e:   # L beyond one workgroup's transform
        big.precompute()
    assert e.value.code == -5
