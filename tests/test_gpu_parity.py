"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars (float64 throughout the oracle):
  * GPU F64 vs the oracle's compressed method on the same plan and the same
    nodes (the oracle's nodes are passed to the library): rel <= 1e-12 per
    right-hand side (the same thresholded matrix, rounding only);
  * GPU F64 vs the direct product: rel <= (oracle compressed vs direct) + 1e-12;
  * nodes computed on the device: a few ulp of the oracle's (both polish by
    Newton on the recurrence, the Laguerre roots with a double-double step);
  * F32 and split-bf16 against F64 on the same plan: rel <= 1e-6 per
    right-hand side (helpers.REDUCED_TOL).  Rounding of the half spectra is
    amplified by kappa = rms(w) rms(1/w) of the plan and grows with the FFT
    depth; the split-bf16 path therefore runs its FFTs in float64 arithmetic
    where float32 ones would move its result by more than 5e-7
    (spt_params.reduced_fft);
  * with the device's own nodes, the end-to-end product differs from the
    direct one by the compression error plus the node rounding it amplifies
    (entries near the interval ends move by ~k^2 ulp when a node moves by one).
"""

import numpy as np
import pytest

import workloads
from tests.helpers import (REDUCED_TOL, oracle_compressed, oracle_direct, oracle_family,
                           rel_rows, say, to_dev, to_host)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2004_11610_amd as m
    return m


def run(spt, plan, X, prec):
    import torch
    dt = torch.float64 if prec == spt.F64 else torch.float32
    Y = plan.execute(to_dev(X, dt), prec=prec)
    return to_host(Y)


# ------------------------------------------------------------------ precompute pieces
@pytest.mark.parametrize("fam,N,kw", [
    ("chebyshev_t", 1000, {}), ("legendre", 256, {}), ("legendre", 4096, {}),
    ("jacobi", 1000, dict(alpha=-0.5, beta=-0.5)), ("jacobi", 777, dict(alpha=2.0, beta=3.0)),
    ("laguerre_fn", 1000, {}), ("hermite_fn", 1001, {})])
def test_nodes_match_oracle(spt, fam, N, kw):
    say("nodes", fam, N, kw)
    p = spt.Plan(fam, N, 1e-7, **kw).precompute()
    x = p.nodes()
    ref = oracle_family(fam, N, kw.get("alpha", 0.0), kw.get("beta", 0.0)).nodes()
    # relative: a few ulp; absolute: the oracle's cos(pi t) carries ~eps
    # absolute error near x = 0
    tol = 8 * np.finfo(float).eps * np.abs(ref) + 4 * np.finfo(float).eps
    assert np.all(np.abs(x - ref) <= tol)


@pytest.mark.parametrize("fam,N,eps", [("legendre", 256, 1e-12), ("chebyshev_t", 512, 1e-10),
                                       ("legendre", 1000, 1e-8)])
def test_compressed_rows_match_oracle(spt, fam, N, eps):
    """Stored tiles = c_k * (kept entries of A_e W F) on the half spectrum."""
    say("compressed rows", fam, N, eps)
    p = spt.Plan(fam, N, eps, mode=spt.MODE_ROW, nodes=oracle_family(fam, N).nodes()).precompute()
    C = oracle_compressed(fam, N, eps)
    info = p.info()
    for b, (blk, S) in enumerate(zip(C.plan.blocks, C.mats)):
        P = blk.L // 2
        rows = np.arange(0, N, max(1, N // 64))
        got = np.array([p.compressed_rows(b, int(r), 1)[0] for r in rows])
        ref = S[rows].toarray()[:, : P + 1]
        ck = np.full(P + 1, 2.0)
        ck[0] = ck[P] = 1.0
        ref = ref * ck[None, :]
        scale = np.abs(ref).max()
        # the float64 recurrences drift by ~k eps near x = +-1 (k up to L)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)
        assert info["max_abs"][b] == pytest.approx(C.maxabs[b], rel=1e-12)


# ------------------------------------------------------------------ F64 against the oracle
def _check_f64(spt, fam, N, eps, X, tol=1e-12, own_nodes=False, tuning=None, **kw):
    """ROW mode unless kw says otherwise; the oracle's nodes unless own_nodes;
    launch choices `tuning` (spt_plan_set_tuning fields) if given."""
    kw.setdefault("mode", spt.MODE_ROW)
    f = oracle_family(fam, N, kw.get("alpha", 0.0), kw.get("beta", 0.0))
    nodes = None if own_nodes else f.nodes()
    p = spt.Plan(fam, N, eps, nodes=nodes, **kw).precompute()
    if tuning:
        p.set_tuning(**tuning)
    Y = run(spt, p, X, spt.F64)
    C = oracle_compressed(fam, N, eps, kw.get("eps2", 1e-2), kw.get("min_block", 32),
                          kw.get("alpha", 0.0), kw.get("beta", 0.0), kw.get("unweighted", False),
                          kw.get("power", 2))
    Yc = C.execute(X)
    Yd = oracle_direct(fam, N, X, alpha=kw.get("alpha", 0.0), beta=kw.get("beta", 0.0),
                       unweighted=kw.get("unweighted", False), power=kw.get("power", 2))
    e_c, e_d, e_cd = rel_rows(Y, Yc), rel_rows(Y, Yd), rel_rows(Yc, Yd)
    say("  rel vs oracle-C %.3e  vs direct %.3e  (oracle-C vs direct %.3e)" % (e_c, e_d, e_cd))
    if not own_nodes:
        assert e_c <= tol
    assert e_d <= e_cd + tol
    return p, Y


@pytest.mark.parametrize("fam,N,R,kw", [
    ("sine", 1000, 3, {}), ("sine", 3001, 2, {}), ("cos_power", 777, 3, dict(power=2)),
    ("cos_power", 1500, 2, dict(power=3)), ("cos_power", 1024, 1, dict(power=5))])
def test_trig_generators_fp64(spt, fam, N, R, kw):
    """sin(m theta_j) (sec. 2) and cos^s(m theta_j) (eq. cosd2) through Algorithm
    1 (extras on both sides): F64 parity with the oracle's compressed method on
    the same thresholded matrix; F32 and split-bf16 within the reduced bar."""
    say("trig generator", fam, N, R, kw)
    X = workloads.rhs("normal", R, N, 61)
    p, Y64 = _check_f64(spt, fam, N, 1e-9, X, **kw)
    assert p.blocks()[0][1] < 0  # left extras: Algorithm 1
    for prec in (spt.F32, spt.SPLIT_BF16):
        e = rel_rows(run(spt, p, X, prec), Y64)
        say("  prec", prec, "rel vs F64 %.3e" % e)
        assert e <= REDUCED_TOL


@pytest.mark.parametrize("fam,N,eps,R,kw", [
    ("chebyshev_t", 1000, 1e-9, 3, {}), ("sine", 2048, 1e-7, 2, {}),
    ("cos_power", 1500, 1e-8, 1, dict(power=3)), ("cos_power", 777, 1e-10, 2, dict(power=2))])
def test_appendix_a_precompute_fp64(spt, fam, N, eps, R, kw):
    """Appendix A (trig_conv_q = 12): the compressed rows from the closed-form
    row spectra convolved with 25 window coefficients, on the device; F64
    parity with the oracle's Appendix A method (same truncation, same
    threshold), and against A x no worse than the FFT-built rows."""
    from oracle import appendix_a, compressed
    say("appendix A", fam, N, eps, R, kw)
    f = oracle_family(fam, N, power=kw.get("power", 2))
    X = workloads.rhs("normal", R, N, 71)
    p = spt.Plan(fam, N, eps, mode=spt.MODE_ROW, trig_conv_q=12, **kw).precompute()
    Y = run(spt, p, X, spt.F64)
    oplan = compressed.Plan(f, eps, 1e-2)
    Ca = appendix_a.compressed_method(oplan, q=12)
    Yd = oracle_direct(fam, N, X, power=kw.get("power", 2))
    e_fft = rel_rows(compressed.Compressed(oplan).execute(X), Yd)
    e_a, e_d = rel_rows(Y, Ca.execute(X)), rel_rows(Y, Yd)
    say("  vs oracle Appendix A %.3e  vs direct %.3e  (FFT rows vs direct %.3e)" % (e_a, e_d, e_fft))
    # the oracle forms x = phi - 2 pi k / L in float64, so sin(L x / 2) carries an
    # absolute error of ~L u; the library reduces its angles exactly in integers.
    # A wrong tone, phase or truncation shows at the eps1 level, far above.
    assert e_a <= 1e-11
    assert e_d <= 1.05 * e_fft + 1e-12
    # the same kept set: the oracle counts the full spectrum (k and L - k), the
    # library the half (k = 0 and L/2 once)
    full = sum(Ca.nnz())
    assert abs(2 * p.info()["nnz"] - full) <= 0.01 * full + 2 * N
    for prec in (spt.F32, spt.SPLIT_BF16):
        assert rel_rows(run(spt, p, X, prec), Y) <= REDUCED_TOL


def test_legendre_256_fp64(spt):
    w = workloads.LEGENDRE_256
    say(w["name"])
    X = workloads.rhs(w["rhs"], w["nrhs"], w["N"], w["seed"])
    _check_f64(spt, "legendre", w["N"], w["eps"], X)
    say(w["name"], "own nodes")
    _check_f64(spt, "legendre", w["N"], w["eps"], X, own_nodes=True)


@pytest.mark.parametrize("w", workloads.THREE_PLANS_4096, ids=lambda w: w["name"])
def test_three_plans_4096_fp64(spt, w):
    say(w["name"], "row mode")
    fam = {1: "chebyshev_t", 2: "legendre", 4: "laguerre_fn"}[w["family"]]
    X = workloads.rhs(w["rhs"], w["nrhs"], w["N"], w["seed"])
    _check_f64(spt, fam, w["N"], w["eps"], X)
    say(w["name"], "row mode, own nodes")
    _check_f64(spt, fam, w["N"], w["eps"], X, own_nodes=True,
               tol=1e-11 if fam == "laguerre_fn" else 1e-12)


def test_laguerre_4096_auto_and_direct(spt):
    w = workloads.THREE_PLANS_4096[2]
    X = workloads.rhs(w["rhs"], 2, w["N"], w["seed"])
    say(w["name"], "direct mode")
    nodes = oracle_family("laguerre_fn", w["N"]).nodes()
    p = spt.Plan("laguerre_fn", w["N"], w["eps"], mode=spt.MODE_DIRECT, nodes=nodes).precompute()
    Yd = oracle_direct("laguerre_fn", w["N"], X)
    assert rel_rows(run(spt, p, X, spt.F64), Yd) <= 1e-12
    say(w["name"], "auto mode")
    pa = spt.Plan("laguerre_fn", w["N"], w["eps"]).precompute()
    pr = spt.Plan("laguerre_fn", w["N"], w["eps"], mode=spt.MODE_ROW).precompute()
    ia, ir = pa.info(), pr.info()
    # AUTO keeps the row compression only when it stores fewer reals than A
    row_reals = 2 * ir["stored"] + ir["tail"] * w["N"]
    assert ia["mode"] == (spt.MODE_ROW if row_reals <= w["N"] ** 2 else spt.MODE_DIRECT)
    assert rel_rows(run(spt, pa, X, spt.F64), Yd) <= 1e-6


@pytest.mark.parametrize("fam,N,eps,kw", [
    ("legendre", 17, 1e-7, {}), ("legendre", 100, 1e-9, dict(min_block=8)),
    ("chebyshev_t", 333, 1e-9, {}), ("jacobi", 1000, 1e-10, dict(alpha=0.5, beta=1.5)),
    ("jacobi", 999, 1e-8, dict(alpha=-0.5, beta=-0.5)),
    ("jacobi", 1500, 1e-7, dict(alpha=2.0, beta=3.0)),
    ("hermite_fn", 700, 1e-9, {}), ("legendre", 640, 1e-8, dict(unweighted=True)),
    ("legendre", 2000, 1e-9, dict(eps2=1e-3, min_block=16)),
])
@pytest.mark.parametrize("R", [1, 3, 65])
def test_ragged_shapes_fp64(spt, fam, N, eps, kw, R):
    say("ragged", fam, N, eps, kw, "R =", R)
    X = workloads.rhs("normal", R, N, 100 + N)
    _check_f64(spt, fam, N, eps, X, **kw)


def test_auto_mode_picks_fewest_stored_reals(spt):
    # N = 100 at eps 1e-9: the tile boxes of three blocks hold more reals than A
    say("auto mode, legendre 100")
    X = workloads.rhs("normal", 3, 100, 5)
    pa = spt.Plan("legendre", 100, 1e-9, min_block=8).precompute()
    pr = spt.Plan("legendre", 100, 1e-9, min_block=8, mode=spt.MODE_ROW).precompute()
    ir = pr.info()
    row_reals = 2 * ir["stored"] + ir["tail"] * 100
    assert pa.info()["mode"] == (spt.MODE_ROW if row_reals <= 100 ** 2 else spt.MODE_DIRECT)
    if pa.info()["mode"] == spt.MODE_DIRECT:
        assert pa.blocks() == [] and pa.info()["tail"] == 100
    Yd = oracle_direct("legendre", 100, X)
    assert rel_rows(run(spt, pa, X, spt.F64), Yd) <= 1e-6


def test_user_nodes(spt):
    say("user nodes")
    f = oracle_family("legendre", 500)
    X = workloads.rhs("normal", 4, 500, 7)
    p = spt.Plan("legendre", 500, 1e-9, nodes=f.nodes()).precompute()
    assert np.array_equal(p.nodes(), f.nodes())
    Yc = oracle_compressed("legendre", 500, 1e-9).execute(X)
    assert rel_rows(run(spt, p, X, spt.F64), Yc) <= 1e-12


# ------------------------------------------------------------------ precisions


@pytest.mark.parametrize("fam,N,eps,R,kw", [("legendre", 2048, 1e-7, 70, {}),
                                            ("chebyshev_t", 3000, 1e-7, 64, {}),
                                            ("chebyshev_t", 3000, 1e-7, 64, dict(eps2=3e-2)),
                                            ("jacobi", 1111, 1e-7, 5, dict(alpha=2.0, beta=3.0))])
def test_reduced_precisions_vs_fp64(spt, fam, N, eps, R, kw):
    say("precisions", fam, N, eps, R, kw)
    p = spt.Plan(fam, N, eps, **kw).precompute()
    X = workloads.rhs("normal", R, N, 11)
    Y64 = run(spt, p, X, spt.F64)
    tol = REDUCED_TOL
    say("  kappa %.2f tol %.2e" % (p.info()["kappa"], tol))
    for prec in (spt.F32, spt.SPLIT_BF16):
        e = rel_rows(run(spt, p, X, prec), Y64)
        say("  prec", prec, "rel vs F64 %.3e" % e)
        assert e <= tol


def test_legendre_16384_r64_all_precisions(spt):
    """The benchmark workload at full size: F64 against sampled direct rows of
    the oracle, F32 and split-bf16 against F64 on every output."""
    w = workloads.LEGENDRE_16384
    say(w["name"])
    N, R = w["N"], w["nrhs"]
    X = workloads.rhs(w["rhs"], R, N, w["seed"])
    p = spt.Plan("legendre", N, w["eps"]).precompute()
    Y64 = run(spt, p, X, spt.F64)
    rows = np.arange(0, N, 97)
    Yd = oracle_direct("legendre", N, X, rows=rows)
    e = rel_rows(Y64[:, rows], Yd)
    say("  F64 vs direct (sampled rows) %.3e" % e)
    assert e <= 1e-6           # compression error at eps1 = 1e-7, eps2 = 1e-2 is 2.4e-7
    for prec in (spt.F32, spt.SPLIT_BF16):
        e = rel_rows(run(spt, p, X, prec), Y64)
        say("  prec", prec, "rel vs F64 %.3e" % e)
        assert e <= 1e-6


@pytest.mark.parametrize("fam,N,R,kw", [("legendre", 16384, 16, {}),
                                         ("jacobi", 48785, 4, dict(alpha=2.0, beta=3.0)),
                                         ("hermite_fn", 11522, 8, dict(mode=1)),
                                         ("chebyshev_t", 3000, 8, {})])
def test_reduced_fft_arithmetic(spt, fam, N, R, kw):
    """The float32 and split-bf16 paths with float32 and with float64 FFTs
    (fused blocks, and four-step blocks beyond one workgroup) against float64:
    with float64 FFTs both stay within 1e-6; the automatic choice measured what
    it reports and chose by it."""
    say("reduced fft", fam, N, R, kw)
    X = workloads.rhs("normal", R, N, 61)
    p = spt.Plan(fam, N, 1e-7, **kw).precompute()
    info = p.info()
    Y64 = run(spt, p, X, spt.F64)
    errs = {}
    for mode in (spt.FFT_F32, spt.FFT_F64):
        q = spt.Plan(fam, N, 1e-7, reduced_fft=mode, **kw).precompute()
        assert q.info()["reduced_fft_f64"] == (mode == spt.FFT_F64)
        for prec in (spt.F32, spt.SPLIT_BF16):
            errs[mode, prec] = rel_rows(run(spt, q, X, prec), Y64)
        q.close()
    say("  kappa %.2f; vs F64: F32 %.2e / %.2e, split %.2e / %.2e (float32 / float64 FFTs); "
        "auto measured %.2e -> %d" % (info["kappa"], errs[1, 1], errs[2, 1], errs[1, 2],
                                      errs[2, 2], info["reduced_fft_f32_err"],
                                      info["reduced_fft_f64"]))
    for prec in (spt.F32, spt.SPLIT_BF16):
        assert errs[spt.FFT_F64, prec] <= REDUCED_TOL
        assert rel_rows(run(spt, p, X, prec), Y64) <= REDUCED_TOL
    assert info["reduced_fft_f32_err"] > 0
    assert info["reduced_fft_f64"] == (info["reduced_fft_f32_err"] > 7e-7)
    # without a float64 path the choice compares the two FFT arithmetics
    q = spt.Plan(fam, N, 1e-7, precisions=1 << spt.SPLIT_BF16, **kw).precompute()
    qi = q.info()
    say("  split only: measured %.2e -> %d" % (qi["reduced_fft_f32_err"], qi["reduced_fft_f64"]))
    assert qi["reduced_fft_f64"] == (qi["reduced_fft_f32_err"] > 5e-7)
    assert rel_rows(run(spt, q, X, spt.SPLIT_BF16), Y64) <= REDUCED_TOL


def test_legendre_16384_r64_transposed(spt):
    """The transposed product on the benchmark plan at full size: the adjoint
    of the forward product to rounding, F32 against F64, and the same bits
    from a second call (partial sums are added in a fixed order).  Sampled
    degrees against the direct A^T f: test_long_block_transposed."""
    import torch
    w = workloads.LEGENDRE_16384
    say(w["name"], "transposed")
    N, R = w["N"], w["nrhs"]
    X = workloads.rhs(w["rhs"], R, N, w["seed"])
    F = workloads.rhs(w["rhs"], R, N, w["seed"] + 1)
    p = spt.Plan("legendre", N, w["eps"]).precompute()
    Yf = run(spt, p, X, spt.F64)
    Fd = to_dev(F, torch.float64)
    Yt = to_host(p.execute_transposed(Fd, prec=spt.F64))
    assert np.array_equal(to_host(p.execute_transposed(Fd, prec=spt.F64)), Yt)
    lhs, rhs = np.sum(Yf * F, axis=1), np.sum(X * Yt, axis=1)
    e_adj = np.max(np.abs(lhs - rhs) / (np.linalg.norm(Yf, axis=1) * np.linalg.norm(F, axis=1)))
    e_32 = rel_rows(to_host(p.execute_transposed(to_dev(F, torch.float32), prec=spt.F32)), Yt)
    say("  adjoint %.3e  F32 vs F64 %.3e" % (e_adj, e_32))
    assert e_adj <= 1e-12
    assert e_32 <= 1e-6


# ------------------------------------------------------------------ error paths on the GPU
def test_unprepared_precision_and_overlap(spt):
    import torch
    say("error paths")
    p = spt.Plan("legendre", 256, 1e-7, precisions=1 << spt.F64).precompute()
    X = torch.zeros((1, 256), dtype=torch.float32, device="cuda")
    with pytest.raises(spt.SptError) as e:
        p.execute(X, prec=spt.F32)
    assert e.value.code == -5
    X64 = torch.zeros((2, 256), dtype=torch.float64, device="cuda")
    with pytest.raises(spt.SptError) as e:
        p.execute(X64, Y=X64)
    assert e.value.code == -1


def test_nonfinite_input_propagates(spt):
    say("nan input")
    p = spt.Plan("legendre", 512, 1e-8).precompute()
    X = workloads.rhs("normal", 2, 512, 3)
    X[1, 300] = np.nan
    Y = run(spt, p, X, spt.F64)
    assert np.all(np.isfinite(Y[0])) and np.any(np.isnan(Y[1]))


# ------------------------------------------------------------------ transposed product (Alg. 2/4)
@pytest.mark.parametrize("fam,N,eps,kw", [
    ("legendre", 256, 1e-12, {}), ("chebyshev_t", 1000, 1e-10, {}),
    ("jacobi", 1234, 1e-9, dict(alpha=0.5, beta=1.5)), ("legendre", 4096, 1e-12, {}),
    ("hermite_fn", 500, 1e-10, {}), ("sine", 900, 1e-10, {}),
    ("cos_power", 700, 1e-10, dict(power=4))])
@pytest.mark.parametrize("R", [1, 66])
def test_transposed_fp64(spt, fam, N, eps, kw, R):
    from oracle import direct, transposed
    say("transposed", fam, N, eps, kw, "R =", R)
    f = oracle_family(fam, N, kw.get("alpha", 0.0), kw.get("beta", 0.0),
                      power=kw.get("power", 2))
    p = spt.Plan(fam, N, eps, mode=spt.MODE_ROW, nodes=f.nodes(), **kw).precompute()
    F = workloads.rhs("normal", R, N, 300 + N)
    import torch
    Y = to_host(p.execute_transposed(to_dev(F, torch.float64), prec=spt.F64))
    C = oracle_compressed(fam, N, eps, 1e-2, 32, kw.get("alpha", 0.0), kw.get("beta", 0.0),
                          power=kw.get("power", 2))
    Yt = transposed.execute(C, F)
    Yd = direct.matvec_transposed(f, F)
    e_c, e_d, e_cd = rel_rows(Y, Yt), rel_rows(Y, Yd), rel_rows(Yt, Yd)
    say("  rel vs oracle-T %.3e  vs direct %.3e  (oracle-T vs direct %.3e)" % (e_c, e_d, e_cd))
    assert e_c <= 1e-12
    assert e_d <= e_cd + 1e-12
    Y32 = to_host(p.execute_transposed(to_dev(F, torch.float32), prec=spt.F32))
    assert rel_rows(Y32, Y) <= REDUCED_TOL


@pytest.mark.parametrize("fam,N,R", [("legendre", 300, 3), ("hermite_fn", 257, 70)])
def test_transposed_direct_mode(spt, fam, N, R):
    """A plan in DIRECT mode (the whole matrix as the direct tail, no blocks):
    the transposed product is A^T f by the tail kernel alone, against the
    oracle's direct product; F32 against F64."""
    from oracle import direct
    import torch
    say("transposed direct mode", fam, N, R)
    f = oracle_family(fam, N)
    p = spt.Plan(fam, N, 1e-7, mode=spt.MODE_DIRECT, nodes=f.nodes()).precompute()
    assert p.info()["mode"] == spt.MODE_DIRECT and p.info()["tail"] == N
    F = workloads.rhs("normal", R, N, 91)
    Y = to_host(p.execute_transposed(to_dev(F, torch.float64), prec=spt.F64))
    e = rel_rows(Y, direct.matvec_transposed(f, F))
    say("  rel vs direct %.3e" % e)
    assert e <= 1e-12
    Y32 = to_host(p.execute_transposed(to_dev(F, torch.float32), prec=spt.F32))
    assert rel_rows(Y32, Y) <= 1e-5


@pytest.mark.parametrize("fam,N,kw", [
    ("legendre", 7000, {}), ("jacobi", 9000, dict(alpha=-0.5, beta=-0.5))])
def test_transposed_four_step_fp64(spt, fam, N, kw):
    """The four-step inverse transform of the transposed product, forced on
    first blocks that also fit one workgroup (Legendre 7000: P = 4374, Jacobi
    9000: P = 5625, odd): oracle parity, and agreement with the
    single-workgroup transform."""
    from oracle import transposed
    say("transposed four-step", fam, N, kw)
    f = oracle_family(fam, N, kw.get("alpha", 0.0), kw.get("beta", 0.0))
    p = spt.Plan(fam, N, 1e-7, mode=spt.MODE_ROW, nodes=f.nodes(), **kw).precompute()
    assert p.blocks()[0][0] // 2 > 4096
    F = workloads.rhs("normal", 5, N, 77)
    import torch
    Y1 = to_host(p.execute_transposed(to_dev(F, torch.float64), prec=spt.F64))
    p.set_tuning(inv_four=spt.TUNE_ON)
    Y4 = to_host(p.execute_transposed(to_dev(F, torch.float64), prec=spt.F64))
    C = oracle_compressed(fam, N, 1e-7, 1e-2, 32, kw.get("alpha", 0.0), kw.get("beta", 0.0))
    Yt = transposed.execute(C, F)
    e_c, e_1 = rel_rows(Y4, Yt), rel_rows(Y4, Y1)
    say("  four-step vs oracle-T %.3e  vs one workgroup %.3e" % (e_c, e_1))
    assert e_c <= 1e-12 and e_1 <= 1e-13
    Y32 = to_host(p.execute_transposed(to_dev(F, torch.float32), prec=spt.F32))
    assert rel_rows(Y32, Y4) <= REDUCED_TOL


def test_long_block_transposed(spt):
    """Transposed product with a first block longer than one workgroup's FFT
    (P = 15000 > 10240, four steps): it is the adjoint of the forward product
    over the same compressed blocks, <A_c x, f> = <x, A_c^T f>, to rounding;
    sampled degrees against the direct A^T f; F32 against F64."""
    from oracle import direct
    import torch
    say("long block transposed", LONG_N)
    fam = oracle_family("legendre", LONG_N)
    p = spt.Plan("legendre", LONG_N, 1e-7, mode=spt.MODE_ROW, nodes=fam.nodes()).precompute()
    assert p.blocks()[0][0] // 2 > 10240
    X = workloads.rhs("normal", 3, LONG_N, 81)
    F = workloads.rhs("normal", 3, LONG_N, 82)
    Yf = run(spt, p, X, spt.F64)
    Yt = to_host(p.execute_transposed(to_dev(F, torch.float64), prec=spt.F64))
    lhs, rhs = np.sum(Yf * F, axis=1), np.sum(X * Yt, axis=1)
    scale = np.linalg.norm(Yf, axis=1) * np.linalg.norm(F, axis=1)
    e_adj = np.max(np.abs(lhs - rhs) / scale)
    cols = np.arange(5, LONG_N, 97)
    Yd = direct.matvec_transposed(fam, F, cols=cols)
    e_d = rel_rows(Yt[:, cols], Yd)
    say("  adjoint %.3e  vs direct (sampled degrees) %.3e" % (e_adj, e_d))
    assert e_adj <= 1e-12
    assert e_d <= 1e-6
    Y32 = to_host(p.execute_transposed(to_dev(F, torch.float32), prec=spt.F32))
    assert rel_rows(Y32, Yt) <= REDUCED_TOL


# ------------------------------------------------------------------ batched execution
def test_batched_matches_single_plans(spt):
    import torch
    specs = [("legendre", 1000, {}, 5), ("hermite_fn", 600, {}, 1),
             ("jacobi", 1500, dict(alpha=2.0, beta=3.0), 70), ("chebyshev_t", 777, {}, 3),
             ("jacobi", 2048, dict(alpha=-0.5, beta=-0.5), 130)]
    # single executes on the persistent executor too, so that results match bit for bit
    plans = [spt.Plan(f, N, 1e-7, mode=spt.MODE_ROW, executor=spt.EXECUTOR_PERSISTENT, **kw)
             .precompute() for f, N, kw, _ in specs]
    for prec, dt in ((spt.F64, torch.float64), (spt.F32, torch.float32),
                     (spt.SPLIT_BF16, torch.float32)):
        say("batched prec", prec)
        Xs = [to_dev(workloads.rhs("normal", R, N, 50 + i), dt)
              for i, (_, N, _, R) in enumerate(specs)]
        Ys = [torch.empty_like(x) for x in Xs]
        singles = [to_host(p.execute(x, prec=prec)) for p, x in zip(plans, Xs)]
        spt.execute_batched(plans, Xs, Ys, prec=prec)
        for y, ref in zip(Ys, singles):
            assert np.array_equal(to_host(y), ref)
        # replay of the recorded graph on new data in the same buffers
        for i, x in enumerate(Xs):
            x.copy_(to_dev(workloads.rhs("normal", x.shape[0], x.shape[1], 900 + i), dt))
        singles = [to_host(p.execute(x, prec=prec)) for p, x in zip(plans, Xs)]
        for rep in range(3):
            for y in Ys:
                y.zero_()
            spt.execute_batched(plans, Xs, Ys, prec=prec)
            torch.cuda.synchronize()
            for y, ref in zip(Ys, singles):
                assert np.array_equal(to_host(y), ref), rep


# ------------------------------------------------------------------ executors
@pytest.mark.parametrize("fam,N,eps,R,kw", [
    ("legendre", 7000, 1e-7, 3, {}),
    ("chebyshev_t", 5000, 1e-9, 17, {}),
    ("jacobi", 9000, 1e-7, 2, dict(alpha=-0.5, beta=-0.5))])
def test_four_step_blocks_fp64(spt, fam, N, eps, R, kw):
    """First block longer than one workgroup's FFT (P > 4096): the persistent
    executor runs it as column and row items; F64 parity with the oracle."""
    say("four-step", fam, N, eps, R, kw)
    X = workloads.rhs("normal", R, N, 21)
    p, _ = _check_f64(spt, fam, N, eps, X, executor=spt.EXECUTOR_PERSISTENT, **kw)
    assert p.blocks()[0][0] // 2 > 4096


@pytest.mark.parametrize("fam,N,R,kw", [
    ("legendre", 7000, 3, {}), ("jacobi", 9000, 1, dict(alpha=-0.5, beta=-0.5))])
def test_parity_halves_fp64(spt, fam, N, R, kw):
    """Blocks with an even P >= 4096 points go through the fused FFT as two
    workgroups, one per parity of the outputs (Legendre 7000: P = 4374); an
    odd P stays whole (Jacobi 9000: P = 5625); F64 parity with the oracle."""
    say("parity halves", fam, N, R, kw)
    X = workloads.rhs("normal", R, N, 23)
    p, _ = _check_f64(spt, fam, N, 1e-7, X, executor=spt.EXECUTOR_STAGED, **kw)
    assert p.blocks()[0][0] // 2 >= 4096


@pytest.mark.parametrize("fam,N,eps,R,kw", [
    ("legendre", 8192, 1e-7, 13, {}), ("chebyshev_t", 5000, 1e-9, 8, {})])
def test_eight_way_split(spt, fam, N, eps, R, kw):
    """A block's real transform split by output residue mod 8, five workgroups
    per right-hand side (Legendre 8192: P = 5120 with three shorter blocks in
    the same launch; Chebyshev 5000, Algorithm 1: one block, P = 4320): F64
    parity with the oracle; F32 and split-bf16 against F64 and against the
    default parity split."""
    say("eight-way split", fam, N, eps, R, kw)
    X = workloads.rhs("normal", R, N, 27)
    p, Y64 = _check_f64(spt, fam, N, eps, X, executor=spt.EXECUTOR_STAGED,
                        tuning=dict(fft_half=spt.FFT_EIGHT), **kw)
    assert p.blocks()[0][0] // 2 >= 4096 and (p.blocks()[0][0] // 2) % 4 == 0
    for prec in (spt.F32, spt.SPLIT_BF16):
        p.set_tuning(fft_half=spt.FFT_EIGHT)
        Ye = run(spt, p, X, prec)
        p.set_tuning(fft_half=spt.TUNE_ON)
        Yh = run(spt, p, X, prec)
        e, eh = rel_rows(Ye, Y64), rel_rows(Ye, Yh)
        say("  prec %d: vs F64 %.3e, vs parity split %.3e" % (prec, e, eh))
        assert e <= REDUCED_TOL and eh <= REDUCED_TOL


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "split_bf16"])
def test_staged_executor_matches_persistent(spt, prec):
    """The two-launch executor and the persistent one compute the same stage
    (different FFT factorisations and summation orders)."""
    say("staged vs persistent, prec", prec)
    N, R = 7000, 70
    X = workloads.rhs("normal", R, N, 31)
    a = spt.Plan("legendre", N, 1e-7, executor=spt.EXECUTOR_PERSISTENT).precompute()
    b = spt.Plan("legendre", N, 1e-7, executor=spt.EXECUTOR_STAGED).precompute()
    Ya, Yb = run(spt, a, X, prec), run(spt, b, X, prec)
    e = rel_rows(Ya, Yb)
    say("  rel %.3e" % e)
    assert e <= (1e-13 if prec == spt.F64 else REDUCED_TOL)


def test_persistent_launches_repeat_exactly(spt):
    """Counters return to zero after every launch: repeated and interleaved
    launches (two right-hand-side counts, i.e. two work queues) give identical
    results and no waits that gave up (those write NaN)."""
    import torch
    p = spt.Plan("legendre", 7000, 1e-7, executor=spt.EXECUTOR_PERSISTENT).precompute()
    Xa = to_dev(workloads.rhs("normal", 3, 7000, 41), torch.float32)
    Xb = to_dev(workloads.rhs("normal", 70, 7000, 42), torch.float32)
    ya = to_host(p.execute(Xa, prec=spt.SPLIT_BF16))
    yb = to_host(p.execute(Xb, prec=spt.SPLIT_BF16))
    assert np.all(np.isfinite(ya)) and np.all(np.isfinite(yb))
    for i in range(4):
        say("  repeat", i)
        assert np.array_equal(to_host(p.execute(Xb, prec=spt.SPLIT_BF16)), yb)
        assert np.array_equal(to_host(p.execute(Xa, prec=spt.SPLIT_BF16)), ya)


def test_persistent_wait_give_up_is_reported(spt):
    """A dependency wait that reaches its bound (set from the host to one
    tick, so every wait that is not met at once gives up) makes the launch
    drain with NaN outputs; the next persistent execute on that context
    reports it as SPT_E_HIP without running, and with the default bound the
    same context then computes the staged executor's result again."""
    import torch
    N, R = 16384, 64
    say("persistent give-up", N, R)
    X = to_dev(workloads.rhs("normal", R, N, 43), torch.float64)
    p = spt.Plan("legendre", N, 1e-7, executor=spt.EXECUTOR_PERSISTENT,
                 precisions=1 << spt.F64).precompute()
    q = spt.Plan("legendre", N, 1e-7, precisions=1 << spt.F64).precompute()
    ref = to_host(q.execute(X, prec=spt.F64))
    Y = torch.empty_like(X)
    p.execute(X, Y, prec=spt.F64)
    torch.cuda.synchronize()
    p.set_exec_wait(1)
    p.execute(X, Y, prec=spt.F64)
    torch.cuda.synchronize()
    assert np.any(np.isnan(to_host(Y)))
    with pytest.raises(spt.SptError) as e:
        p.execute(X, Y, prec=spt.F64)
    assert e.value.code == -3 and "gave up" in str(e.value)
    p.set_exec_wait(0)
    for i in range(2):
        say("  clean launch", i)
        y = to_host(p.execute(X, Y, prec=spt.F64))
        assert np.all(np.isfinite(y))
        assert rel_rows(y, ref) <= 1e-13


def test_nonfinite_precompute_is_numeric_error(spt):
    """Nodes far outside the Legendre interval overflow the recurrence: the
    precomputation stops with SPT_E_NUMERIC and leaves the plan valid but not
    precomputed."""
    import torch
    say("numeric error")
    p = spt.Plan("legendre", 64, 1e-7, mode=spt.MODE_ROW, nodes=np.full(64, 1e200))
    with pytest.raises(spt.SptError) as e:
        p.precompute()
    assert e.value.code == -6
    assert p.info()["precomputed"] == 0
    with pytest.raises(spt.SptError) as e:
        p.execute(torch.zeros((1, 64), dtype=torch.float64, device="cuda"))
    assert e.value.code == -2


# ------------------------------------------------------------------ long blocks
# first block L = 30000: P = 15000 > 10240, four-step precompute and inverse
# transforms; the staged forward FFT in parity halves of 7500 points
LONG_N = 24000


def test_long_block_precompute_sampled_rows(spt):
    """Precompute of a block whose rows do not fit one workgroup's FFT (four
    steps, float64): sampled stored rows against the oracle's A_e W F rows,
    thresholded at the library's block maximum (entries within 0.1% of the
    threshold are not compared)."""
    from oracle import compressed as oc
    say("long block precompute", LONG_N)
    fam = oracle_family("legendre", LONG_N)
    p = spt.Plan("legendre", LONG_N, 1e-7, mode=spt.MODE_ROW, nodes=fam.nodes()).precompute()
    op = oc.Plan(fam, 1e-7)
    blk = op.blocks[0]
    L = p.blocks()[0][0]
    assert L == blk.L and L // 2 > 10240
    P = L // 2
    rows = np.arange(7, LONG_N, LONG_N // 12)
    ref = oc._spectrum(op, blk, rows)[:, : P + 1]
    got = np.array([p.compressed_rows(0, int(r), 1)[0] for r in rows])
    ck = np.full(P + 1, 2.0)
    ck[0] = ck[P] = 1.0
    mx = p.info()["max_abs"][0]
    assert np.abs(ref).max() <= mx * (1 + 1e-12)
    thr = 1e-7 * mx
    keep = np.abs(ref) > thr * 1.001
    drop = np.abs(ref) < thr * 0.999
    err = np.abs(got[keep] - (ref * ck[None, :])[keep]).max() / mx
    say("  max |stored - oracle| / max %.3e over %d kept entries" % (err, int(keep.sum())))
    # the float64 recurrences drift by ~k eps near x = +-1, k up to L
    assert err <= 4 * L * np.finfo(float).eps
    assert np.all(got[drop] == 0)


@pytest.mark.parametrize("executor", ["staged", "persistent"])
def test_long_block_execute(spt, executor):
    """Execute with a first block longer than one workgroup's whole transform
    (P = 15000: parity halves in the staged executor's fused FFT, four-step
    items in the persistent one): F64 against sampled rows of the direct
    product, F32 and split-bf16 against F64."""
    say("long block execute", executor)
    ex = spt.EXECUTOR_STAGED if executor == "staged" else spt.EXECUTOR_PERSISTENT
    fam = oracle_family("legendre", LONG_N)
    p = spt.Plan("legendre", LONG_N, 1e-7, nodes=fam.nodes(), executor=ex).precompute()
    X = workloads.rhs("normal", 3, LONG_N, 61)
    Y64 = run(spt, p, X, spt.F64)
    rows = np.arange(0, LONG_N, 211)
    Yd = oracle_direct("legendre", LONG_N, X, rows=rows)
    e = rel_rows(Y64[:, rows], Yd)
    say("  F64 vs direct (sampled rows) %.3e" % e)
    assert e <= 1e-6
    for prec in (spt.F32, spt.SPLIT_BF16):
        e = rel_rows(run(spt, p, X, prec), Y64)
        say("  prec", prec, "rel vs F64 %.3e" % e)
        assert e <= REDUCED_TOL


def test_batched_staged_matches_single_plans(spt):
    """Staged batch (FFT items of every plan, then one product launch) against
    single executes of the same plans (whose FFTs may take the fused kernel:
    rounding differs)."""
    import torch
    specs = [("legendre", 1000, {}, 5), ("hermite_fn", 600, {}, 1),
             ("jacobi", 1500, dict(alpha=2.0, beta=3.0), 70), ("chebyshev_t", 777, {}, 3),
             ("jacobi", 9000, dict(alpha=-0.5, beta=-0.5), 130), ("legendre", 24000, {}, 2)]
    plans = [spt.Plan(f, N, 1e-7, mode=spt.MODE_ROW, **kw).precompute() for f, N, kw, _ in specs]
    for prec, dt in ((spt.F64, torch.float64), (spt.F32, torch.float32),
                     (spt.SPLIT_BF16, torch.float32)):
        say("staged batch prec", prec)
        Xs = [to_dev(workloads.rhs("normal", R, N, 70 + i), dt)
              for i, (_, N, _, R) in enumerate(specs)]
        Ys = [torch.full_like(x, float("nan")) for x in Xs]
        singles = [to_host(p.execute(x, prec=prec)) for p, x in zip(plans, Xs)]
        for rep in range(2):
            spt.execute_batched(plans, Xs, Ys, prec=prec)
            for p, y, ref in zip(plans, Ys, singles):
                e = rel_rows(to_host(y), ref)
                assert e <= (1e-13 if prec == spt.F64 else REDUCED_TOL), (rep, e)


@pytest.mark.parametrize("fam,N,R", [("legendre", 7000, 3), ("legendre", 16384, 64),
                                     ("legendre", LONG_N, 2), ("chebyshev_t", 3000, 130)])
def test_forced_chunks_match_per_tile(spt, fam, N, R):
    """The chunked products (split-bf16 and float64) on plans whose windows
    would fit whole (asked for: spt_tuning.product): the same bits as the
    per-tile products; a first
    block of four-step transforms (N = 24000), no direct tail (Chebyshev, one
    two-sided block), several right-hand-side chunks."""
    say("forced chunks", fam, N, R)
    p = spt.Plan(fam, N, 1e-7).set_tuning(product=spt.PRODUCT_CHUNKED).precompute()
    q = spt.Plan(fam, N, 1e-7).set_tuning(product=spt.PRODUCT_TILE).precompute()
    assert p.info()["window_chunked"] == 1 and q.info()["window_lds"] == 0
    if fam == "chebyshev_t":
        assert p.info()["tail"] == 0
    X = workloads.rhs("normal", R, N, 75)
    assert np.array_equal(run(spt, p, X, spt.F64), run(spt, q, X, spt.F64))
    assert np.array_equal(run(spt, p, X, spt.SPLIT_BF16), run(spt, q, X, spt.SPLIT_BF16))


def test_batch_of_windowed_plans_matches_single(spt):
    """A staged split-bf16 batch whose plans all have windows runs only the
    chunked product's items (the per-tile item list holds one padding entry);
    a plan whose FFTs are four-step items in both paths (Legendre 30000, first
    block P = 18750, longer than the fused FFT's split parts) gives the same
    bits batched, alone or beside another plan, as executed singly; with
    a plan without windows in the batch, both product launches run."""
    import torch
    say("batch of windowed plans")
    big = spt.Plan("legendre", 30000, 1e-7).precompute()
    small = spt.Plan("legendre", 1000, 1e-7).precompute()
    assert big.blocks()[0][0] // 2 > 16384
    assert big.info()["window_lds"] > 0 and small.info()["window_lds"] > 0
    Xb = to_dev(workloads.rhs("normal", 2, 30000, 75), torch.float32)
    Xs = to_dev(workloads.rhs("normal", 5, 1000, 70), torch.float32)
    ref = to_host(big.execute(Xb, prec=spt.SPLIT_BF16))
    for plans, Xl in (([big], [Xb]), ([small, big], [Xs, Xb])):
        Ys = [torch.full_like(x, float("nan")) for x in Xl]
        spt.execute_batched(plans, Xl, Ys, prec=spt.SPLIT_BF16)
        assert np.array_equal(to_host(Ys[-1]), ref)
    # with a plan that has no windows (DIRECT mode: per-tile items) in the
    # same batch, both product launches run
    dense = spt.Plan("hermite_fn", 300, 1e-7, mode=spt.MODE_DIRECT).precompute()
    assert dense.info()["window_lds"] == 0
    Xd = to_dev(workloads.rhs("normal", 70, 300, 76), torch.float32)
    refd = to_host(dense.execute(Xd, prec=spt.SPLIT_BF16))
    Ys = [torch.full_like(x, float("nan")) for x in (Xs, Xd, Xb)]
    spt.execute_batched([small, dense, big], [Xs, Xd, Xb], Ys, prec=spt.SPLIT_BF16)
    assert np.array_equal(to_host(Ys[2]), ref)
    assert rel_rows(to_host(Ys[1]), refd) <= 1e-6
    assert np.all(np.isfinite(to_host(Ys[0])))


@pytest.mark.parametrize("R", [256, 300, 513])
def test_split_product_chunks_match_alone(spt, R):
    """Right-hand sides are taken 64 per product workgroup; the first 64 of a
    larger set come out bit for bit as when executed alone (same FFTs, same
    order of the sums), and all of them within the bar of F64."""
    import torch
    say("split product chunks", R)
    p = spt.Plan("legendre", 2048, 1e-7).precompute()
    X = workloads.rhs("normal", R, 2048, 81)
    Xd = to_dev(X, torch.float32)
    Y = to_host(p.execute(Xd, prec=spt.SPLIT_BF16))
    Y64 = to_host(p.execute(Xd[:64].contiguous(), prec=spt.SPLIT_BF16))
    assert np.array_equal(Y[:64], Y64)
    e = rel_rows(Y, run(spt, p, X, spt.F64))
    say("  rel vs F64 %.3e" % e)
    assert e <= REDUCED_TOL


def test_one_plan_on_several_streams(spt):
    """Executes of one plan on different streams overlap in time; each stream
    has its own workspace, so every result equals the one-stream result."""
    import torch
    say("one plan, three streams")
    p = spt.Plan("legendre", 4096, 1e-7).precompute()
    Xs = [to_dev(workloads.rhs("normal", 64, 4096, 90 + i), torch.float32) for i in range(3)]
    ref = [to_host(p.execute(x, prec=spt.SPLIT_BF16)) for x in Xs]
    streams = [torch.cuda.Stream() for _ in range(3)]
    Ys = [torch.empty_like(x) for x in Xs]
    for rep in range(20):
        for s, x, y in zip(streams, Xs, Ys):
            with torch.cuda.stream(s):
                p.execute(x, y, prec=spt.SPLIT_BF16)
    torch.cuda.synchronize()
    for y, r in zip(Ys, ref):
        assert np.array_equal(to_host(y), r)



@pytest.mark.parametrize("rg", ["4", "2", "2w"])
@pytest.mark.parametrize("fam,N,R,kw", [
    ("legendre", 16384, 64, {}), ("legendre", 1000, 1, {}), ("legendre", 1000, 70, {}),
    ("chebyshev_t", 3000, 130, {}), ("laguerre_fn", 5000, 64, {}),
    ("laguerre_fn", 3001, 130, {}), ("hermite_fn", 2049, 17, {}),
    ("jacobi", 4100, 200, dict(alpha=-0.5, beta=0.5))])
def test_windowed_product_matches_per_tile(spt, fam, N, R, kw, rg):
    """The windowed split-bf16 product (spectra staged in LDS per group of four
    row tiles, 64 or 32 right-hand sides per workgroup; for windows too wide
    for LDS, in chunks of 32 columns) takes the same steps in the same order as
    the per-tile product, so both give the same bits (up to the sign of an
    exact zero); ragged tile groups (N not a multiple of 64), right-hand-side
    chunks with fewer columns than a workgroup's and several chunks.  rg "2w":
    windows of 64 right-hand sides with two waves per row tile."""
    say("windowed product", fam, N, R, kw, "rg", rg)
    tune = (dict(product=spt.PRODUCT_WINDOW_2W) if rg == "2w"
            else dict(window_rhs=16 * int(rg)))
    p = spt.Plan(fam, N, 1e-7, **kw).set_tuning(**tune).precompute()
    info = p.info()
    q = spt.Plan(fam, N, 1e-7, **kw).set_tuning(product=spt.PRODUCT_TILE).precompute()
    assert q.info()["window_lds"] == 0
    say("  blocks %d window LDS %d B, %d columns, chunked %d" % (
        info["n_blocks"], info["window_lds"], info["window_cols"], info["window_chunked"]))
    if fam == "legendre" and N == 16384:
        assert info["window_lds"] > 0 and info["window_chunked"] == 0
    if fam == "laguerre_fn":
        assert info["window_chunked"] == 1
    X = workloads.rhs("normal", R, N, 97)
    assert np.array_equal(run(spt, p, X, spt.SPLIT_BF16), run(spt, q, X, spt.SPLIT_BF16))
    if info["window_chunked"]:
        # the float64 product through the same chunked windows
        assert np.array_equal(run(spt, p, X, spt.F64), run(spt, q, X, spt.F64))


def test_autotuned_plan_keeps_parity(spt, tmp_path):
    """The autotuner (every launch choice timed on the device, the fastest
    kept, the result cached as JSON): the tuned plan's float64 result equals
    the oracle's compressed method at 1e-12 and its split-bf16 result stays
    within 1e-6 of float64; the cache gives the same choice without timing."""
    import torch
    from tests.helpers import oracle_compressed, oracle_family
    N, R = 4096, 32
    say("autotune", N, R)
    f = oracle_family("legendre", N)
    p = spt.Plan("legendre", N, 1e-7, mode=spt.MODE_ROW, nodes=f.nodes()).precompute()
    cache = tmp_path / "tuning.json"
    chosen, us = p.autotune(R, prec=spt.SPLIT_BF16, cache_path=cache)
    say("  chosen %s, %.1f us per execute" % (chosen, us))
    assert us > 0 and cache.exists() and p.tuning() == chosen
    X = workloads.rhs("normal", R, N, 81)
    Y64 = run(spt, p, X, spt.F64)
    assert rel_rows(Y64, oracle_compressed("legendre", N, 1e-7).execute(X)) <= 1e-12
    assert rel_rows(run(spt, p, X, spt.SPLIT_BF16), Y64) <= REDUCED_TOL
    q = spt.Plan("legendre", N, 1e-7, mode=spt.MODE_ROW, nodes=f.nodes()).precompute()
    again, us2 = q.autotune(R, prec=spt.SPLIT_BF16, cache_path=cache)
    assert again == chosen and us2 == 0.0
    assert np.array_equal(run(spt, q, X, spt.SPLIT_BF16), run(spt, p, X, spt.SPLIT_BF16))


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["f64", "f32", "split_bf16"])
def test_unaligned_input_matches_aligned(spt, prec):
    """X starting one element past an aligned address (a view into a larger
    buffer) takes the FFT's scalar loads instead of the paired or 16-byte ones:
    the same spectra, so the same result up to the product's summation (the
    same bits here)."""
    import torch
    dt = torch.float64 if prec == spt.F64 else torch.float32
    N, R = 16384, 8
    say("unaligned X, prec", prec)
    p = spt.Plan("legendre", N, 1e-7).precompute()
    Xh = workloads.rhs("normal", R, N, 99)
    buf = torch.zeros(R * N + 1, dtype=dt, device="cuda")
    buf[1:].copy_(to_dev(Xh, dt).reshape(-1))
    Xu = buf[1:].view(R, N)
    assert Xu.data_ptr() % 8 != 0 or dt == torch.float64
    ya = to_host(p.execute(to_dev(Xh, dt), prec=prec))
    yu = to_host(p.execute(Xu, prec=prec))
    e = rel_rows(yu, ya)
    say("  rel %.3e" % e)
    assert e <= (1e-14 if prec == spt.F64 else 1e-7)


@pytest.mark.parametrize("fam,N,kw", [("sine", 16384, {}), ("chebyshev_t", 16384, {}),
                                      ("cos_power", 16384, dict(power=3)),
                                      ("legendre", LONG_N, {})])
def test_transposed_reduced_long_blocks(spt, fam, N, kw):
    """The float32 transposed product on plans whose inverse transforms take
    four steps (P > 10240): within 1e-6 of float64, the float32 path running
    those transforms in float64 arithmetic where the plan chose that
    (spt_params.reduced_fft)."""
    import torch
    say("transposed float32, long blocks", fam, N, kw)
    p = spt.Plan(fam, N, 1e-7, **kw).precompute()
    assert max(L for L, _, _, _ in p.blocks()) // 2 > 10240
    X = workloads.rhs("normal", 8, N, 113)
    y64 = to_host(p.execute_transposed(to_dev(X, torch.float64), prec=spt.F64))
    y32 = to_host(p.execute_transposed(to_dev(X, torch.float32), prec=spt.F32))
    e = rel_rows(y32, y64)
    say("  rel %.3e (float64 FFTs %d)" % (e, p.info()["reduced_fft_f64"]))
    assert e <= REDUCED_TOL


@pytest.mark.parametrize("fam,N,R,kw", [("sine", 16384, 5, {}), ("legendre", 26000, 3, {}),
                                        ("legendre", LONG_N, 2, dict(fft_half=3))])
def test_fused_split_beyond_one_workgroup(spt, fam, N, R, kw):
    """First blocks longer than one workgroup's whole transform (10240 < P <=
    16384): the staged executor's forward FFT runs fused as parity halves (or
    the eight-way split), the persistent executor's as four-step items; both
    float64 results agree to 1e-12 and the float32 and split-bf16 paths stay
    within 1e-6 of float64."""
    say("fused split beyond one workgroup", fam, N, R, kw)
    tune = {k: v for k, v in kw.items() if k == "fft_half"}
    p = spt.Plan(fam, N, 1e-7).set_tuning(**tune).precompute()
    q = spt.Plan(fam, N, 1e-7, executor=spt.EXECUTOR_PERSISTENT).precompute()
    P = p.blocks()[0][0] // 2
    assert 10240 < P <= 16384
    X = workloads.rhs("normal", R, N, 131)
    y = run(spt, p, X, spt.F64)
    e = rel_rows(y, run(spt, q, X, spt.F64))
    say("  P %d staged vs persistent F64 %.3e" % (P, e))
    assert e <= 1e-12
    for prec in (spt.F32, spt.SPLIT_BF16):
        e = rel_rows(run(spt, p, X, prec), y)
        say("  prec", prec, "rel vs F64 %.3e" % e)
        assert e <= REDUCED_TOL
