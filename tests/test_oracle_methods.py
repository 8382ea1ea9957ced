"""Pins of the oracle's direct product and of its compressed (Alg. 1/3) and
transposed (Alg. 2/4) methods, against closed forms and identities."""

import numpy as np
import pytest
import scipy.fft

from oracle import compressed, direct, matrix, params, transposed

ALL_FAMS = [(matrix.CHEBYSHEV_T, {}), (matrix.LEGENDRE, {}),
            (matrix.JACOBI, dict(alpha=-0.5, beta=-0.5)), (matrix.JACOBI, dict(alpha=2.0, beta=3.0)),
            (matrix.LAGUERRE_FN, {}), (matrix.HERMITE_FN, {}), (matrix.SINE, {}),
            (matrix.COS_POWER, dict(power=2)), (matrix.COS_POWER, dict(power=5))]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ------------------------------------------------------------------ direct product
@pytest.mark.parametrize("N", [64, 4096])
def test_chebyshev_direct_is_a_dct(N):
    # sec. 2.1: at Chebyshev nodes A x is a fast DCT.  With theta_j = pi(j+1/2)/N,
    # sum_k x_k cos(k theta_j) = (DCT-III(x)_j + x_0) / 2 (SciPy's unnormalised DCT-III)
    x = np.random.default_rng(3).standard_normal(N)
    y = direct.matvec(matrix.MatrixFamily(matrix.CHEBYSHEV_T, N), x[None, :])[0]
    ref = (scipy.fft.dct(x, type=3) + x[0]) / 2.0
    np.testing.assert_allclose(y, ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("N", [64, 4096])
def test_sine_direct_is_a_dst(N):
    # the sine generator (sec. 2): with theta_j = pi(j+1/2)/N, sum_{m<N} x_m sin(m theta_j)
    # = DST-III(x')_j / 2 for x' = (x_1, ..., x_{N-1}, 0) (SciPy's unnormalised DST-III,
    # whose last input enters as (-1)^j x'_{N-1} = 0)
    x = np.random.default_rng(4).standard_normal(N)
    y = direct.matvec(matrix.MatrixFamily(matrix.SINE, N), x[None, :])[0]
    xs = np.concatenate([x[1:], [0.0]])
    ref = scipy.fft.dst(xs, type=3) / 2.0
    np.testing.assert_allclose(y, ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("s", [2, 3, 4, 5])
def test_cos_power_entries_by_power_reduction(s):
    # eq. (cosd2): cos^s(phi) = 2^(1-s) sum_{k < s/2} C(s,k) cos((s-2k) phi)
    # (+ 2^(-s) C(s, s/2) for even s), with cos(n m theta_j) = T_{|n m|}(x_j) from
    # NumPy's Chebyshev series (Clenshaw) at the node x_j = cos(theta_j); negative m too
    from math import comb
    N = 40
    fam = matrix.MatrixFamily(matrix.COS_POWER, N, power=s)
    rows = np.arange(N)
    x = np.cos(np.pi * (rows + 0.5) / N)
    ms = np.arange(-5, 60)
    ref = np.zeros((N, ms.size))
    for k in range((s + 1) // 2):
        for c, m in enumerate(ms):
            e = np.zeros(abs((s - 2 * k) * m) + 1)
            e[-1] = 1.0
            ref[:, c] += 2.0 ** (1 - s) * comb(s, k) * np.polynomial.chebyshev.chebval(x, e)
    if s % 2 == 0:
        ref += 2.0 ** (-s) * comb(s, s // 2)
    np.testing.assert_allclose(fam.block(rows, -5, 60), ref, atol=1e-12)
    # the family is two-sided (Algorithm 1), like CHEBYSHEV_T
    assert fam.two_sided and matrix.MatrixFamily(matrix.SINE, N).two_sided
    with pytest.raises(ValueError):
        matrix.MatrixFamily(matrix.COS_POWER, N, power=6)


@pytest.mark.parametrize("fam_id,kw", ALL_FAMS)
def test_direct_vs_naive_loop(fam_id, kw):
    N = 24
    fam = matrix.MatrixFamily(fam_id, N, **kw)
    X = np.random.default_rng(5).standard_normal((2, N))
    A = fam.block(np.arange(N), 0, N)
    naive = np.array([[sum(A[j, m] * X[r, m] for m in range(N)) for j in range(N)]
                      for r in range(2)])
    np.testing.assert_allclose(direct.matvec(fam, X, panel=7), naive, rtol=1e-13, atol=1e-15)
    rows = np.array([3, 0, 23])
    np.testing.assert_allclose(direct.matvec(fam, X, rows=rows), naive[:, rows], rtol=1e-13,
                               atol=1e-15)
    # the transposed product is the same matrix read by columns
    naiveT = np.array([[sum(A[j, m] * X[r, j] for j in range(N)) for m in range(N)]
                       for r in range(2)])
    np.testing.assert_allclose(direct.matvec_transposed(fam, X, panel=5), naiveT, rtol=1e-13,
                               atol=1e-15)


# ------------------------------------------------------------------ DFT convention
@pytest.mark.parametrize("N,theta", [(16, 0.5), (128, 1.3), (1000, 2.9)])
def test_row_dft_matches_geometric_series(N, theta):
    # Appendix A: (1/sqrt N) sum_j e^{i j theta} w^{jk} = (1/sqrt N)(e^{iN theta}-1)/(e^{i theta} w^k - 1),
    # w = exp(-2 pi i/N); and the cos row is the mean of the +theta and -theta series.
    # This fixes the sign and normalisation of F in eq. (1).
    k = np.arange(N)
    w = np.exp(-2j * np.pi / N)

    def yexp(t):
        return (np.exp(1j * N * t) - 1) / (np.exp(1j * t) * w ** k - 1) / np.sqrt(N)

    row = np.exp(1j * theta * np.arange(N))
    np.testing.assert_allclose(np.fft.fft(row, norm="ortho"), yexp(theta), atol=1e-12)
    ycos = (yexp(theta) + yexp(-theta)) / 2
    # the oracle's compressed rows with zeta = 0 (rectangular window, W = I)
    plan = compressed.Plan.__new__(compressed.Plan)
    plan.fam, plan.zeta = matrix.MatrixFamily(matrix.CHEBYSHEV_T, 4), 0.0
    blk = params.Block(N, 0, 0, N)
    plan.fam.block = lambda rows, m0, m1: np.cos(theta * np.arange(m0, m1))[None, :]
    np.testing.assert_allclose(compressed._spectrum(plan, blk, np.arange(1))[0], ycos,
                               atol=1e-12)


# ------------------------------------------------------------------ exact identity, eq. (comp1)
@pytest.mark.parametrize("fam_id,kw", ALL_FAMS)
@pytest.mark.parametrize("N", [8, 16, 64, 256])
def test_unthresholded_method_is_exact(fam_id, kw, N):
    # with every entry of Add kept, Add F* W^{-1} v = A_e v: the extension, window,
    # DFT convention and block bookkeeping (sec. 3) must reproduce A x exactly
    fam = matrix.MatrixFamily(fam_id, N, **kw)
    plan = compressed.Plan(fam, 1e-10, 1e-2, min_block=4)
    C = compressed.Compressed(plan, threshold=False)
    X = np.random.default_rng(7).standard_normal((3, N))
    Yd = direct.matvec(fam, X)
    assert rel(C.execute(X), Yd) <= 1e-13
    # and the transposed product of Alg. 2/4
    Fv = np.random.default_rng(8).standard_normal((2, N))
    assert rel(transposed.execute(C, Fv), direct.matvec_transposed(fam, Fv)) <= 1e-13


def test_planted_sign_error_is_caught(monkeypatch):
    # a wrong DFT sign in the execute step must break the identity above
    fam = matrix.MatrixFamily(matrix.LEGENDRE, 64)
    C = compressed.Compressed(compressed.Plan(fam, 1e-10, 1e-2, min_block=4), threshold=False)
    X = np.random.default_rng(7).standard_normal((1, 64))
    monkeypatch.setattr(compressed.np.fft, "ifft", np.fft.fft)
    with pytest.raises(AssertionError):
        assert rel(C.execute(X), direct.matvec(fam, X)) <= 1e-13


def test_planted_block_offset_error_is_caught(monkeypatch):
    # a retained range shifted by one column (reading A-5's off-by-one the other way)
    fam = matrix.MatrixFamily(matrix.LEGENDRE, 64)
    plan = compressed.Plan(fam, 1e-10, 1e-2, min_block=4)
    for b in plan.blocks:
        b.c_lo += 1
    C = compressed.Compressed(plan, threshold=False)
    X = np.random.default_rng(7).standard_normal((1, 64))
    assert rel(C.execute(X), direct.matvec(fam, X)) > 1e-3


# ------------------------------------------------------------------ threshold behaviour
def test_error_falls_with_eps1_and_scales_with_eps1_over_eps2():
    # sec. 2.2: accuracy proportional to eps1/eps2
    N = 512
    fam = matrix.MatrixFamily(matrix.LEGENDRE, N)
    X = np.random.default_rng(9).standard_normal((4, N))
    Yd = direct.matvec(fam, X)
    errs = {}
    for eps2 in (1e-3, 1e-2):
        last = np.inf
        for eps1 in (1e-5, 1e-7, 1e-9, 1e-11):
            C = compressed.Compressed(compressed.Plan(fam, eps1, eps2, min_block=16))
            e = rel(C.execute(X), Yd)
            assert e < last
            last = e
            errs[eps1, eps2] = e
            assert 1e-4 * eps1 / eps2 <= e <= 3.0 * eps1 / eps2, (eps1, eps2, e)


def test_trig_generators_compress_like_the_cosine():
    # sec. 2 / eq. (cosd2): Algorithm 1 compresses sin(m theta) and cos^s(m theta)
    # rows as it does cos(m theta): error of order eps1/eps2, and a sparsity that
    # grows with the number of tones in the row (sin: one pair +-theta, like cos;
    # cos^3: +-theta and +-3 theta, two pairs)
    N, eps1, eps2 = 512, 1e-8, 1e-2
    X = np.random.default_rng(9).standard_normal((4, N))
    kept = {}
    for name, fam in (("cos", matrix.MatrixFamily(matrix.CHEBYSHEV_T, N)),
                      ("sin", matrix.MatrixFamily(matrix.SINE, N)),
                      ("cos3", matrix.MatrixFamily(matrix.COS_POWER, N, power=3))):
        C = compressed.Compressed(compressed.Plan(fam, eps1, eps2))
        e = rel(C.execute(X), direct.matvec(fam, X))
        assert 1e-4 * eps1 / eps2 <= e <= 3.0 * eps1 / eps2, (name, e)
        kept[name] = sum(C.nnz()) / N
    assert abs(kept["sin"] - kept["cos"]) <= 0.05 * kept["cos"]
    assert 1.5 * kept["cos"] <= kept["cos3"] <= 2.2 * kept["cos"]


def test_kept_pattern_is_hermitian_and_banded():
    # real rows give conjugate-symmetric spectra (sec. 5.1), so the kept set is
    # symmetric under k <-> L-k; for the Jacobi family row n is close to a tone of
    # frequency theta_n, so its band sits near k = theta_n L / (2 pi)
    N = 1024
    fam = matrix.MatrixFamily(matrix.LEGENDRE, N)
    plan = compressed.Plan(fam, 1e-8, 1e-2)
    C = compressed.Compressed(plan)
    theta = np.arccos(fam.nodes())
    for blk, S in zip(plan.blocks, C.mats):
        S = S.tocsr()
        for n in range(0, N, 37):
            cols = S.indices[S.indptr[n]:S.indptr[n + 1]]
            mirrored = np.sort((blk.L - cols) % blk.L)
            np.testing.assert_array_equal(np.sort(cols), mirrored)
            half = cols[cols <= blk.L // 2]
            centre = theta[n] * blk.L / (2 * np.pi)
            assert half.min() - 2 <= centre <= half.max() + 2
            assert half.max() - half.min() + 1 <= 16


def test_transposed_thresholded_accuracy():
    N = 512
    fam = matrix.MatrixFamily(matrix.JACOBI, N, alpha=0.5, beta=1.5)
    C = compressed.Compressed(compressed.Plan(fam, 1e-9, 1e-2))
    Fv = np.random.default_rng(11).standard_normal((3, N))
    e = rel(transposed.execute(C, Fv), direct.matvec_transposed(fam, Fv))
    assert e <= 3e-7


@pytest.mark.parametrize("fam_id,N,kw", [(matrix.JACOBI, 400, dict(alpha=0.5, beta=1.5)),
                                         (matrix.CHEBYSHEV_T, 300, {}),
                                         (matrix.HERMITE_FN, 200, {})])
def test_transposed_is_adjoint_of_compressed(fam_id, N, kw):
    """With the threshold on, the transposed method (Alg. 2/4: sparse product,
    inverse DFT, division by the window, truncation) is the exact adjoint of
    the row-compressed method over the same blocks (sec. 3): <A_c x, f> =
    <x, A_c^T f> to rounding, while both differ from A by the compression
    error.  The two share no arithmetic beyond the stored blocks."""
    fam = matrix.MatrixFamily(fam_id, N, **kw)
    C = compressed.Compressed(compressed.Plan(fam, 1e-6, 1e-2))
    rng = np.random.default_rng(13)
    X, F = rng.standard_normal((2, N)), rng.standard_normal((2, N))
    Yf, Yt = C.execute(X), transposed.execute(C, F)
    lhs, rhs_ = np.sum(Yf * F, axis=1), np.sum(X * Yt, axis=1)
    scale = np.linalg.norm(Yf, axis=1) * np.linalg.norm(F, axis=1)
    assert np.max(np.abs(lhs - rhs_) / scale) <= 1e-13
    # ... and the threshold is on: the compressed product is not A
    Yd = direct.matvec(fam, X)
    assert rel(Yf, Yd) > 1e-12


# ------------------------------------------------------------------ Appendix A
APPA_FAMS = [(matrix.CHEBYSHEV_T, {}), (matrix.SINE, {}), (matrix.COS_POWER, dict(power=2)),
             (matrix.COS_POWER, dict(power=3))]


@pytest.mark.parametrize("fam_id,kw", APPA_FAMS)
@pytest.mark.parametrize("N,L,m_off,rows", [(100, 300, -37, [0, 1, 50, 99]),
                                            (1000, 1728, -364, [0, 687, 999])])
def test_appendix_a_row_spectra_are_the_rows_dft(fam_id, kw, N, L, m_off, rows):
    # eqs. y1-y3: the closed-form DFT of a trigonometric row equals NumPy's FFT of
    # the explicit row, including the left extras' phase (m_off < 0); row 687
    # of N = 1000 puts its tone exactly on bin 594 of L = 1728, where the
    # quotient form of the geometric series divides two rounding errors
    from oracle import appendix_a
    fam = matrix.MatrixFamily(fam_id, N, **kw)
    rows = np.array(rows)
    U = appendix_a.row_spectra(fam, rows, m_off, L)
    ref = np.fft.fft(fam.block(rows, m_off, m_off + L), axis=1, norm="ortho")
    np.testing.assert_allclose(U, ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("fam_id,kw", APPA_FAMS)
def test_appendix_a_full_convolution_is_eq_a_comp(fam_id, kw):
    # eq. conv_appendix with every window coefficient is exactly A_e W F (eq. A_comp)
    from oracle import appendix_a
    fam = matrix.MatrixFamily(fam_id, 80, **kw)
    plan = compressed.Plan(fam, 1e-7, 1e-2)
    blk = plan.blocks[0]
    rows = np.arange(0, 80, 9)
    U = appendix_a.row_spectra(fam, rows, blk.m_offset, blk.L)
    vt = appendix_a.window_spectrum(plan, blk)
    S = sum(vt[m] * np.roll(U, m, axis=1) for m in range(blk.L)) / np.sqrt(blk.L)
    ref = compressed._spectrum(plan, blk, rows)
    np.testing.assert_allclose(S, ref, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("fam_id,kw", APPA_FAMS)
@pytest.mark.parametrize("eps1", [1e-7, 1e-10])
def test_appendix_a_truncation_stays_below_the_threshold(fam_id, kw, eps1):
    # with q = 12 window coefficients each entry moves by a fraction of the
    # threshold eps1 * max (measured: at most 0.15 of it; the window's side lobes
    # stand at ~eps1 / m), so the method's error against A x stays that of the
    # FFT-built rows
    from oracle import appendix_a
    N = 512
    fam = matrix.MatrixFamily(fam_id, N, **kw)
    plan = compressed.Plan(fam, eps1, 1e-2)
    blk = plan.blocks[0]
    rows = np.arange(0, N, 11)
    S = compressed._spectrum(plan, blk, rows)
    Sa = appendix_a.spectrum(plan, blk, rows, q=12)
    mx = np.abs(S).max()
    assert np.abs(Sa - S).max() <= 0.25 * eps1 * mx
    X = np.random.default_rng(3).standard_normal((3, N))
    Yd = direct.matvec(fam, X)
    ef = rel(compressed.Compressed(plan).execute(X), Yd)
    Ya = appendix_a.compressed_method(plan, q=12).execute(X)
    assert rel(Ya, Yd) <= 1.05 * ef


# ------------------------------------------------------------------ sampled rows of the method
@pytest.mark.parametrize("fam_id,N,kw", [(matrix.LEGENDRE, 300, {}),
                                         (matrix.JACOBI, 257, dict(alpha=2.0, beta=3.0)),
                                         (matrix.HERMITE_FN, 200, {}),
                                         (matrix.LAGUERRE_FN, 240, {})])
def test_execute_rows_and_block_max_rows(fam_id, N, kw):
    """The sampled-row form of the compressed method with the block maxima of
    block_max_rows reproduces the full method's rows (shared closed-form nodes,
    which the family then uses for every entry), and block_max_rows finds each
    block's maximum."""
    import workloads
    from oracle import compressed
    fam = matrix.MatrixFamily(fam_id, N, given_nodes=workloads.shared_nodes(fam_id, N), **kw)
    plan = compressed.Plan(fam, 1e-7, 1e-2)
    full = compressed.Compressed(plan)
    X = workloads.rhs("normal", 3, N, 7)
    Y = full.execute(X)
    mrows = compressed.block_max_rows(plan, panel=64)
    for (r, m), mx in zip(mrows, full.maxabs):
        assert m == mx
    rows = np.array([0, 5, N // 2, N - 1])
    Yr, maxabs = compressed.execute_rows(plan, X, rows, [r for r, _ in mrows])
    assert maxabs == full.maxabs
    assert np.max(np.abs(Yr - Y[:, rows])) <= 1e-13 * np.max(np.abs(Y))
    # without the maximum's rows a smaller threshold keeps more entries
    Yp, maxp = compressed.execute_rows(plan, X, rows[:1])
    assert all(a <= b for a, b in zip(maxp, full.maxabs))


class _ScaledRows:
    """A family whose rows ``rows`` are multiplied by ``c`` (everything else
    delegated): scaling a row scales that row of Add = A_e W F, since the
    window and the DFT act along the columns."""

    def __init__(self, fam, rows, c):
        self._fam, self._rows, self._c = fam, np.asarray(rows), c

    def __getattr__(self, name):
        return getattr(self._fam, name)

    def block(self, rows, m0, m1):
        B = self._fam.block(rows, m0, m1)
        B[np.isin(np.asarray(rows), self._rows)] *= self._c
        return B


def _kept_per_row(fam, eps1):
    C = compressed.Compressed(compressed.Plan(fam, eps1))
    return [np.diff(m.indptr) for m in C.mats]


@pytest.mark.parametrize("fam_id,kw", [(matrix.LEGENDRE, {}), (matrix.LAGUERRE_FN, {})])
def test_threshold_is_relative_to_the_whole_block(fam_id, kw):
    # Alg. 1 step 1.3: an entry is dropped when it is below eps1 times the largest
    # entry of the (block's) matrix, one threshold for all rows.  So the kept
    # pattern is invariant under scaling the whole matrix, while scaling one row
    # up by 1e4 raises the threshold of every other row of each block and drops
    # entries there (a per-row threshold would leave the other rows unchanged).
    N, eps1, j0 = 256, 1e-7, 100
    fam = matrix.MatrixFamily(fam_id, N, **kw)
    base = _kept_per_row(fam, eps1)
    every = _kept_per_row(_ScaledRows(fam, np.arange(N), 8.0), eps1)
    for a, b in zip(base, every):
        np.testing.assert_array_equal(a, b)
    one = _kept_per_row(_ScaledRows(fam, [j0], 1e4), eps1)
    others = np.arange(N) != j0
    for a, b in zip(base, one):
        assert b[j0] >= a[j0]
        assert b[others].sum() < a[others].sum()
        assert np.all(b[others] <= a[others])
