"""Pins of the oracle's complex generators (CPU, no GPU):

* exp(i m theta_j) at the Chebyshev-Gauss angles (sec. 2, after Algorithm 2):
  the product A x is a zero-padded DFT of length 2N, y_j = sum_m (x_m
  e^{i pi m / 2N}) e^{2 pi i m j / 2N};
* the spectral-domain Laguerre matrix C of sec. 4.1 (eq. lag_matrix):
  - its entries equal the powers of eq. (main_formula2), (-eta/2 - i k)^m /
    (eta/2 - i k)^(m+1), computed with 40-digit mpmath;
  - they solve the Laguerre-transformed advection equations (eq.
    advection_laguerre3) mode by mode: (eta/2 - i k) v_0 = 1 and
    (eta/2 - i k) v_m = (-eta/2 - i k) v_(m-1);
  - the closed form printed after eq. (main_formula2), i exp(-i m phi) /
    (eta/2 - i k), differs from them by the factor i at m = 0 (the reading
    taken: main_formula2 defines C);
* for both: the unthresholded compressed method and its transpose equal the
  direct products (eq. comp1, Alg. 2), the error of the thresholded method
  falls with eps1 at fixed eps2, and each row keeps a narrow band around its
  tone's frequency theta L / 2 pi (mod L).
"""

import mpmath
import numpy as np
import pytest

from oracle import compressed, direct, entries, matrix, transposed

LAG = dict(eta=100.0, period=4.0)


def rhs(R, N, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal((R, N)) + 1j * g.standard_normal((R, N))


def test_cexp_product_is_a_padded_dft():
    N = 512
    X = rhs(3, N, 1)
    Y = direct.matvec(matrix.MatrixFamily(matrix.CEXP, N), X)
    m = np.arange(N)
    xt = np.zeros((3, 2 * N), dtype=complex)
    xt[:, :N] = X * np.exp(1j * np.pi * m / (2 * N))[None, :]
    ref = np.fft.ifft(xt, axis=1)[:, :N] * (2 * N)
    assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("eta,T", [(100.0, 4.0), (2500.0, 4.0), (1.0, 30.0)])
def test_laguerre_spectral_entries_vs_main_formula2(eta, T):
    N = 16
    C = entries.laguerre_spectral(np.arange(N), eta, T, 0, N)
    with mpmath.workdps(40):
        for j in range(N):
            k = 2 * mpmath.pi * j / T
            a, b = -mpmath.mpf(eta) / 2 - 1j * k, mpmath.mpf(eta) / 2 - 1j * k
            for m in range(N):
                ref = a ** m / b ** (m + 1)
                assert abs(complex(ref) - C[j, m]) <= 1e-14 * abs(complex(ref)), (j, m)


def test_laguerre_spectral_solves_the_transformed_advection():
    N, eta, T = 512, 500.0, 4.0
    j = np.arange(N)
    k = entries.laguerre_spectral_k(j, T)
    C = entries.laguerre_spectral(j, eta, T, 0, N)
    lhs = (0.5 * eta - 1j * k)[:, None] * C
    assert np.max(np.abs(lhs[:, 0] - 1.0)) <= 1e-13
    rec = lhs[:, 1:] - (-0.5 * eta - 1j * k)[:, None] * C[:, :-1]
    assert np.max(np.abs(rec)) <= 1e-11 * np.max(np.abs(lhs))
    # the printed closed form i exp(-i m phi) / (eta/2 - i k) misses the m = 0
    # equation by the factor i
    printed0 = 1j / (0.5 * eta - 1j * k)
    assert np.min(np.abs((0.5 * eta - 1j * k) * printed0 - 1.0)) > 1.0


def test_laguerre_spectral_phase_is_the_ratio_argument():
    j = np.arange(1, 300)
    eta, T = 300.0, 2.0
    k = entries.laguerre_spectral_k(j, T)
    ratio = (-0.5 * eta - 1j * k) / (0.5 * eta - 1j * k)
    assert np.max(np.abs(np.abs(ratio) - 1.0)) <= 1e-15
    assert np.max(np.abs(np.exp(1j * entries.laguerre_spectral_phase(j, eta, T)) - ratio)) <= 1e-14


FAMS = [(matrix.CEXP, {}), (matrix.LAGUERRE_SPECTRAL, LAG)]


@pytest.mark.parametrize("fam_id,kw", FAMS)
@pytest.mark.parametrize("N", [64, 256])
def test_unthresholded_method_is_the_product(fam_id, kw, N):
    fam = matrix.MatrixFamily(fam_id, N, **kw)
    comp = compressed.Compressed(compressed.Plan(fam, 1e-10, 1e-2), threshold=False)
    X = rhs(3, N, 2)
    Y, Yd = comp.execute(X), direct.matvec(fam, X)
    assert np.linalg.norm(Y - Yd) <= 1e-13 * np.linalg.norm(Yd)
    Ft, Fd = transposed.execute(comp, X), direct.matvec_transposed(fam, X)
    assert np.linalg.norm(Ft - Fd) <= 1e-13 * np.linalg.norm(Fd)


@pytest.mark.parametrize("fam_id,kw", FAMS)
def test_thresholded_error_falls_with_eps1(fam_id, kw):
    N = 300
    fam = matrix.MatrixFamily(fam_id, N, **kw)
    X = rhs(2, N, 3)
    Yd = direct.matvec(fam, X)
    errs = []
    for e1 in (1e-6, 1e-8, 1e-10, 1e-12):
        Y = compressed.Compressed(compressed.Plan(fam, e1, 1e-2)).execute(X)
        errs.append(np.linalg.norm(Y - Yd) / np.linalg.norm(Yd))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] <= 1e-10


@pytest.mark.parametrize("fam_id,kw", FAMS)
def test_rows_keep_a_band_at_their_tone(fam_id, kw):
    N = 400
    fam = matrix.MatrixFamily(fam_id, N, **kw)
    comp = compressed.Compressed(compressed.Plan(fam, 1e-8, 1e-2))
    (blk,), (S,) = comp.plan.blocks, comp.mats
    L = blk.L
    ang = np.pi * (2 * np.arange(N) + 1) / (2 * N) if fam_id == matrix.CEXP else fam.nodes()
    centre = np.mod(ang * L / (2 * np.pi), L)
    worst = 0
    for j in range(N):
        ks = S[j].indices
        d = np.abs(((ks - centre[j] + L / 2) % L) - L / 2)   # circular distance
        worst = max(worst, d.max())
    assert worst <= 24, worst
    assert S.nnz <= 40 * N
