"""Pins of the oracle's nodes, weights and matrix entries.

Independent references: SciPy's quadrature routines (another implementation),
mpmath at 50 digits (brute force at N <= 16 and large arguments), and the
discrete orthogonality the paper relies on (sec. 5.2: B^{-1} = B^T)."""

import math

import mpmath
import numpy as np
import pytest
from scipy.special import roots_hermite, roots_jacobi, roots_laguerre, roots_legendre

from oracle import entries, matrix, nodes

JACOBI_AB = [(0.0, 0.0), (-0.5, -0.5), (0.5, 1.5), (2.0, 3.0)]


# ------------------------------------------------------------------ nodes vs SciPy
@pytest.mark.parametrize("N", [5, 16, 64, 256])
def test_gauss_legendre_vs_scipy(N):
    x = nodes.gauss_jacobi(N, 0.0, 0.0)
    xs, ws = roots_legendre(N)
    assert np.all(np.diff(x) < 0)                                   # descending
    np.testing.assert_allclose(x[::-1], xs, atol=4e-16, rtol=0)
    lam = nodes.christoffel_weights(N, 0.0, 0.0, x)
    # SciPy's own weights carry 1e-12 (N = 64) to 1e-10 (N = 256) relative error;
    # the precision pin is the 50-digit closed form below (ours held to 2e-13)
    np.testing.assert_allclose(lam[::-1], ws, rtol=5e-10)


def test_gauss_legendre_weights_closed_form():
    # lambda_j = 2 / ((1 - x_j^2) P_N'(x_j)^2) at the roots of P_N, in 40 digits
    N = 64
    x = nodes.gauss_jacobi(N, 0.0, 0.0)
    lam = nodes.christoffel_weights(N, 0.0, 0.0, x)
    with mpmath.workdps(40):
        for j in range(0, N, 3):
            r = mpmath.findroot(lambda t: mpmath.legendre(N, t), mpmath.mpf(x[j]), tol=1e-30)
            d = mpmath.diff(lambda t: mpmath.legendre(N, t), r)
            ref = 2 / ((1 - r * r) * d * d)
            assert abs(float((lam[j] - ref) / ref)) <= 2e-13


@pytest.mark.parametrize("ab", JACOBI_AB)
@pytest.mark.parametrize("N", [7, 100])
def test_gauss_jacobi_vs_scipy(N, ab):
    a, b = ab
    x = nodes.gauss_jacobi(N, a, b)
    xs, ws = roots_jacobi(N, a, b)
    np.testing.assert_allclose(x[::-1], xs, atol=2e-15, rtol=0)
    lam = nodes.christoffel_weights(N, a, b, x)
    np.testing.assert_allclose(lam[::-1], ws, rtol=5e-10)
    assert lam.sum() == pytest.approx(nodes.jacobi_mu0(a, b), rel=1e-13)


@pytest.mark.parametrize("N", [8, 64, 200])
def test_gauss_laguerre_hermite_vs_scipy(N):
    xl = nodes.gauss_laguerre(N)
    np.testing.assert_allclose(xl, roots_laguerre(N)[0], rtol=1e-13)
    xh = nodes.gauss_hermite(N)
    np.testing.assert_allclose(xh, roots_hermite(N)[0], rtol=1e-13, atol=1e-14)


def test_node_subset_matches_full_set():
    for fam_id, kw in [(matrix.LEGENDRE, {}), (matrix.JACOBI, dict(alpha=2.0, beta=3.0)),
                       (matrix.LAGUERRE_FN, {}), (matrix.HERMITE_FN, {})]:
        fam = matrix.MatrixFamily(fam_id, 300, **kw)
        full = fam._compute_nodes(np.arange(300))
        pick = np.array([0, 1, 150, 151, 299, 7])
        sub = fam._compute_nodes(pick)
        # Newton on the recurrence determines a node to ~1e-13 relative (its
        # evaluation noise near the small Laguerre roots); subsets agree to that
        np.testing.assert_allclose(sub, full[pick], rtol=1e-12, atol=0)


# ------------------------------------------------------------------ brute force, mpmath
mpmath.mp.dps = 50


def _mp_jacobi(n, a, b, x):
    """P_n^{(a,b)}(x) by the explicit finite sum (DLMF 18.5.8)."""
    a, b = mpmath.mpf(a), mpmath.mpf(b)
    return sum(mpmath.binomial(n + a, n - s) * mpmath.binomial(n + b, s)
               * ((x - 1) / 2) ** s * ((x + 1) / 2) ** (n - s) for s in range(n + 1))


def _mp_laguerre(n, x):
    """L_n(x) = sum_k binom(n, k) (-x)^k / k! (DLMF 18.5.12, alpha = 0)."""
    return sum(mpmath.binomial(n, k) * (-x) ** k / mpmath.factorial(k) for k in range(n + 1))


def _mp_hermite(n, x):
    """H_n(x) = n! sum_m (-1)^m (2x)^(n-2m) / (m! (n-2m)!) (DLMF 18.5.13)."""
    return mpmath.factorial(n) * sum((-1) ** m * (2 * x) ** (n - 2 * m)
                                     / (mpmath.factorial(m) * mpmath.factorial(n - 2 * m))
                                     for m in range(n // 2 + 1))


def _mp_orthonormal_jacobi(n, a, b, x):
    a, b = mpmath.mpf(a), mpmath.mpf(b)
    if n == 0:   # the general norm formula is 0/0 at n = 0 when a + b = -1
        h = 2 ** (a + b + 1) * mpmath.gamma(a + 1) * mpmath.gamma(b + 1) / mpmath.gamma(a + b + 2)
    else:
        h = (2 ** (a + b + 1) / (2 * n + a + b + 1) * mpmath.gamma(n + a + 1)
             * mpmath.gamma(n + b + 1) / (mpmath.gamma(n + a + b + 1) * mpmath.factorial(n)))
    return _mp_jacobi(n, a, b, x) / mpmath.sqrt(h)


def _mp_entry(fam, x, j, m):
    f = fam.family
    if f == matrix.CHEBYSHEV_T:
        return mpmath.cos(m * mpmath.acos(x))
    if f in (matrix.LEGENDRE, matrix.JACOBI):
        return _mp_orthonormal_jacobi(m, fam.alpha, fam.beta, x)
    if f == matrix.LAGUERRE_FN:
        return mpmath.exp(-x / 2) * _mp_laguerre(m, x)
    return (mpmath.exp(-x * x / 2) * _mp_hermite(m, x)
            / mpmath.sqrt(2 ** m * mpmath.factorial(m) * mpmath.sqrt(mpmath.pi)))


def _mp_poly(fam, N):
    f = fam.family
    if f in (matrix.LEGENDRE, matrix.JACOBI):
        return lambda t: _mp_jacobi(N, fam.alpha, fam.beta, t)
    if f == matrix.LAGUERRE_FN:
        return lambda t: _mp_laguerre(N, t)
    return lambda t: _mp_hermite(N, t)


FAMS16 = [(matrix.CHEBYSHEV_T, {}), (matrix.LEGENDRE, {}),
          (matrix.JACOBI, dict(alpha=-0.5, beta=-0.5)), (matrix.JACOBI, dict(alpha=0.5, beta=1.5)),
          (matrix.JACOBI, dict(alpha=2.0, beta=3.0)), (matrix.LAGUERRE_FN, {}),
          (matrix.HERMITE_FN, {})]


@pytest.mark.parametrize("fam_id,kw", FAMS16)
@pytest.mark.parametrize("N", [4, 9, 16])
def test_brute_force_small(fam_id, kw, N):
    fam = matrix.MatrixFamily(fam_id, N, **kw)
    x = fam.nodes()
    # nodes: roots of the degree-N polynomial (50-digit Newton); Newton on the
    # float64 recurrence leaves up to ~N ulp near the small Laguerre roots
    if fam_id != matrix.CHEBYSHEV_T:
        p = _mp_poly(fam, N)
        for xj in x:
            r = mpmath.findroot(p, mpmath.mpf(xj), tol=1e-30)
            assert abs(float(r) - xj) <= 2 * N * np.spacing(max(abs(xj), 1e-3))
        assert len(set(np.round(x, 12))) == N
    # entries, including extension columns m >= N (and m < 0 for Chebyshev)
    m0 = -3 if fam_id == matrix.CHEBYSHEV_T else 0
    A = fam.block(np.arange(N), m0, N + 5)
    ref = np.zeros_like(A)
    for j in range(N):
        xj = mpmath.mpf(x[j]) if fam_id != matrix.CHEBYSHEV_T else mpmath.cos(
            mpmath.pi * (2 * j + 1) / (2 * N))
        for c, m in enumerate(range(m0, N + 5)):
            v = _mp_entry(fam, xj, j, abs(m) if fam_id == matrix.CHEBYSHEV_T else m)
            if fam_id in (matrix.LEGENDRE, matrix.JACOBI):
                v = v * mpmath.sqrt(fam.weights()[j])
            ref[j, c] = float(v)
    np.testing.assert_allclose(A, ref, rtol=0, atol=2e-14 * np.abs(ref).max())


def test_scaled_recurrences_at_large_arguments():
    # exp(-x/2) underflows for x > 1417 and exp(-x^2/2) for |x| > 38.6: the scaled
    # recurrences must still give the O(1) values past the turning point.
    x = np.array([3000.0, 5000.5])
    L = entries.laguerre_fn(x, 0, 2001)
    for i, xv in enumerate(x):
        for m in (800, 1300, 2000):
            ref = mpmath.exp(-mpmath.mpf(xv) / 2) * mpmath.laguerre(m, 0, mpmath.mpf(xv))
            assert L[i, m] == pytest.approx(float(ref), rel=1e-11, abs=1e-300)
        assert np.all(np.abs(L[i]) <= 1.0 + 1e-12)          # |l_m(x)| <= 1 on x >= 0
    xh = np.array([40.0, -45.25])
    H = entries.hermite_fn(xh, 0, 1501)
    for i, xv in enumerate(xh):
        for m in (900, 1200, 1500):
            ref = (mpmath.exp(-mpmath.mpf(xv) ** 2 / 2) * mpmath.hermite(m, mpmath.mpf(xv))
                   / mpmath.sqrt(2 ** m * mpmath.factorial(m) * mpmath.sqrt(mpmath.pi)))
            assert H[i, m] == pytest.approx(float(ref), rel=1e-11, abs=1e-300)


# ------------------------------------------------------------------ discrete orthogonality
@pytest.mark.parametrize("ab", JACOBI_AB)
@pytest.mark.parametrize("N", [256, 1024])
def test_orthonormal_jacobi_matrix_is_orthogonal(N, ab):
    # sec. 5.2: with Gauss-Jacobi nodes and weights the matrix B is orthogonal
    fam = matrix.MatrixFamily(matrix.JACOBI, N, alpha=ab[0], beta=ab[1])
    A = fam.block(np.arange(N), 0, N)
    err = np.abs(A.T @ A - np.eye(N)).max()
    assert err <= 1e-13 * math.sqrt(N) * (1 + max(ab))


@pytest.mark.parametrize("N", [64, 1000])
def test_chebyshev_gauss_orthogonality(N):
    A = matrix.MatrixFamily(matrix.CHEBYSHEV_T, N).block(np.arange(N), 0, N)
    G = A.T @ A
    ref = np.diag(np.full(N, N / 2.0))
    ref[0, 0] = N
    np.testing.assert_allclose(G, ref, atol=1e-10 * N)


@pytest.mark.parametrize("N", [20, 64])
def test_laguerre_hermite_function_orthogonality(N):
    # Gauss quadrature (SciPy's weights) is exact to degree 2N-1
    xl, wl = roots_laguerre(N)
    L = entries.laguerre_fn(nodes.gauss_laguerre(N), 0, N)
    G = (L * (wl * np.exp(xl))[:, None]).T @ L
    np.testing.assert_allclose(G, np.eye(N), atol=1e-11)
    xh, wh = roots_hermite(N)
    H = entries.hermite_fn(nodes.gauss_hermite(N), 0, N)
    G = (H * (wh * np.exp(xh * xh))[:, None]).T @ H
    np.testing.assert_allclose(G, np.eye(N), atol=1e-11)


# ------------------------------------------------------------------ large-N Laguerre roots
def _mp_laguerre_rec(n, x):
    """L_n(x) and L_{n-1}(x) by the three-term recurrence
    (k+1) L_{k+1} = (2k+1-x) L_k - k L_{k-1}, in mpmath arithmetic."""
    l0, l1 = mpmath.mpf(1), 1 - x
    for k in range(1, n):
        l0, l1 = l1, ((2 * k + 1 - x) * l1 - k * l0) / (k + 1)
    return l1, l0


@pytest.mark.slow
@pytest.mark.parametrize("N", [1024, 4096])
def test_gauss_laguerre_large_n_vs_mpmath(N):
    """Roots of L_N at N >= 1024 (the smallest, where the float64 recurrence has
    a near double root at 0 and the oracle takes a double-double Newton step; a
    middle one; the largest) against Newton iterations in 80-digit arithmetic:
    the 80-digit root lies in a sign change of L_N and agrees with the oracle's
    to 4 ulp."""
    idx = [0, 1, 2, N // 2, N - 2, N - 1]
    x = nodes.gauss_laguerre(N, idx)
    with mpmath.workdps(80):
        for j, xj in zip(idx, x):
            r = mpmath.mpf(xj)
            for _ in range(30):
                ln, lm = _mp_laguerre_rec(N, r)
                d = N * (ln - lm) / r          # L_N' = N (L_N - L_{N-1}) / x
                step = ln / d
                r -= step
                if abs(step) <= mpmath.mpf(10) ** -60 * abs(r):
                    break
            delta = r * mpmath.mpf(10) ** -12
            assert _mp_laguerre_rec(N, r - delta)[0] * _mp_laguerre_rec(N, r + delta)[0] < 0
            assert abs(float(r) - xj) <= 4 * np.spacing(float(r)), (j, float(r), xj)
