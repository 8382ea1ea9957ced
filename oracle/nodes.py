"""Quadrature nodes (and Christoffel weights) for every matrix family.

Test infrastructure only (see ``oracle/__init__``).

Nodes of sec. 5.2 (Gauss-Jacobi quadrature) and of the configurations:
Chebyshev-Gauss (closed form), Gauss-Jacobi / Gauss-Legendre, Gauss-Laguerre
and Gauss-Hermite.  The Gauss nodes are the eigenvalues of the symmetric
tridiagonal Jacobi matrix of the orthonormal three-term recurrence (DLMF 3.5.31,
Golub-Welsch), computed by LAPACK through ``scipy.linalg.eigvalsh_tridiagonal``
and then polished by Newton steps on the degree-N orthogonal polynomial
evaluated by the same recurrence.  The Christoffel weights of the orthonormal
Jacobi system are lambda_j = 1 / sum_{k<N} p_k(x_j)^2.

Order: the Jacobi family is returned with x descending (theta = arccos x
ascending, as x_n = cos(n pi / N) in sec. 2.1); Laguerre and Hermite nodes
ascending.

``idx`` selects a subset of node indices (in the returned order), so that
sampled rows of very large matrices cost O(N) per row.
"""

import math

import numpy as np
from scipy.linalg import eigvalsh_tridiagonal

from . import entries


def chebyshev_gauss(N, idx=None):
    """x_j = cos(pi (j + 1/2) / N), j = 0 .. N-1 (descending)."""
    j = np.arange(N) if idx is None else np.asarray(idx)
    return np.cos(np.pi * (2 * j + 1) / (2.0 * N))


def _eig_subset(diag, off, idx_ascending):
    """Selected eigenvalues (by ascending index) of a symmetric tridiagonal matrix."""
    idx_ascending = np.asarray(idx_ascending)
    if idx_ascending.size == len(diag):
        return eigvalsh_tridiagonal(diag, off)[idx_ascending]
    out = np.empty(idx_ascending.size)
    # contiguous runs keep the number of LAPACK calls small
    order = np.argsort(idx_ascending)
    sidx = idx_ascending[order]
    start = 0
    while start < sidx.size:
        stop = start
        while stop + 1 < sidx.size and sidx[stop + 1] == sidx[stop] + 1:
            stop += 1
        vals = eigvalsh_tridiagonal(diag, off, select="i",
                                    select_range=(int(sidx[start]), int(sidx[stop])))
        out[order[start:stop + 1]] = vals
        start = stop + 1
    return out


def _newton(x, value_and_derivative, iters=8):
    """Newton polish x <- x - p_N(x)/p_N'(x), stopping at relative change 2 ulp."""
    x = np.array(x, dtype=np.float64)
    for _ in range(iters):
        p, dp = value_and_derivative(x)
        dx = p / dp
        x = x - dx
        if np.all(np.abs(dx) <= 4.0 * np.finfo(float).eps * np.maximum(np.abs(x), 1e-300)):
            break
    return x


def gauss_jacobi(N, alpha, beta, idx=None):
    """Gauss-Jacobi nodes, x descending."""
    a, b = entries.jacobi_coefficients(N, alpha, beta)
    j = np.arange(N) if idx is None else np.asarray(idx)
    x0 = _eig_subset(b[:N], a[1:N], N - 1 - j)
    return _newton(x0, lambda x: entries.jacobi_pn_dpn(N, alpha, beta, x))


def christoffel_weights(N, alpha, beta, x):
    """lambda_j = 1 / sum_{k=0}^{N-1} p_k(x_j)^2 for the orthonormal Jacobi system."""
    P = entries.jacobi_orthonormal(alpha, beta, x, 0, N)
    return 1.0 / np.sum(P * P, axis=1)


def gauss_laguerre(N, idx=None):
    """Gauss-Laguerre nodes (alpha = 0), ascending."""
    k = np.arange(N, dtype=np.float64)
    j = np.arange(N) if idx is None else np.asarray(idx)
    x0 = _eig_subset(2.0 * k + 1.0, k[1:], j)
    x = _newton(x0, lambda x: entries.laguerre_ln_dln(N, x))
    # one Newton correction with L_N evaluated in double-double (see entries)
    p, dp = entries.laguerre_ln_dln_dd(N, x)
    return x - p / dp


def gauss_hermite(N, idx=None):
    """Gauss-Hermite nodes, ascending."""
    k = np.arange(N, dtype=np.float64)
    j = np.arange(N) if idx is None else np.asarray(idx)
    x0 = _eig_subset(np.zeros(N), np.sqrt(k[1:] / 2.0), j)
    return _newton(x0, lambda x: entries.hermite_hn_dhn(N, x))


def jacobi_mu0(alpha, beta):
    """Integral of the Jacobi weight (1-x)^alpha (1+x)^beta over [-1, 1]."""
    return math.exp((alpha + beta + 1.0) * math.log(2.0) + math.lgamma(alpha + 1.0)
                    + math.lgamma(beta + 1.0) - math.lgamma(alpha + beta + 2.0))
