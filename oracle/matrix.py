"""The special-function matrices A[j, m] of the configurations, row by row.

Test infrastructure only (see ``oracle/__init__``).

family          A[j, m]                                    nodes x_j
CHEBYSHEV_T     T_m(x_j) = cos(m theta_j)   eq. (cheb_matrix)   Chebyshev-Gauss, descending
SINE            sin(m theta_j)              sec. 2            Chebyshev-Gauss angles
COS_POWER       cos(m theta_j)^s, s=2..5    eq. (cosd2)       Chebyshev-Gauss angles
LEGENDRE        sqrt(lambda_j) p_m(x_j)     sec. 5.2          Gauss-Legendre, descending
JACOBI          sqrt(lambda_j) p_m^{(a,b)}(x_j)  sec. 5.2     Gauss-Jacobi, descending
LAGUERRE_FN     l_m(x_j) = exp(-x_j/2) L_m(x_j)   sec. 4      Gauss-Laguerre, ascending
HERMITE_FN      psi_m(x_j)                                    Gauss-Hermite, ascending
CEXP            exp(i m theta_j)            sec. 2            Chebyshev-Gauss angles (complex)
LAGUERRE_SPECTRAL  C[j, m] of eq. (lag_matrix)  sec. 4.1      row j: wave number k_j = 2 pi j / T,
                (-eta/2 - i k_j)^m / (eta/2 - i k_j)^(m+1)     phase phi_j (complex)

p_m is the orthonormal Jacobi polynomial and lambda_j the Christoffel weight, so
the LEGENDRE/JACOBI matrix is orthogonal (B^{-1} = B^T, sec. 5.2).  With
``orthonormal=False`` the sqrt(lambda_j) factor is left out.  Column m may run
past N-1 (the right extras of a block are the continued recurrence) and, for
the trigonometric generators only (CHEBYSHEV_T, SINE, COS_POWER), below 0 (the
left extras of Algorithm 1).
"""

import numpy as np

from . import entries, nodes

CHEBYSHEV_T, LEGENDRE, JACOBI, LAGUERRE_FN, HERMITE_FN, SINE, COS_POWER = 1, 2, 3, 4, 5, 6, 7
CEXP, LAGUERRE_SPECTRAL = 8, 9
FAMILY_NAMES = {CHEBYSHEV_T: "chebyshev_t", LEGENDRE: "legendre", JACOBI: "jacobi",
                LAGUERRE_FN: "laguerre_fn", HERMITE_FN: "hermite_fn", SINE: "sine",
                COS_POWER: "cos_power", CEXP: "cexp", LAGUERRE_SPECTRAL: "laguerre_spectral"}
TRIG = (CHEBYSHEV_T, SINE, COS_POWER)
COMPLEX = (CEXP, LAGUERRE_SPECTRAL)


class MatrixFamily:
    """``given_nodes``: the N nodes x_j to use instead of the family's quadrature
    nodes (the same entry formulas at other points; the Christoffel weights of
    the Jacobi family are then those of the given points).  The trigonometric
    generators always take the Chebyshev-Gauss angles."""

    def __init__(self, family, N, alpha=0.0, beta=0.0, orthonormal=True, power=2,
                 given_nodes=None, eta=1.0, period=1.0):
        if family == LEGENDRE:
            alpha, beta = 0.0, 0.0
        if family == COS_POWER and power not in (2, 3, 4, 5):
            raise ValueError("cos power s must be 2, 3, 4 or 5")
        self.family, self.N, self.power = family, N, int(power)
        self.alpha, self.beta, self.orthonormal = float(alpha), float(beta), bool(orthonormal)
        self.eta, self.period = float(eta), float(period)
        self._x = {}
        self._lam = {}
        if given_nodes is not None:
            if family in TRIG or family == CEXP:
                raise ValueError("the trigonometric generators take no nodes")
            x = np.array(given_nodes, dtype=np.float64)
            if x.shape != (N,) or not np.all(np.isfinite(x)):
                raise ValueError("need N finite nodes")
            self._x["all"] = x

    @property
    def two_sided(self):
        """Algorithm 1 (extras on both sides) applies only where m < 0 is defined."""
        return self.family in TRIG or self.family in COMPLEX

    @property
    def is_complex(self):
        return self.family in COMPLEX

    def _compute_nodes(self, rows):
        f, N = self.family, self.N
        if f in TRIG or f == CEXP:
            return nodes.chebyshev_gauss(N, rows)
        if f == LAGUERRE_SPECTRAL:   # the row phases phi_j
            return entries.laguerre_spectral_phase(rows, self.eta, self.period)
        if f in (LEGENDRE, JACOBI):
            return nodes.gauss_jacobi(N, self.alpha, self.beta, rows)
        if f == LAGUERRE_FN:
            return nodes.gauss_laguerre(N, rows)
        if f == HERMITE_FN:
            return nodes.gauss_hermite(N, rows)
        raise ValueError("unknown family %r" % (f,))

    def nodes(self, rows=None):
        """Nodes x_j for the selected rows; all N nodes are computed (once) when the
        selection is large, single nodes otherwise."""
        rows = np.arange(self.N) if rows is None else np.asarray(rows)
        if "all" in self._x:
            return self._x["all"][rows]
        if rows.size * 8 >= self.N:
            self._x["all"] = self._compute_nodes(np.arange(self.N))
            return self._x["all"][rows]
        return self._compute_nodes(rows)

    def weights(self, rows=None):
        """Christoffel weights lambda_j of the Jacobi family at the selected nodes."""
        rows = np.arange(self.N) if rows is None else np.asarray(rows)
        if "all" in self._lam:
            return self._lam["all"][rows]
        if rows.size * 8 >= self.N:
            self._lam["all"] = nodes.christoffel_weights(self.N, self.alpha, self.beta,
                                                         self.nodes())
            return self._lam["all"][rows]
        return nodes.christoffel_weights(self.N, self.alpha, self.beta, self.nodes(rows))

    def block(self, rows, m0, m1):
        """A[rows, m0:m1] as a dense float64 array."""
        rows = np.asarray(rows)
        f = self.family
        if f == CHEBYSHEV_T:
            return entries.chebyshev_t(rows, self.N, m0, m1)
        if f == SINE:
            return entries.sine(rows, self.N, m0, m1)
        if f == COS_POWER:
            return entries.cos_power(rows, self.N, m0, m1, self.power)
        if f == CEXP:
            return entries.cexp(rows, self.N, m0, m1)
        if f == LAGUERRE_SPECTRAL:
            return entries.laguerre_spectral(rows, self.eta, self.period, m0, m1,
                                             phi=self.nodes(rows))
        if m0 < 0:
            raise ValueError("negative degrees are defined only for the trigonometric generators")
        x = self.nodes(rows)
        if f in (LEGENDRE, JACOBI):
            P = entries.jacobi_orthonormal(self.alpha, self.beta, x, m0, m1)
            if self.orthonormal:
                P *= np.sqrt(self.weights(rows))[:, None]
            return P
        if f == LAGUERRE_FN:
            return entries.laguerre_fn(x, m0, m1)
        return entries.hermite_fn(x, m0, m1)
