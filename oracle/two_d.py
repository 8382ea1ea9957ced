"""The two-dimensional compression of sec. 4.2, eq. (comp_2d), as a density
measure: D'' = F W_M D W_N F for an M x N matrix D (F the unitary DFT, W the
Kaiser windows of sec. 2.1 with zeta(eps1)), beside the one-dimensional row
and column compressions D W_N F and F W_M D of the paper's figure; the
fraction of entries above eps1 times each one's maximum.

Test infrastructure only (see ``oracle/__init__``).  No extra components are
added in either direction (as in the paper's figure of the compressed
matrices): this measures how compressible the matrix itself is.
"""

import numpy as np

from . import params


def densities(D, eps1):
    """(row, column, two-dimensional) kept fractions of D at threshold eps1."""
    D = np.asarray(D, dtype=np.float64)
    M, N = D.shape
    z = params.zeta_of_eps(eps1)
    wM = params.kaiser(np.arange(M), M - 1, z)
    wN = params.kaiser(np.arange(N), N - 1, z)
    row = np.fft.fft(D * wN[None, :], axis=1, norm="ortho")
    col = np.fft.fft(wM[:, None] * D, axis=0, norm="ortho")
    both = np.fft.fft(np.fft.fft(wM[:, None] * D * wN[None, :], axis=0, norm="ortho"), axis=1,
                      norm="ortho")

    def kept(S):
        a = np.abs(S)
        return float(np.mean(a > eps1 * a.max()))

    return kept(row), kept(col), kept(both)
