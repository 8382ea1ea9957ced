"""The plain definition y = A x, dense float64 (the paper's direct method).

Test infrastructure only (see ``oracle/__init__``).

X holds one right-hand side per row (R x N, RHS-major); the result Y is
R x len(rows), Y[r, j] = sum_m A[j, m] X[r, m].  A is generated in row panels so
that large N never holds the whole matrix; ``rows`` restricts the product to a
sample of output rows (each costs O(N) to generate and O(N R) to apply).
"""

import numpy as np


def matvec(fam, X, rows=None, panel=1024):
    cplx = getattr(fam, "is_complex", False)
    X = np.atleast_2d(np.asarray(X, dtype=np.complex128 if cplx else np.float64))
    rows = np.arange(fam.N) if rows is None else np.asarray(rows)
    Y = np.empty((X.shape[0], rows.size), dtype=X.dtype)
    for p in range(0, rows.size, panel):
        A = fam.block(rows[p:p + panel], 0, fam.N)
        Y[:, p:p + panel] = X @ A.T
    return Y


def matvec_transposed(fam, F, cols=None, panel=1024):
    """fhat = A^T f: fhat[r, m] = sum_j A[j, m] F[r, j] for degrees m in ``cols``."""
    cplx = getattr(fam, "is_complex", False)
    F = np.atleast_2d(np.asarray(F, dtype=np.complex128 if cplx else np.float64))
    cols = np.arange(fam.N) if cols is None else np.asarray(cols)
    out = np.zeros((F.shape[0], cols.size), dtype=F.dtype)
    lo, hi = int(cols.min()), int(cols.max()) + 1
    for p in range(0, fam.N, panel):
        rows = np.arange(p, min(p + panel, fam.N))
        A = fam.block(rows, lo, hi)[:, cols - lo]
        out += F[:, rows] @ A
    return out
