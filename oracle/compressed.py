"""Algorithm 1 and the block Algorithm 3, y = A x, float64, full complex spectrum.

Test infrastructure only (see ``oracle/__init__``).

Precomputation (Alg. 1 steps 1.1-1.3; sec. 3 for blocks):
  zeta(eps1), s(zeta, eps2), block geometry            -> oracle.params
  A_e: the block's columns of the extended matrix     (Alg. 1 step 1.2, sec. 3)
  Add = A_e W F, F the unitary DFT of eq. (1)          eq. (A_comp)
  keep the entries with |Add| > eps1 * max|Add|        (Alg. 1 step 1.3; the max is
                                                        taken per block)
Computation (Alg. 1 steps 2.1-2.2; sec. 3):
  v = x on the block's retained columns, 0 on its extras       eq. (Fe1)
  y += Add F* W^{-1} v                                          eq. (comp1)
  y += A[:, :t] x[:t] for the t columns left to the direct method (sec. 3)

The whole spectrum k = 0 .. L-1 is kept and summed, and the imaginary part of
the result is checked to vanish (A and x are real); the library instead stores
half of the spectrum (sec. 5.1).  ``threshold=False`` keeps every entry, which
turns the method into an exact identity (eq. comp1).
"""

import numpy as np
import scipy.sparse as sp

from . import params


class Plan:
    def __init__(self, fam, eps1, eps2=1e-2, min_block=32, round_fft=True, direct=False):
        if not (0.0 < eps1 < eps2 < 1.0):
            raise ValueError("need 0 < eps1 < eps2 < 1")
        self.fam, self.eps1, self.eps2 = fam, eps1, eps2
        self.zeta = params.zeta_of_eps(eps1)
        if direct:
            self.blocks, self.tail = [], fam.N
        elif fam.two_sided:
            self.blocks, self.tail = params.partition_two_sided(fam.N, self.zeta, eps2, round_fft)
        else:
            self.blocks, self.tail = params.partition_one_sided(fam.N, self.zeta, eps2,
                                                               min_block, round_fft)

    def window(self, blk):
        return params.kaiser(np.arange(blk.L), blk.L - 1, self.zeta)


def _spectrum(plan, blk, rows):
    """Add[rows, :] = A_e[rows, :] W F for one block (eq. A_comp)."""
    w = plan.window(blk)
    Ae = plan.fam.block(rows, blk.m_offset, blk.m_offset + blk.L)
    return np.fft.fft(Ae * w[None, :], axis=1, norm="ortho")


class Compressed:
    """The thresholded compressed blocks Add_i (scipy CSR, N x L_i) and the tail."""

    def __init__(self, plan, threshold=True, panel=2048, spectrum=None):
        """spectrum(plan, blk, rows): the rows of Add (default: eq. A_comp by FFT;
        oracle.appendix_a gives the fast precomputation of Appendix A)."""
        self.plan = plan
        N = plan.fam.N
        self.mats, self.maxabs, self.thresholds = [], [], []
        _spectrum = spectrum or globals()["_spectrum"]
        for blk in plan.blocks:
            panels = [np.arange(p, min(p + panel, N)) for p in range(0, N, panel)]
            if len(panels) == 1:
                S = _spectrum(plan, blk, panels[0])
                mx = np.abs(S).max()
                cache = [S]
            else:
                mx = max(np.abs(_spectrum(plan, blk, r)).max() for r in panels)
                cache = None
            thr = plan.eps1 * mx if threshold else -1.0
            parts = []
            for i, r in enumerate(panels):
                S = cache[i] if cache else _spectrum(plan, blk, r)
                S[np.abs(S) <= thr] = 0.0
                parts.append(sp.csr_matrix(S))
            self.mats.append(sp.vstack(parts, format="csr"))
            self.maxabs.append(mx)
            self.thresholds.append(thr)
        t = plan.tail
        self.tail_matrix = plan.fam.block(np.arange(N), 0, t) if t > 0 else np.zeros((N, 0))

    def nnz(self):
        return [m.nnz for m in self.mats]

    def execute(self, X):
        """Y = A X^T for X of shape (R, N) (one right-hand side per row); complex
        families take and return complex X and Y."""
        cplx = self.plan.fam.is_complex
        X = np.atleast_2d(np.asarray(X, dtype=np.complex128 if cplx else np.float64))
        R, N = X.shape
        Y = np.zeros((R, N), dtype=np.complex128)
        for blk, S in zip(self.plan.blocks, self.mats):
            w = self.plan.window(blk)
            v = np.zeros((R, blk.L), dtype=X.dtype)
            m_lo, m_hi = blk.c_lo + blk.m_offset, blk.c_hi + blk.m_offset
            v[:, blk.c_lo:blk.c_hi] = X[:, m_lo:m_hi] / w[None, blk.c_lo:blk.c_hi]
            z = np.fft.ifft(v, axis=1, norm="ortho")       # F* W^{-1} v
            Y += (S @ z.T).T
        t = self.plan.tail
        if t:
            Y += X[:, :t] @ self.tail_matrix.T
        if cplx:
            return Y
        imag = np.abs(Y.imag).max() if Y.size else 0.0
        real = np.abs(Y.real).max() if Y.size else 0.0
        assert imag <= 1e-9 * max(real, 1e-300), "imaginary part does not vanish"
        return Y.real.copy()


def execute_rows(plan, X, rows, max_rows=()):
    """Rows ``rows`` of the compressed method's Y = A X^T (the full Compressed
    execute restricted to some output rows; each row costs O(L log L) per
    block).  Block i keeps |Add| > eps1 * M_i with M_i the maximum of |Add_i|
    over the rows ``rows`` and ``max_rows``: the whole block's maximum, and so
    the full method's rows, when ``max_rows`` holds the rows where it is
    attained (found once by ``block_max_rows``)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    R = X.shape[0]
    rows = np.asarray(rows)
    Y = np.zeros((R, rows.size), dtype=np.complex128)
    maxabs = []
    for blk in plan.blocks:
        S = _spectrum(plan, blk, rows)
        mx = np.abs(S).max()
        if len(max_rows):
            mx = max(mx, np.abs(_spectrum(plan, blk, np.asarray(max_rows))).max())
        maxabs.append(mx)
        S[np.abs(S) <= plan.eps1 * mx] = 0.0
        w = plan.window(blk)
        v = np.zeros((R, blk.L))
        m_lo, m_hi = blk.c_lo + blk.m_offset, blk.c_hi + blk.m_offset
        v[:, blk.c_lo:blk.c_hi] = X[:, m_lo:m_hi] / w[None, blk.c_lo:blk.c_hi]
        z = np.fft.ifft(v, axis=1, norm="ortho")       # F* W^{-1} v
        Y += z @ S.T
    t = plan.tail
    if t:
        Y += X[:, :t] @ plan.fam.block(rows, 0, t).T
    imag = np.abs(Y.imag).max() if Y.size else 0.0
    real = np.abs(Y.real).max() if Y.size else 0.0
    assert imag <= 1e-9 * max(real, 1e-300), "imaginary part does not vanish"
    return Y.real.copy(), maxabs


def block_max_rows(plan, panel=1024):
    """For every block: (row, max) where max_n,k |Add[n, k]| is attained (all
    rows, in panels; nothing is kept)."""
    N = plan.fam.N
    out = []
    for blk in plan.blocks:
        best = (-1, -1.0)
        for p in range(0, N, panel):
            rows = np.arange(p, min(p + panel, N))
            a = np.abs(_spectrum(plan, blk, rows)).max(axis=1)
            i = int(np.argmax(a))
            if a[i] > best[1]:
                best = (int(rows[i]), float(a[i]))
        out.append(best)
    return out
