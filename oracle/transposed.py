"""Algorithm 2 and the block Algorithm 4, fhat = A^T f, float64, full spectrum.

Test infrastructure only (see ``oracle/__init__``).

The column-compressed matrix of Alg. 2 step 1.3 is F W A_e^T, the transpose of
the row-compressed block A_e W F (F is symmetric), so it is taken from the same
``Compressed`` object.  Computation (Alg. 2 steps 2.1-2.2, sec. 3 for blocks):
  u = Add^T f                        sparse product
  g = W^{-1} F* u                    inverse DFT, divide by the window
  keep g on the block's retained columns, discard the extras   eq. (Fe2)
  the first t degrees come from the direct product A[:, :t]^T f.
"""

import numpy as np


def execute(comp, F):
    """Fhat (R x N) with Fhat[r, m] = sum_j A[j, m] F[r, j] (the transpose, not
    the conjugate transpose, for the complex families: eq. lag_matrix's
    V = C^T F)."""
    plan = comp.plan
    cplx = plan.fam.is_complex
    F = np.atleast_2d(np.asarray(F, dtype=np.complex128 if cplx else np.float64))
    R, N = F.shape
    out = np.zeros((R, N), dtype=F.dtype)
    for blk, S in zip(plan.blocks, comp.mats):
        w = plan.window(blk)
        u = (S.T @ F.T).T                                   # (R, L)
        g = np.fft.ifft(u, axis=1, norm="ortho")            # F* u
        if cplx:
            g = g / w[None, :]
        else:
            assert np.abs(g.imag).max() <= 1e-9 * max(np.abs(g.real).max(), 1e-300)
            g = g.real / w[None, :]
        m_lo, m_hi = blk.c_lo + blk.m_offset, blk.c_hi + blk.m_offset
        out[:, m_lo:m_hi] += g[:, blk.c_lo:blk.c_hi]
    t = plan.tail
    if t:
        out[:, :t] += F @ comp.tail_matrix
    return out
