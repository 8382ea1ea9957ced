"""Appendix A: the fast precomputation of the compressed rows of the
trigonometric generators, float64.

Test infrastructure only (see ``oracle/__init__``).

A compressed row is the DFT of a windowed row, F(u . w) = (F u) * (F w) with
the circular convolution (X * Y)_k = L^{-1/2} sum_m X_m Y_{(k-m) mod L}
(eq. conv_appendix).  F u has a closed form for every k (the geometric series
of eq. y3, from which eqs. y1 and y2 follow: cos and sin are the halves of two
exponentials), and F w, the window's spectrum, is concentrated near m = 0, so
the convolution keeps only the 2q + 1 window coefficients m = -q .. q.

Rows here are the block's columns m_off .. m_off + L - 1 (Algorithm 1: m_off =
-s), u_c = g((c + m_off) theta_j), so each exponential carries the phase
exp(i t m_off theta_j).  The generators are sums of tones:
  cos(m theta)    = (e^{i m theta} + e^{-i m theta}) / 2
  sin(m theta)    = (e^{i m theta} - e^{-i m theta}) / (2i)
  cos^s(m theta)  = 2^{1-s} sum_{k < s/2} C(s,k) cos((s-2k) m theta)
                    (+ 2^{-s} C(s, s/2) for even s)
Truncating F w is an approximation: the Kaiser window ends at 1/I0(zeta) =
eps1, so its spectrum's side lobes stand at about eps1 / m; with q = 12 the
dropped terms move an entry by at most ~0.15 eps1 max|Add|, below the
threshold, and the method's error against A x stays that of the FFT-built
rows (parity unpinned against the paper's own figure of 1e-15 for about 24
terms, which these windows do not reach).
"""

from math import comb

import numpy as np

from . import matrix


def tones(fam):
    """[(t, c, kind)]: the generator as sum_t c * cos or sin (t m theta)."""
    if fam.family == matrix.CHEBYSHEV_T:
        return [(1, 1.0, "cos")]
    if fam.family == matrix.SINE:
        return [(1, 1.0, "sin")]
    if fam.family == matrix.COS_POWER:
        s = fam.power
        out = [(s - 2 * k, 2.0 ** (1 - s) * comb(s, k), "cos") for k in range((s + 1) // 2)]
        if s % 2 == 0:
            out.append((0, 2.0 ** (-s) * comb(s, s // 2), "cos"))
        return out
    raise ValueError("Appendix A covers the trigonometric generators only")


def geometric(phi, L):
    """G_k(phi) = L^{-1/2} sum_{c<L} e^{i c phi} w^{ck}, w = e^{-2 pi i/L}, for k = 0 .. L-1
    (eq. y3; phi is an array of one angle per row, the result rows x L).

    The sum of e^{i c x}, x = phi - 2 pi k / L, is written as the Dirichlet
    kernel e^{i (L-1) x/2} sin(L x/2) / sin(x/2) (L at x = 0), with x reduced
    into [-pi, pi): the quotient of eq. y3, (e^{i L x} - 1) / (e^{i x} - 1),
    divides two rounding errors when phi falls on a bin."""
    k = np.arange(L)
    x = np.asarray(phi, dtype=np.float64)[:, None] - 2.0 * np.pi * k[None, :] / L
    x = x - 2.0 * np.pi * np.round(x / (2.0 * np.pi))
    with np.errstate(divide="ignore", invalid="ignore"):
        d = np.sin(L * x / 2.0) / np.sin(x / 2.0)
    d = np.where(x == 0.0, float(L), d)
    return np.exp(0.5j * (L - 1) * x) * d / np.sqrt(L)


def row_spectra(fam, rows, m_off, L):
    """F u for the rows' u_c = g((c + m_off) theta_j), c < L, by the closed forms."""
    theta = np.pi * (2 * np.asarray(rows) + 1) / (2.0 * fam.N)
    U = np.zeros((len(theta), L), dtype=np.complex128)
    for t, c, kind in tones(fam):
        ph = np.exp(1j * t * m_off * theta)[:, None]
        gp, gm = geometric(t * theta, L), geometric(-t * theta, L)
        if kind == "cos":
            U += c * (ph * gp + np.conj(ph) * gm) / 2.0
        else:
            U += c * (ph * gp - np.conj(ph) * gm) / 2j
    return U


def window_spectrum(plan, blk):
    """F w of the block's Kaiser window (one FFT per block, O(L log L))."""
    return np.fft.fft(plan.window(blk), norm="ortho")


def spectrum(plan, blk, rows, q=12):
    """Add[rows, :] by Appendix A: L^{-1/2} sum_{|m| <= q} (F w)_m (F u)_{(k-m) mod L}.

    The rows are real, so their spectra are conjugate-symmetric (sec. 5.1): the
    entries k = 0 .. L/2 are evaluated and k > L/2 is their mirror, so that the
    threshold keeps k and L - k together (evaluated separately, the two closed
    forms round differently)."""
    L = blk.L
    U = row_spectra(plan.fam, rows, blk.m_offset, L)
    vt = window_spectrum(plan, blk)
    S = np.zeros_like(U)
    for m in range(-q, q + 1):
        S += vt[m % L] * np.roll(U, m, axis=1)
    S /= np.sqrt(L)
    h = L // 2
    S[:, L - np.arange(1, (L + 1) // 2)] = np.conj(S[:, np.arange(1, (L + 1) // 2)])
    if L % 2 == 0:
        S[:, h] = S[:, h].real
    S[:, 0] = S[:, 0].real
    return S


def compressed_method(plan, q=12, threshold=True):
    """Algorithm 1 with its compressed rows from Appendix A."""
    from . import compressed
    return compressed.Compressed(plan, threshold=threshold,
                                 spectrum=lambda p, b, r: spectrum(p, b, r, q))
