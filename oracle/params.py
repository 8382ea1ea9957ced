"""Plan parameters of the extra-component method, written from the paper.

Test infrastructure only (see ``oracle/__init__``).

* Kaiser window w_n^{zeta,M}, 0 <= n <= M                      -- sec. 2.1
* zeta(eps1): root of 1/I0(zeta) = eps1 by Newton from 50     -- sec. 2.2
* s(zeta, eps2): extra components, exhaustive search s=1,2,.. -- sec. 2.2
* block partition of the one-sided (block) method            -- sec. 3, Table 1
* two-sided geometry of Algorithm 1                           -- sec. 2.2, Alg. 1

Readings of the paper taken here (each is listed in the design notes):
* Newton is run on I0(zeta) - 1/eps1 (same root as 1/I0 - eps1; with the
  reciprocal form the first step from zeta0 = 50 leaves the domain).
* The printed s-condition "w_s < eps2" is met at s = 1 for every eps2 > eps1;
  read as: s is the smallest s >= 1 whose window value at the first retained
  column, w_s^{zeta, M+2s} with M+1 = W retained columns, reaches eps2.
  This reading reproduces the block orders of Table 1.
* A block of width W gets s extras on the right (continuation of the
  recurrence) and uses its own first s columns as the left extras; its length is
  L = W + s and its window is w^{zeta, L-1} over the L columns.  The next block
  has width W' = s.  Recursion stops when W' <= min_block, or when s >= W;
  those W' columns are multiplied directly.
* L is enlarged to a fast FFT length (sec. 5.1 suggests taking a slightly
  larger s): the smallest even L whose half is 2^a 3^b 5^c.
"""

import numpy as np
from scipy.special import i0, i1


def kaiser(n, M, zeta):
    """w_n^{zeta,M} = I0(zeta*sqrt(1-(2n/M-1)^2)) / I0(zeta), 0 <= n <= M (sec. 2.1)."""
    n = np.asarray(n, dtype=np.float64)
    t = 2.0 * n / M - 1.0
    arg = np.sqrt(np.maximum(0.0, 1.0 - t * t))
    return i0(zeta * arg) / i0(zeta)


def zeta_of_eps(eps1, zeta0=50.0):
    """Solve 1/I0(zeta) = eps1 by Newton's method from zeta0 = 50 (sec. 2.2).

    h(z) = I0(z) - 1/eps1 is increasing and convex for z > 0 and h(50) > 0 for
    every eps1 >= 1e-20, so the iteration decreases monotonically to the root.
    """
    if not (0.0 < eps1 < 1.0):
        raise ValueError("eps1 must lie in (0, 1)")
    z = zeta0
    for _ in range(500):
        dz = (i0(z) - 1.0 / eps1) / i1(z)
        z -= dz
        if abs(dz) <= 1e-14 * z:
            break
    return float(z)


def extra_count(W, zeta, eps2):
    """Smallest s >= 1 with w_s^{zeta, W-1+2s} >= eps2 (sec. 2.2, read as above)."""
    s = 1
    while kaiser(s, W - 1 + 2 * s, zeta) < eps2:
        s += 1
    return s


def is_smooth5(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def fft_length(lmin):
    """Smallest even L >= lmin whose half L/2 is 2^a 3^b 5^c."""
    L = max(2, lmin + (lmin & 1))
    while not is_smooth5(L // 2):
        L += 2
    return L


class Block:
    """One compressed block.

    Block columns c = 0 .. L-1 hold degrees m = c + m_offset.  Columns
    [c_lo, c_hi) carry the input; the others are extras (zero input).
    The window of the block is w^{zeta, L-1} over its L columns.
    """

    def __init__(self, L, m_offset, c_lo, c_hi):
        self.L, self.m_offset, self.c_lo, self.c_hi = L, m_offset, c_lo, c_hi

    def as_tuple(self):
        return (self.L, self.m_offset, self.c_lo, self.c_hi)

    def __repr__(self):
        return "Block(L=%d, m_offset=%d, retained=[%d,%d))" % self.as_tuple()


def partition_one_sided(N, zeta, eps2, min_block=32, round_fft=True):
    """Block partition of sec. 3 (Algorithms 3/4): returns (blocks, tail).

    Block i has width W_i (W_1 = N): its retained columns are [s_i, W_i), its
    extras are columns [0, s_i) (zeroed input) and [W_i, W_i + s_i) (continued
    recurrence).  W_{i+1} = s_i.  The first ``tail`` columns are multiplied
    directly.
    """
    blocks = []
    W = N
    while W > min_block:
        s = extra_count(W, zeta, eps2)
        L = W + s
        if round_fft:
            L = fft_length(L)
            s = L - W
        if s >= W:
            break
        blocks.append(Block(L, 0, s, W))
        W = s
    return blocks, W


def partition_two_sided(N, zeta, eps2, round_fft=True):
    """Geometry of Algorithm 1: one block, degrees m = -s .. N-1+s_r.

    s extras on the left, s_r >= s on the right (s_r = s unless the FFT length is
    rounded up), retained columns [s, s+N).
    """
    s = extra_count(N, zeta, eps2)
    L = N + 2 * s
    if round_fft:
        L = fft_length(L)
    return [Block(L, -s, s, s + N)], 0
