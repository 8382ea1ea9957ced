"""Pins of the oracle's plan parameters (window, zeta, s, blocks) to the paper."""

import json
import os

import numpy as np
import pytest
from scipy.special import i0

from oracle import params

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("eps1", [1e-6, 1e-7, 1e-10, 1e-12, 1e-15])
def test_zeta_solves_its_equation(eps1):
    # sec. 2.2: 1/I0(zeta) = eps1
    z = params.zeta_of_eps(eps1)
    assert abs(1.0 / i0(z) - eps1) <= 1e-13 * eps1


@pytest.mark.parametrize("M", [8, 9, 100, 1001])
def test_kaiser_window_shape(M):
    # sec. 2.1: w_n^{zeta,M} = I0(zeta sqrt(1-(2n/M-1)^2)) / I0(zeta), 0 <= n <= M
    z = params.zeta_of_eps(1e-8)
    w = params.kaiser(np.arange(M + 1), M, z)
    assert w[0] == pytest.approx(1e-8, rel=1e-12) and w[-1] == pytest.approx(1e-8, rel=1e-12)
    np.testing.assert_allclose(w, w[::-1], rtol=1e-13)                    # symmetric
    assert np.all(np.diff(w[: M // 2 + 1]) > 0)                            # rises to the centre
    if M % 2 == 0:
        assert w[M // 2] == pytest.approx(1.0, abs=1e-15)                  # peak 1
    # a hand-evaluated point: n = M/4 gives sqrt(1 - 1/4)
    if M % 4 == 0:
        assert w[M // 4] == pytest.approx(i0(z * np.sqrt(0.75)) / i0(z), rel=1e-14)


@pytest.mark.parametrize("W,eps1,eps2", [(256, 1e-12, 1e-2), (4096, 1e-7, 1e-2),
                                         (16384, 1e-10, 1e-4), (100, 1e-6, 1e-3)])
def test_extra_count_is_minimal(W, eps1, eps2):
    # sec. 2.2: s is the smallest s = 1, 2, ... meeting the window condition
    z = params.zeta_of_eps(eps1)
    s = params.extra_count(W, z, eps2)
    assert params.kaiser(s, W - 1 + 2 * s, z) >= eps2
    for t in range(1, s):
        assert params.kaiser(t, W - 1 + 2 * t, z) < eps2


def test_fft_length_brute_force():
    def smooth(n):
        return all(f in (2, 3, 5) for f in _factors(n))

    for lmin in range(1, 400):
        L = params.fft_length(lmin)
        expect = next(L2 for L2 in range(max(2, lmin), 10 * lmin + 10)
                      if L2 % 2 == 0 and smooth(L2 // 2))
        assert L == expect


def _factors(n):
    out, p = [], 2
    while n > 1:
        while n % p == 0:
            out.append(p)
            n //= p
        p += 1
    return out


def test_block_partition_reproduces_table1():
    """Table 1 (sec. 5.2): orders N_i = W_i + s_i of the block submatrices.

    Soft pin: the paper's own sizes may include its FFT-size choices, so the
    unrounded rule must give N_1 within 1.5% for N >= 2048 (4% below) and the
    same recursion W_{i+1} = s_i (N_{i+1} > s_i relation checked on the paper's
    numbers themselves)."""
    with open(os.path.join(GOLDEN, "table1.json")) as f:
        t1 = json.load(f)
    for col in ("1e-6", "1e-10"):
        eps1 = t1["columns"][col]["eps1"]
        z = params.zeta_of_eps(eps1)
        for N, row in t1["rows"].items():
            N = int(N)
            blocks, tail = params.partition_one_sided(N, z, 1e-4, min_block=20, round_fft=False)
            got = [b.L for b in blocks]
            ref = row[col]
            tol = 0.015 if N >= 2048 else 0.04
            assert abs(got[0] / ref[0] - 1.0) <= tol, (col, N, got, ref)
            # block geometry: each block is W + s with W the previous s
            W = N
            for b in blocks:
                assert b.c_hi == W and b.L == W + b.c_lo
                W = b.c_lo
            assert tail == W


def test_two_sided_geometry():
    # Algorithm 1: degrees -s .. N-1+s_r, retained columns [s, s+N)
    z = params.zeta_of_eps(1e-12)
    (blk,), tail = params.partition_two_sided(4096, z, 1e-2)
    s = params.extra_count(4096, z, 1e-2)
    assert tail == 0 and blk.m_offset == -s and blk.c_lo == s and blk.c_hi == s + 4096
    assert blk.L >= 4096 + 2 * s and blk.L == params.fft_length(4096 + 2 * s)
