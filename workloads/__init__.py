"""Seeded synthetic workloads: shapes, seeds and right-hand sides.

This module is shared by the tests, the benchmark and the oracle checks, and
therefore holds none of the method's arithmetic: only random inputs and the
sizes of the workloads the paper's experiments (sec. 5) and the configurations
describe.  Every array is float64, one right-hand side per row (R x N).
"""

import math

import numpy as np

# family codes (the same integers the C ABI uses)
CHEBYSHEV_T, LEGENDRE, JACOBI, LAGUERRE_FN, HERMITE_FN = 1, 2, 3, 4, 5


def rhs(kind, R, N, seed):
    """Right-hand sides X (R x N).

    normal          x ~ N(0, 1)
    uniform11       x ~ U(-1, 1)
    uniform01       x ~ U(0, 1)                 (sec. 5.1 timing inputs)
    normal_decay    x_k ~ N(0, 1) * exp(-k/N)   (Laguerre series coefficients)
    """
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.standard_normal((R, N))
    if kind == "uniform11":
        return rng.uniform(-1.0, 1.0, (R, N))
    if kind == "uniform01":
        return rng.uniform(0.0, 1.0, (R, N))
    if kind == "normal_decay":
        return rng.standard_normal((R, N)) * np.exp(-np.arange(N) / N)[None, :]
    raise ValueError(kind)


# The five workloads.  eps is eps1 (threshold and 1/I0(zeta)); eps2 = 1e-2.
LEGENDRE_256 = dict(name="legendre-n256-fp64-r1", family=LEGENDRE, N=256, eps=1e-12,
                    nrhs=1, rhs="normal", seed=0)
THREE_PLANS_4096 = [
    dict(name="chebyshev-n4096-r1", family=CHEBYSHEV_T, N=4096, eps=1e-12, nrhs=1,
         rhs="uniform11", seed=2),
    dict(name="legendre-n4096-r1", family=LEGENDRE, N=4096, eps=1e-12, nrhs=1,
         rhs="uniform11", seed=2),
    dict(name="laguerre-fn-n4096-r1", family=LAGUERRE_FN, N=4096, eps=1e-12, nrhs=1,
         rhs="uniform11", seed=2),
]
LEGENDRE_16384 = dict(name="legendre-n16384-r64", family=LEGENDRE, N=16384, eps=1e-7,
                      nrhs=64, rhs="normal", seed=1)
LAGUERRE_65536 = dict(name="laguerre-fn-n65536-r1024", family=LAGUERRE_FN, N=65536,
                      eps=1e-7, nrhs=1024, rhs="normal_decay", seed=5)

BATCH_FAMILIES = [(JACOBI, -0.5, -0.5), (JACOBI, 0.0, 0.0), (JACOBI, 0.5, 1.5),
                  (JACOBI, 2.0, 3.0), (HERMITE_FN, 0.0, 0.0)]


def batch_plans(count=48, seed=4, n_lo=1024, n_hi=65536, r_hi=256):
    """Uneven plans: family uniform over BATCH_FAMILIES, N log-uniform in
    [n_lo, n_hi], nrhs uniform in [1, r_hi]; RHS of plan p drawn with seed 1000+p."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(count):
        fam, a, b = BATCH_FAMILIES[int(rng.integers(len(BATCH_FAMILIES)))]
        N = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        R = int(rng.integers(1, r_hi + 1))
        out.append(dict(name="batch-%02d" % p, family=fam, alpha=a, beta=b, N=N, eps=1e-7,
                        nrhs=R, rhs="normal", seed=1000 + p))
    return out


def shared_nodes(family, N):
    """Closed-form nodes that both the library (through spt_params.nodes) and
    the oracle take, so that full-size comparisons of the two hold at rounding
    level (each side's own quadrature nodes differ by a few ulp, which moves the
    entries by far more).  Synthetic points with the spread of each family's
    Gauss nodes:
      Jacobi family  x_j = cos(pi (2j+1) / (2N)), descending;
      Hermite        x_j = -sqrt(2N+1) cos(pi (2j+1) / (2N)), ascending;
      Laguerre       x_j = (4N+2) sin(pi (2j+1) / (4N))^2, ascending."""
    t = np.pi * (2.0 * np.arange(N) + 1.0)
    if family in (LEGENDRE, JACOBI):
        return np.cos(t / (2.0 * N))
    if family == HERMITE_FN:
        return -math.sqrt(2.0 * N + 1.0) * np.cos(t / (2.0 * N))
    if family == LAGUERRE_FN:
        return (4.0 * N + 2.0) * np.sin(t / (4.0 * N)) ** 2
    raise ValueError(family)


# Plans of the 48-plan batch checked against the oracle's compressed method at
# rounding level (shared nodes, row mode): every family, the largest sizes
# (four-step transforms) and a few small ones.
BATCH_ORACLE_C = [13, 10, 30, 17, 32, 6, 41, 1]
