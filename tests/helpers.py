"""Shared helpers of the GPU tests: oracle objects for a plan's parameters,
device transfers and error measures (no arithmetic of the method here)."""

import functools
import sys

import numpy as np

from oracle import compressed, direct, matrix

FAM_IDS = {"chebyshev_t": matrix.CHEBYSHEV_T, "legendre": matrix.LEGENDRE,
           "jacobi": matrix.JACOBI, "laguerre_fn": matrix.LAGUERRE_FN,
           "hermite_fn": matrix.HERMITE_FN, "sine": matrix.SINE,
           "cos_power": matrix.COS_POWER}


def say(*msg):
    """Name the case before a GPU step (flushed, so that a crash still shows it)."""
    print("[case]", *msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=32)
def oracle_family(fam, N, alpha=0.0, beta=0.0, unweighted=False, power=2):
    return matrix.MatrixFamily(FAM_IDS[fam], N, alpha=alpha, beta=beta,
                               orthonormal=not unweighted, power=power)


@functools.lru_cache(maxsize=16)
def oracle_compressed(fam, N, eps, eps2=1e-2, min_block=32, alpha=0.0, beta=0.0,
                      unweighted=False, power=2):
    f = oracle_family(fam, N, alpha, beta, unweighted, power)
    return compressed.Compressed(compressed.Plan(f, eps, eps2, min_block=min_block))


def oracle_direct(fam, N, X, rows=None, alpha=0.0, beta=0.0, unweighted=False, power=2):
    return direct.matvec(oracle_family(fam, N, alpha, beta, unweighted, power), X, rows=rows)


def to_dev(X, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(X)).to(dtype=dtype, device="cuda")


def to_host(Y):
    import torch
    torch.cuda.synchronize()
    return Y.double().cpu().numpy()


def rel_rows(Y, Yref):
    """max over right-hand sides of ||y - yref||_2 / ||yref||_2"""
    num = np.linalg.norm(np.atleast_2d(Y) - np.atleast_2d(Yref), axis=1)
    den = np.linalg.norm(np.atleast_2d(Yref), axis=1)
    return float(np.max(num / den))


# Bar of the float32 and split-bf16 paths against float64 on the same plan:
# relative 2-norm per right-hand side.
REDUCED_TOL = 1e-6
