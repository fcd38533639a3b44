"""FP64 reference of the multi-grid transfer operators and FP64 reductions.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.

Section V introduces a restriction I_h^{h-1} and a prolongation I_{h-1}^h
between the target level and the next coarse level without defining them.
The reading used here: the coarse grid is cell-centred over 2^d blocks of
fine points; restriction averages each block; prolongation copies each
coarse value to its block (piecewise constant), which is 2^d times the
transpose of the restriction.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["restrict", "prolong", "restrict_lower", "dot", "norm2"]


def restrict(fine: np.ndarray) -> np.ndarray:
    """x_c[I] = 2^-d * sum over the block {2I + delta, delta in {0,1}^d}."""
    f = np.asarray(fine, dtype=np.float64)
    nd = f.ndim
    acc = np.zeros(tuple(s // 2 for s in f.shape))
    for corner in np.ndindex(*([2] * nd)):
        acc += f[tuple(slice(c, None, 2) for c in corner)]
    return acc / (2 ** nd)


def prolong(coarse: np.ndarray) -> np.ndarray:
    """x_f[i] = x_c[floor(i / 2)] along every axis."""
    c = np.asarray(coarse, dtype=np.float64)
    for ax in range(c.ndim):
        c = np.repeat(c, 2, axis=ax)
    return c


def restrict_lower(fine: np.ndarray, fine_lower=None) -> np.ndarray:
    """The restricted bound of equation constraint (section V-C):
    lower[I] = (R y)[I] - min_{j in block I} (y_j - l_j), the index set
    I_{h,i} of the paper being the 2^d fine points averaged into coarse
    point i.  The paper's fine bound is l = 0 (nonnegativity, the default);
    a bound l at an intermediate level of more than two levels restricts the
    same way, so that every coarse x >= lower keeps y + P(x - R y) >= l."""
    f = np.asarray(fine, dtype=np.float64)
    d = f if fine_lower is None else f - np.asarray(fine_lower, dtype=np.float64)
    nd = f.ndim
    mn = np.full(tuple(s // 2 for s in f.shape), np.inf)
    for corner in np.ndindex(*([2] * nd)):
        mn = np.minimum(mn, d[tuple(slice(c, None, 2) for c in corner)])
    return restrict(f) - mn


def dot(a: np.ndarray, b: np.ndarray) -> float:
    """sum_i a_i b_i, correctly rounded: each product of two float32 values is
    exact in FP64 and math.fsum adds them without intermediate rounding."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return math.fsum((a * b).tolist())


def norm2(a: np.ndarray) -> float:
    """Squared 2-norm, via `dot`."""
    return dot(a, a)
