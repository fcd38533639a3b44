"""Pins of the FP64 prox, transfer and reduction oracles."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.optimize import lsq_linear

from oracle import prox as P
from oracle import transfer as T


# ---------------------------------------------------------------- operators
@pytest.mark.parametrize("shape", [(7,), (6, 5), (4, 3, 5)])
def test_L_is_transpose_of_Lt(shape):
    """<L p, x> = <p, Lt x> for random p, x, by dense matrices."""
    rng = np.random.default_rng(0)
    N = int(np.prod(shape))
    nd = len(shape)
    A = np.zeros((nd * N, N))
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1
        A[:, i] = np.concatenate([g.ravel() for g in P.Lt(e.reshape(shape))])
    B = np.zeros((N, nd * N))
    for i in range(nd * N):
        e = np.zeros(nd * N)
        e[i] = 1
        parts = [e[a * N:(a + 1) * N].reshape(shape) for a in range(nd)]
        B[:, i] = P.L(parts).ravel()
    # the dual components on each axis' last index are unused by both
    assert np.allclose(A.T, B, atol=0) or np.abs(A.T - B).max() < 1e-15
    # ||L||^2 <= 4 d
    s = np.linalg.svd(B, compute_uv=False)[0]
    assert s ** 2 <= 4 * nd + 1e-12


def test_Lt_is_minus_forward_difference():
    x = np.array([[1.0, 4.0, 9.0], [2.0, 2.0, 7.0]])
    gy, gx = P.Lt(x)  # numpy axis 0 (y) then axis 1 (x)
    assert np.array_equal(gx, [[-3.0, -5.0, 0.0], [0.0, -5.0, 0.0]])
    assert np.array_equal(gy, [[-1.0, 2.0, 2.0], [0.0, 0.0, 0.0]])


# ---------------------------------------------------------------- P10
def test_p10_zero_lambda_is_projection():
    rng = np.random.default_rng(1)
    z = rng.standard_normal((9, 7))
    lo = rng.uniform(-0.5, 0.5, size=z.shape)
    assert np.array_equal(P.tv_prox(z, 0.0, 20, lo), np.maximum(z, lo))
    assert np.array_equal(P.tv_prox(z, 0.0), np.maximum(z, 0.0))


def test_p10_constant_is_fixed_point():
    z = np.full((8, 8), 2.5)
    assert np.allclose(P.tv_prox(z, 0.3, 20), z, atol=1e-15)
    z3 = np.full((4, 5, 6), 1.25)
    assert np.allclose(P.tv_prox(z3, 0.1, 20), z3, atol=1e-15)


def test_p10_y_constant_reduces_to_1d():
    """An image constant along y has no y-differences; with the same dual
    step, the 2D iteration equals the 1-D one on each row."""
    rng = np.random.default_rng(2)
    row = rng.uniform(0, 2, size=17)
    img = np.tile(row, (6, 1))
    lam = 0.2
    step = 1.0 / (8.0 * lam)
    out2 = P.tv_prox(img, lam, 20, step=step)
    out1 = P.tv_prox(row, lam, 20, step=step)
    assert np.allclose(out2, np.tile(out1, (6, 1)), rtol=0, atol=1e-14)


def _tv1d_exact(z, lam):
    """1-D TV denoising by its dual, a box-constrained least-squares problem
    solved by scipy: min_w 1/2||z - D^T w||^2, |w| <= lam; x = z - D^T w."""
    n = z.size
    D = np.zeros((n - 1, n))
    for i in range(n - 1):
        D[i, i] = -1
        D[i, i + 1] = 1
    res = lsq_linear(D.T, z, bounds=(-lam, lam), method="bvls", tol=1e-15, lsmr_tol=None,
                     max_iter=10000)
    return z - D.T @ res.x


def test_p10_converged_fgp_matches_exact_1d_solution():
    rng = np.random.default_rng(3)
    z = 10.0 + np.cumsum(rng.standard_normal(40)) * 0.5 + rng.standard_normal(40)
    lam = 0.7
    exact = _tv1d_exact(z, lam)
    got = P.tv_prox(z, lam, 20000)
    assert np.abs(got - exact).max() < 1e-6


def test_p10_prox_decreases_objective_and_is_feasible():
    rng = np.random.default_rng(4)
    z = rng.standard_normal((16, 16))
    lam = 0.15
    x = P.tv_prox(z, lam, 200)
    assert x.min() >= 0
    obj = lambda v: lam * P.tv_value(v) + 0.5 * np.sum((v - z) ** 2)
    xz = np.maximum(z, 0)
    assert obj(x) < obj(xz)
    # a random feasible perturbation does not improve the converged point
    for _ in range(10):
        v = np.maximum(x + 1e-3 * rng.standard_normal(x.shape), 0)
        assert obj(v) >= obj(x) - 1e-6


# ---------------------------------------------------------------- P11
@pytest.mark.parametrize("shape", [(8, 6), (4, 6, 8)])
def test_p11_transfers(shape):
    rng = np.random.default_rng(5)
    nd = len(shape)
    c = np.full(shape, 3.25)
    assert np.array_equal(T.restrict(c), np.full(tuple(s // 2 for s in shape), 3.25))
    xc = rng.standard_normal(tuple(s // 2 for s in shape))
    assert np.allclose(T.restrict(T.prolong(xc)), xc, rtol=0, atol=1e-15)
    x = rng.standard_normal(shape)
    lhs = float(np.sum(T.restrict(x) * xc))
    rhs = float(np.sum(x * T.prolong(xc))) / 2 ** nd
    assert math.isclose(lhs, rhs, rel_tol=1e-13, abs_tol=1e-13)
    # explicit block average at one index
    I = tuple(1 for _ in shape)
    blk = x[tuple(slice(2, 4) for _ in shape)]
    assert math.isclose(T.restrict(x)[I], blk.mean(), rel_tol=1e-14)


# ---------------------------------------------------------------- P12
def test_p12_dot_is_correctly_rounded():
    """Against exact rational arithmetic on float32 inputs."""
    rng = np.random.default_rng(6)
    a = (rng.standard_normal(5000) * 10.0 ** rng.integers(-3, 4, 5000)).astype(np.float32)
    b = (rng.standard_normal(5000)).astype(np.float32)
    exact = sum(Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b))
    assert T.dot(a, b) == float(exact)
    assert T.norm2(a) == float(sum(Fraction(float(x)) ** 2 for x in a))
