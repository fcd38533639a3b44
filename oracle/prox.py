"""FP64 reference of the TV proximal map (the prox of lambda*TV + bound).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.

The proximal step of ISTA/FISTA (equation proxmal, section IV) with
g = lambda*J + delta_C, J the isotropic total variation (equation
Thirty-two with rho = 0) and C = {x >= lower}, is computed, as in the paper,
by the dual approach of Beck and Teboulle [Beck-b]: fast gradient projection
(FGP) on the dual field, a fixed number of iterations.

    argmin_x  lam * TV(x) + 1/2 ||x - z||^2   subject to x >= lower

Discrete operators (d = 2 or 3 axes, Neumann boundary):
* Lt = -grad with forward differences, zero on each axis' last index
  (the dual field has no component across the last face);
* L = its transpose, a divergence with backward differences;
* dual projection P_P: each point's d-vector divided by max(1, its 2-norm);
* primal projection P_C: max(x, lower);
* dual step 1 / (4 d lam), since ||L||^2 <= 4 d.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

__all__ = ["Lt", "L", "tv_prox", "tv_value", "tv_smooth"]


def Lt(x: np.ndarray):
    """-grad x by forward differences; component along numpy axis a is zero
    on that axis' last index."""
    out = []
    for ax in range(x.ndim):
        d = np.zeros_like(x)
        sl_lo = [slice(None)] * x.ndim
        sl_hi = [slice(None)] * x.ndim
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        d[tuple(sl_lo)] = x[tuple(sl_lo)] - x[tuple(sl_hi)]
        out.append(d)
    return out


def L(p) -> np.ndarray:
    """Adjoint of Lt: (L p)_i = sum_a p_a[i] - p_a[i - e_a] (terms with an
    index outside the grid, or on the last index, are zero)."""
    x = np.zeros_like(p[0])
    nd = x.ndim
    for ax in range(nd):
        pa = p[ax].copy()
        sl_last = [slice(None)] * nd
        sl_last[ax] = -1
        pa[tuple(sl_last)] = 0.0
        x += pa
        sl_lo = [slice(None)] * nd
        sl_hi = [slice(None)] * nd
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        x[tuple(sl_hi)] -= pa[tuple(sl_lo)]
    return x


def _proj_dual(p):
    nrm = np.sqrt(sum(pa * pa for pa in p))
    s = np.maximum(1.0, nrm)
    return [pa / s for pa in p]


def tv_prox(z: np.ndarray, lam: float, n_iter: int = 20, lower: Optional[np.ndarray] = None,
            step: Optional[float] = None) -> np.ndarray:
    """FGP for the bound-constrained isotropic-TV prox; lam = alpha*lambda.

    ``step`` overrides the dual step 1/(4 d lam) (used by tests that compare
    a d-dimensional run with a lower-dimensional one)."""
    z = np.asarray(z, dtype=np.float64)
    lo = np.zeros_like(z) if lower is None else np.asarray(lower, dtype=np.float64)

    def proj_c(v):
        return np.maximum(v, lo)

    if lam == 0.0:
        return proj_c(z)
    nd = z.ndim
    if step is None:
        step = 1.0 / (4.0 * nd * lam)
    r = [np.zeros_like(z) for _ in range(nd)]
    p_prev = [np.zeros_like(z) for _ in range(nd)]
    t = 1.0
    for _ in range(n_iter):
        x = proj_c(z - lam * L(r))
        g = Lt(x)
        p = _proj_dual([r[a] + step * g[a] for a in range(nd)])
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        r = [p[a] + ((t - 1.0) / t_next) * (p[a] - p_prev[a]) for a in range(nd)]
        p_prev = p
        t = t_next
    return proj_c(z - lam * L(p_prev))


def tv_value(x: np.ndarray) -> float:
    """Isotropic TV with the same forward differences (zero across the last face)."""
    g = Lt(np.asarray(x, dtype=np.float64))
    return float(np.sqrt(sum(ga * ga for ga in g)).sum())


def tv_smooth(x: np.ndarray, rho: float):
    """Smoothed TV of equation Thirty-two and its gradient (section V-B):

        J_rho(x) = sum_j sqrt(|Lt x|_j^2 + rho^2) - rho,
        grad J_rho(x) = L w,  w = Lt x / sqrt(|Lt x|^2 + rho^2)

    (L = Lt^T; with rho = 0, w is taken as 0 where Lt x = 0).  The gradient is
    the TV term of equation Twentyone, -div(grad x / sqrt(|grad x|^2 +
    rho^2)) in the differences used by the prox.  Returns (J, grad)."""
    x = np.asarray(x, dtype=np.float64)
    g = Lt(x)
    s = np.sqrt(sum(ga * ga for ga in g) + rho * rho)
    value = float((s - rho).sum())
    with np.errstate(invalid="ignore", divide="ignore"):
        w = [np.where(s > 0, ga / s, 0.0) for ga in g]
    return value, L(w)
