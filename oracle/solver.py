"""FP64 reference of the reconstruction iterations (sections IV and V).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.

The problem of equation two: minimise F(x) = f(x) + g(x) with
f(x) = 1/2 ||H x - p_hat||^2 (gradient H^T (H x - p_hat), equation Six) and
g(x) = lam TV(x) + indicator(x >= 0).

* ``power_iteration``: the Lipschitz constant L_f, the largest eigenvalue of
  H^T H, by the power method (section IV).
* ``fista`` (Alg. FISTA; momentum off gives Alg. ISTA): x_k = P_L(y_k) with
  P_L(y) = prox_{alpha g}(y - alpha grad f(y)) (the gradient and proximal
  lines of Alg. ISTA; the prox by FGP, ``prox.tv_prox``), then
  t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, theta_k = (t_k - 1) / t_{k+1},
  y_{k+1} = x_k + theta_k (x_k - x_{k-1}).
* ``mg_fista`` (Alg. FISTAMG) on two or more levels: at iteration k > 1 the decision
  rule (equation conditions) chooses between the direct step P_L(y_k) and a
  recursive step: coarse start x0 = R y_k, coherence term
  v = R grad F_rho,h(y_k) - grad F_rho,h-1(x0) (equation Fourteen; F_rho the
  objective with the smoothed TV of equation Thirty-two, gradient equation
  Twentyone), restricted bound lower = R y_k - blockmin(y_k) (equation
  constraint), FISTA on phi = F_rho,h-1 + <v, .> with projections onto
  x >= lower, and the correction x_k = y_k + P (x_c - x0).
* more than two levels (section I: the method extends to more levels):
  the coarse solve at level i is itself FISTAMG-like -- at each of its
  iterations after the first the same decision rule, applied to
  grad phi_i, may replace the projected gradient step by a recursive step
  to level i + 1 with coherence v_{i+1} = R grad phi_i(y) - grad
  F_rho,i+1(R y) and bound R y - blockmin(y - lower_i) (``coarse_mg``).

Readings where the paper is silent or garbled:
* the coarse level has its own plan (grid halved, time step doubled, PML
  halved) and its data are the fine data at even sample indices;
* the coarse step size is the caller's (the same rule as the fine level's,
  from the coarse L_f), the coarse lambda is the fine one;
* coarse termination: stop after the update that makes
  phi_k - phi_{k+1} < eps_c max(|phi_k|, |phi_{k+1}|) (phi can be negative
  through <v, x>), or after q_c updates;
* fine termination (optional): F_{k-1} - F_k < eps_d max(F_{k-1}, F_k);
* the norms of the decision rule are 2-norms over the grid; R and P are the
  block average and its piecewise-constant transpose (``transfer``);
* more than two levels: each coarse level's step size and lambda are the
  caller's, its data the fine data at every 2^i-th sample; its
  coarse solve counts updates like the two-level one (q_c, eps_c), its first
  iteration is a projected gradient step, and its decision rule keeps its
  own K_d, K_r and last transfer point within one coarse solve.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import kspace, prox, transfer

__all__ = ["Level", "power_iteration", "grad_f", "value_f", "objective", "smoothed", "fista", "coarse_fista",
           "coarse_mg", "mg_fista", "MGParams"]


@dataclass
class Level:
    """One grid level: its forward model, data, lambda and step size."""
    op: object               # oracle plan (kspace.make_plan)
    data: np.ndarray         # (nt, ns) measured data p_hat at this level
    lam: float
    alpha: float

    @property
    def shape(self):
        return self.op.shape


def grad_f(level: Level, x: np.ndarray):
    """(f(x), grad f(x)) = (1/2 ||H x - p_hat||^2, H^T (H x - p_hat))."""
    r = kspace.forward(level.op, x) - level.data
    return 0.5 * float(np.sum(r * r)), kspace.adjoint(level.op, r)


def value_f(level: Level, x: np.ndarray) -> float:
    """f(x) alone (one forward solve)."""
    r = kspace.forward(level.op, x) - level.data
    return 0.5 * float(np.sum(r * r))


def objective(level: Level, x: np.ndarray) -> float:
    """F(x) = f(x) + lam TV(x) (x assumed feasible)."""
    r = kspace.forward(level.op, x) - level.data
    return 0.5 * float(np.sum(r * r)) + level.lam * prox.tv_value(x)


def smoothed(level: Level, x: np.ndarray, rho: float):
    """(F_rho(x), grad F_rho(x)): f + lam J_rho and its gradient."""
    fv, g = grad_f(level, x)
    jv, jg = prox.tv_smooth(x, rho)
    return fv + level.lam * jv, g + level.lam * jg


def power_iteration(op, n_iter: int = 30, seed: int = 0, v0: Optional[np.ndarray] = None) -> float:
    """Largest eigenvalue of H^T H by the power method from v0 (default: a
    seeded standard-normal start): v <- H^T H v / ||H^T H v||; returns the
    last ||H^T H v|| with ||v|| = 1."""
    v = np.random.default_rng(seed).standard_normal(op.shape) if v0 is None else np.array(v0, dtype=np.float64)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(n_iter):
        w = kspace.adjoint(op, kspace.forward(op, v))
        lam = float(np.linalg.norm(w))
        v = w / lam
    return lam


def _t_next(t: float) -> float:
    return (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0


def _direct(level: Level, y: np.ndarray, prox_iter: int, g: Optional[np.ndarray] = None) -> np.ndarray:
    """P_L(y) = prox_{alpha g}(y - alpha grad f(y)) (grad f(y) given or computed)."""
    if g is None:
        _, g = grad_f(level, y)
    return prox.tv_prox(y - level.alpha * g, level.alpha * level.lam, prox_iter)


def fista(level: Level, x0: np.ndarray, n_iter: int, momentum: bool = True, prox_iter: int = 20,
          eps_d: Optional[float] = None):
    """Alg. FISTA (or ISTA without momentum); returns (x, [F(x_k)])."""
    x_prev = np.asarray(x0, dtype=np.float64)
    y = x_prev.copy()
    t = 1.0
    hist: List[float] = []
    for _ in range(n_iter):
        x = _direct(level, y, prox_iter)
        hist.append(objective(level, x))
        tn = _t_next(t)
        theta = (t - 1.0) / tn if momentum else 0.0
        y = x + theta * (x - x_prev)
        x_prev, t = x, tn
        if eps_d is not None and len(hist) > 1 and hist[-2] - hist[-1] < eps_d * max(hist[-2], hist[-1]):
            break
    return x_prev, hist


def coarse_fista(level: Level, x0: np.ndarray, v: np.ndarray, lower: np.ndarray, rho: float, q_c: int,
                 eps_c: float, momentum: bool = True):
    """FISTA on phi(x) = F_rho(x) + <v, x> over x >= lower: the proximal map
    of the smooth coarse objective is the projection (section V-E).
    Returns (x, number of updates)."""
    def phi_value(x):
        return value_f(level, x) + level.lam * prox.tv_smooth(x, rho)[0] + transfer.dot(v, x)

    x_prev = np.asarray(x0, dtype=np.float64)
    y = x_prev.copy()
    t = 1.0
    phi_prev = phi_value(x_prev)
    k = 0
    while k < q_c:
        _, g = smoothed(level, y, rho)
        x = np.maximum(y - level.alpha * (g + v), lower)
        k += 1
        phi_x = phi_value(x)
        tn = _t_next(t)
        theta = (t - 1.0) / tn if momentum else 0.0
        y = x + theta * (x - x_prev)
        x_prev, t = x, tn
        if phi_prev - phi_x < eps_c * max(abs(phi_prev), abs(phi_x)):
            break
        phi_prev = phi_x
    return x_prev, k


@dataclass
class MGParams:
    """Parameters of Alg. FISTAMG and the decision rule (the paper's 2D values)."""
    kappa: float = 0.25
    vartheta: float = 0.1
    q_d: int = 3
    q_c: int = 8
    eps_c: float = 1e-2
    rho: float = 1e-2
    eps_d: Optional[float] = None
    momentum: bool = True
    prox_iter: int = 20


@dataclass
class MGRecord:
    kind: str           # "direct" or "recursive"
    F: float            # F_h(x_k)
    coarse_updates: int = 0
    grad_ratio: float = 0.0   # ||R grad F_rho(y)|| / ||grad F_rho(y)|| at a decision
    depth: int = 0            # deepest level a recursive step reached (0: direct step)


def _decide(p: "MGParams", g: np.ndarray, y: np.ndarray, y_tilde, k_d: int, k_r: int):
    """The decision rule (equation conditions) at y with gradient g of the
    level's smoothed objective: (recursive?, ||R g|| / ||g||)."""
    rg = transfer.restrict(g)
    ratio = math.sqrt(transfer.norm2(rg)) / max(math.sqrt(transfer.norm2(g)), 1e-300)
    far = (y_tilde is not None and
           math.sqrt(transfer.norm2(y - y_tilde)) > p.vartheta * math.sqrt(transfer.norm2(y_tilde)))
    return (ratio > p.kappa) and (far or k_r == 0 or k_d > p.q_d), ratio, rg


def coarse_mg(levels, i: int, x0: np.ndarray, v: np.ndarray, lower: np.ndarray, p: "MGParams"):
    """The coarse solve at level i of ``levels`` (0 the target level): FISTA
    on phi_i = F_rho,i + <v, .> over x >= lower, whose iterations after the
    first may take a recursive step to level i + 1 when there is one (same
    decision rule, coherence term and restricted bound as at the target
    level).  With no coarser level it is ``coarse_fista``.  Returns (x,
    number of updates, deepest level reached)."""
    lv = levels[i]
    has_next = i + 1 < len(levels)

    def phi_value(x):
        return value_f(lv, x) + lv.lam * prox.tv_smooth(x, p.rho)[0] + transfer.dot(v, x)

    x_prev = np.asarray(x0, dtype=np.float64)
    y = x_prev.copy()
    t = 1.0
    phi_prev = phi_value(x_prev)
    k = k_d = k_r = 0
    y_tilde = None
    depth = i
    while k < p.q_c:
        _, g = smoothed(lv, y, p.rho)
        g = g + v
        recursive = False
        if has_next and k > 0:
            recursive, _, rg = _decide(p, g, y, y_tilde, k_d, k_r)
        if recursive:
            k_d, k_r = 0, k_r + 1
            xc0 = transfer.restrict(y)
            _, gc = smoothed(levels[i + 1], xc0, p.rho)
            xc, _, d = coarse_mg(levels, i + 1, xc0, rg - gc, transfer.restrict_lower(y, lower), p)
            depth = max(depth, d)
            x = y + transfer.prolong(xc - xc0)
            y_tilde = y.copy()
        else:
            k_d += 1
            x = np.maximum(y - lv.alpha * g, lower)
        k += 1
        phi_x = phi_value(x)
        tn = _t_next(t)
        theta = (t - 1.0) / tn if p.momentum else 0.0
        y = x + theta * (x - x_prev)
        x_prev, t = x, tn
        if phi_prev - phi_x < p.eps_c * max(abs(phi_prev), abs(phi_x)):
            break
        phi_prev = phi_x
    return x_prev, k, depth


def mg_fista(fine: Level, coarse, x0: np.ndarray, n_iter: int, params: MGParams = MGParams()):
    """Alg. FISTAMG; ``coarse`` is the next coarse level, or a list of
    levels from the next coarse one down (more than two levels).  Returns
    (x, [MGRecord])."""
    levels = [fine] + (list(coarse) if isinstance(coarse, (list, tuple)) else [coarse])
    p = params
    x_prev = np.asarray(x0, dtype=np.float64)
    y = x_prev.copy()
    t = 1.0
    k_d = k_r = 0
    y_tilde = None
    hist: List[MGRecord] = []
    for k in range(1, n_iter + 1):
        recursive = False
        ratio = 0.0
        gf = None
        if k > 1:
            # grad f(y) serves the decision (through grad F_rho) and a direct step
            _, gf = grad_f(fine, y)
            gF = gf + fine.lam * prox.tv_smooth(y, p.rho)[1]
            recursive, ratio, rg = _decide(p, gF, y, y_tilde, k_d, k_r)
        if recursive:
            k_d, k_r = 0, k_r + 1
            xc0 = transfer.restrict(y)
            _, gc = smoothed(levels[1], xc0, p.rho)
            v = rg - gc
            lower = transfer.restrict_lower(y)
            xc, nup, depth = coarse_mg(levels, 1, xc0, v, lower, p)
            x = y + transfer.prolong(xc - xc0)
            y_tilde = y.copy()
            rec = MGRecord("recursive", 0.0, nup, ratio, depth)
        else:
            k_d += 1
            x = _direct(fine, y, p.prox_iter, gf)
            rec = MGRecord("direct", 0.0, 0, ratio)
        rec.F = objective(fine, x)
        hist.append(rec)
        tn = _t_next(t)
        theta = (t - 1.0) / tn if p.momentum else 0.0
        y = x + theta * (x - x_prev)
        x_prev, t = x, tn
        if p.eps_d is not None and len(hist) > 1 and \
                hist[-2].F - hist[-1].F < p.eps_d * max(hist[-2].F, hist[-1].F):
            break
    return x_prev, hist
