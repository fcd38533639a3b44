"""Reconstruction iterations of sections IV and V on libpat.

ISTA / FISTA (Alg. ISTA, Alg. FISTA) and MG-FISTA (Alg. FISTAMG) on two
or more levels for

    min_x  F(x) = 1/2 ||H x - p_hat||^2 + lam TV(x)   subject to x >= 0

(equation two, gradient equation Six).  The host loop keeps only scalars
(step sizes, momentum, the decision rule's norms); every vector operation is
a libpat call on device tensors: H and H^T (``Plan.forward/adjoint``), the
float64 residual and inner products, the FGP prox, the smoothed TV and its
gradient (equations Thirty-two and Twentyone), the level transfers, the
restricted bound (equation constraint), the extrapolation ``axpby`` and the
projection.

The iteration follows the paper's algorithms; where it is silent: the coarse
level has its own plan (grid halved, time step doubled) with the fine data
at even sample indices, the coarse step size and lambda are the caller's,
the coarse loop stops after the update with
phi_k - phi_{k+1} < eps_c max(|phi_k|, |phi_{k+1}|) or after q_c updates,
and the fine loop (optionally) when F_{k-1} - F_k < eps_d max(F_{k-1}, F_k).
With more than two levels (the extension section I allows), the coarse
solve at level i takes, at its iterations after the first, the recursive
step to level i + 1 when the same decision rule applied to grad phi_i says
so: coherence v_{i+1} = R grad phi_i(y) - grad F_rho,i+1(R y) and bound
R y - blockmin(y - lower_i).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

from . import Batch, Plan, axpby, dot_f64, project, prolong, residual_f64, restrict, restrict_lower, tv_prox, tv_smooth

__all__ = ["Level", "MGParams", "MGRecord", "IterState", "save_state", "load_state", "power_iteration", "fista",
           "fista_batched", "coarse_fista", "coarse_mg", "mg_fista"]


class Level:
    """One grid level: plan, measured data (device, (nt, ns) float32),
    lambda and step size.  H and H^T run eagerly on the plan, or with
    ``graphs`` through a one-instance batch whose time loop is replayed from
    captured graphs (measured at 512^2: no faster; a single grid's passes
    are bound by their own duration, not by the host's launches)."""

    def __init__(self, plan: Plan, data, lam: float, alpha: float, graphs: bool = False):
        self.plan, self.data, self.lam, self.alpha = plan, data, lam, alpha
        self.res = float("nan")
        self._batch = Batch([plan]) if graphs else None

    def forward(self, x):
        return self._batch.forward([x])[0] if self._batch is not None else self.plan.forward(x)

    def adjoint(self, r):
        return self._batch.adjoint([r])[0] if self._batch is not None else self.plan.adjoint(r)

    def grad_f(self, x):
        """(f(x), grad f(x)) with f = 1/2 ||H x - p_hat||^2."""
        r, half = residual_f64(self.forward(x), self.data)
        return half, self.adjoint(r)

    def value_f(self, x) -> float:
        """f(x) alone (one forward solve)."""
        return residual_f64(self.forward(x), self.data)[1]

    def objective(self, x) -> float:
        """F(x) = f(x) + lam TV(x); keeps the residual norm RES(x) =
        ||H x - p_hat|| (section VI) in ``self.res``."""
        half = self.value_f(x)
        self.res = math.sqrt(2.0 * half)
        return half + self.lam * tv_smooth(x, 0.0)

    def smoothed(self, x, rho: float):
        """(F_rho(x), grad F_rho(x)) = (f + lam J_rho, grad f + lam grad J_rho)."""
        half, g = self.grad_f(x)
        j = tv_smooth(x, rho, grad=g, scale=self.lam)
        return half + self.lam * j, g


def power_iteration(plan: Plan, v0, n_iter: int = 30) -> float:
    """Largest eigenvalue of H^T H by the power method from the start v0
    (device tensor of the grid's shape)."""
    v = axpby(1.0 / math.sqrt(dot_f64(v0)), v0, 0.0, v0)
    lam = 0.0
    for _ in range(n_iter):
        w = plan.adjoint(plan.forward(v))
        lam = math.sqrt(dot_f64(w))
        v = axpby(1.0 / lam, w, 0.0, w)
    return lam


def _t_next(t: float) -> float:
    return (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0


def _direct(level: Level, y, prox_iter: int, g=None):
    """P_L(y) = prox_{alpha g}(y - alpha grad f(y)) (grad f(y) given or computed)."""
    if g is None:
        _, g = level.grad_f(y)
    z = axpby(1.0, y, -level.alpha, g)
    return tv_prox(z, level.alpha * level.lam, prox_iter)


@dataclass
class IterState:
    """What a FISTA or MG-FISTA run resumes from after its iteration k: the
    iterate x_k (``x_prev``), the extrapolated point y_{k+1}, the momentum
    t_{k+1} (Alg. FISTA), the history, and for MG-FISTA the counters K_d,
    K_r and the last recursion point y-tilde (Alg. FISTAMG, eq.
    conditions).  Every later iterate depends on these alone, so a resumed
    run reproduces an uninterrupted one bitwise."""
    k: int
    x_prev: object
    y: object
    t: float
    hist: list
    k_d: int = 0
    k_r: int = 0
    y_tilde: object = None


def save_state(path: str, state: IterState) -> None:
    """Write an IterState to `path` (tensors and plain numbers only: it loads
    with ``torch.load(weights_only=True)``)."""
    import torch
    hist = [r.__dict__.copy() if isinstance(r, MGRecord) else float(r) for r in state.hist]
    blob = {"k": int(state.k), "x_prev": state.x_prev.detach().cpu(), "y": state.y.detach().cpu(), "t": float(state.t),
            "hist": hist, "k_d": int(state.k_d), "k_r": int(state.k_r),
            "y_tilde": None if state.y_tilde is None else state.y_tilde.detach().cpu()}
    torch.save(blob, path)


def load_state(path: str, device) -> IterState:
    """Read an IterState written by ``save_state``, tensors on `device`."""
    import torch
    blob = torch.load(path, map_location="cpu", weights_only=True)
    hist = [MGRecord(**r) if isinstance(r, dict) else float(r) for r in blob["hist"]]
    yt = blob["y_tilde"]
    return IterState(blob["k"], blob["x_prev"].to(device), blob["y"].to(device), blob["t"], hist, blob["k_d"],
                     blob["k_r"], None if yt is None else yt.to(device))


def fista(level: Level, x0, n_iter: int, momentum: bool = True, prox_iter: int = 20,
          eps_d: Optional[float] = None, callback=None, state: Optional[IterState] = None, on_state=None):
    """Alg. FISTA (Alg. ISTA without momentum); returns (x, [F(x_k)]).
    ``callback(k, x_k, F(x_k))`` runs after every iteration.  `n_iter`
    counts every iteration of the run; with `state` (an ``IterState`` from
    an earlier call's ``on_state``, or ``load_state``) the run resumes after
    its iteration ``state.k`` (x0 is then unused).  ``on_state(IterState)``
    runs after every iteration (its tensors are the run's own: save or copy
    them there)."""
    if state is None:
        x_prev, y, t, hist, k0 = x0.clone(), x0.clone(), 1.0, [], 0
    else:
        x_prev, y, t, hist, k0 = state.x_prev.clone(), state.y.clone(), state.t, list(state.hist), state.k
    for _ in range(k0, n_iter):
        if eps_d is not None and len(hist) > 1 and hist[-2] - hist[-1] < eps_d * max(hist[-2], hist[-1]):
            break
        x = _direct(level, y, prox_iter)
        hist.append(level.objective(x))
        if callback is not None:
            callback(len(hist), x, hist[-1])
        tn = _t_next(t)
        theta = (t - 1.0) / tn if momentum else 0.0
        y = axpby(1.0 + theta, x, -theta, x_prev)
        x_prev, t = x, tn
        if on_state is not None:
            on_state(IterState(len(hist), x_prev, y, t, list(hist)))
    return x_prev, hist


def fista_batched(levels, x0s, n_iter: int, momentum: bool = True, prox_iter: int = 20, callback=None):
    """Alg. FISTA (Alg. ISTA without momentum) on several independent
    problems in lockstep: every iteration applies H and H^T of all of them as
    one batch (each pass of the scheme one launch over every instance; 2D
    grids of 128 to 512 points share their launches) and their proxes as one
    batched prox.  Per problem the iterates and objectives are bitwise those
    of ``fista``.  Returns (xs, [[F(x_k)] per problem]); ``callback(k, xs,
    Fs)`` runs after every iteration."""
    from . import tv_prox_batched
    batch = Batch([lv.plan for lv in levels])
    try:
        x_prev = [x.clone() for x in x0s]
        ys = [x.clone() for x in x0s]
        t = 1.0
        hist: List[List[float]] = [[] for _ in levels]
        for k in range(n_iter):
            d = batch.forward(ys)
            rs = [residual_f64(di, lv.data)[0] for di, lv in zip(d, levels)]
            gs = batch.adjoint(rs)
            zs = [axpby(1.0, y, -lv.alpha, g) for y, lv, g in zip(ys, levels, gs)]
            xs = tv_prox_batched(zs, [lv.alpha * lv.lam for lv in levels], prox_iter)
            dx = batch.forward(xs)
            halves = [residual_f64(di, lv.data)[1] for di, lv in zip(dx, levels)]
            Fs = [h + lv.lam * tv_smooth(x, 0.0) for h, lv, x in zip(halves, levels, xs)]
            for lv, h in zip(levels, halves):
                lv.res = math.sqrt(2.0 * h)
            for h, F in zip(hist, Fs):
                h.append(F)
            if callback is not None:
                callback(k + 1, xs, Fs)
            tn = _t_next(t)
            theta = (t - 1.0) / tn if momentum else 0.0
            ys = [axpby(1.0 + theta, x, -theta, xp) for x, xp in zip(xs, x_prev)]
            x_prev, t = xs, tn
        return x_prev, hist
    finally:
        batch.close()


def coarse_fista(level: Level, x0, v, lower, rho: float, q_c: int, eps_c: float, momentum: bool = True):
    """FISTA on phi = F_rho + <v, .> over x >= lower (the coarse proximal map
    is the projection, section V-E); returns (x, number of updates)."""
    def phi_value(x):
        return level.value_f(x) + level.lam * tv_smooth(x, rho) + dot_f64(v, x)

    x_prev = x0.clone()
    y = x0.clone()
    t = 1.0
    phi_prev = phi_value(x_prev)
    k = 0
    while k < q_c:
        _, g = level.smoothed(y, rho)
        g = axpby(1.0, g, 1.0, v, out=g)
        x = project(axpby(1.0, y, -level.alpha, g), lower)
        k += 1
        phi_x = phi_value(x)
        tn = _t_next(t)
        theta = (t - 1.0) / tn if momentum else 0.0
        y = axpby(1.0 + theta, x, -theta, x_prev)
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
    # gradients of two adjacent levels in one batch at every iteration that
    # may recurse (the coarse one ahead of the decision).  In 2D the grids
    # share their launches and the coarse gradient costs next to nothing; in
    # 3D the two run side by side on two streams, which pays once more than
    # about a quarter of the iterations recurse
    batch_levels: bool = True


@dataclass
class MGRecord:
    kind: str                 # "direct" or "recursive"
    F: float                  # F_h(x_k)
    coarse_updates: int = 0
    grad_ratio: float = 0.0   # ||R grad F_rho(y)|| / ||grad F_rho(y)|| at the decision
    depth: int = 0            # deepest level a recursive step reached (0: direct step)
    res: float = 0.0          # RES(x_k) = ||H x_k - p_hat|| at the target level


class _LevelPair:
    """Levels i and i + 1 whose data-term gradients run together: one batch
    over both plans, so that every pass of the scheme is one launch over both
    grids (2D grids of 128 to 512 points share the launches, the coarse level
    stepping at its own rate; otherwise the two run side by side on two
    streams).  Results equal the levels' own calls bitwise."""

    def __init__(self, fine: Level, coarse: Level):
        self.fine, self.coarse = fine, coarse
        self.batch = Batch([fine.plan, coarse.plan])

    def grads(self, y):
        """(grad f_i(y), R y, grad f_{i+1}(R y))."""
        yc = restrict(y)
        d = self.batch.forward([y, yc])
        rf, _ = residual_f64(d[0], self.fine.data)
        rc, _ = residual_f64(d[1], self.coarse.data)
        gf, gc = self.batch.adjoint([rf, rc])
        return gf, yc, gc

    def close(self):
        self.batch.close()


def _pair(pairs, levels, i: int, p: MGParams):
    """The batched pair (i, i + 1), made on first use, or None when the
    levels' gradients run one after the other."""
    if pairs is None or i + 1 >= len(levels):
        return None
    if i not in pairs:
        use = getattr(p, "batch_levels", True)
        pairs[i] = _LevelPair(levels[i], levels[i + 1]) if use else None
    return pairs[i]


def _decide(p: MGParams, g, y, y_tilde, k_d: int, k_r: int):
    """The decision rule at y with gradient g of the level's smoothed
    objective: (recursive?, ||R g|| / ||g||, R g)."""
    rg = restrict(g)
    ratio = math.sqrt(dot_f64(rg)) / max(math.sqrt(dot_f64(g)), 1e-300)
    far = False
    if y_tilde is not None:
        d = axpby(1.0, y, -1.0, y_tilde)
        far = math.sqrt(dot_f64(d)) > p.vartheta * math.sqrt(dot_f64(y_tilde))
    return (ratio > p.kappa) and (far or k_r == 0 or k_d > p.q_d), ratio, rg


def coarse_mg(levels, i: int, x0, v, lower, p: MGParams, pairs=None):
    """The coarse solve at level i of ``levels`` (0 the target level): FISTA
    on phi_i = F_rho,i + <v, .> over x >= lower, whose iterations after the
    first may take a recursive step to level i + 1 when there is one (same
    decision rule, coherence term and restricted bound as at the target
    level); with no coarser level it is ``coarse_fista``.  Returns (x,
    number of updates, deepest level reached).  ``pairs``: the batched
    level pairs of ``mg_fista`` (None: every gradient on its own level)."""
    lv = levels[i]
    has_next = i + 1 < len(levels)

    def phi_value(x):
        return lv.value_f(x) + lv.lam * tv_smooth(x, p.rho) + dot_f64(v, x)

    x_prev = x0.clone()
    y = x0.clone()
    t = 1.0
    phi_prev = phi_value(x_prev)
    k = k_d = k_r = 0
    y_tilde = None
    depth = i
    while k < p.q_c:
        pair = _pair(pairs, levels, i, p) if (has_next and k > 0) else None
        if pair is not None:
            g, xc0, gc = pair.grads(y)
            tv_smooth(y, p.rho, grad=g, scale=lv.lam, value=False)
        else:
            _, g = lv.smoothed(y, p.rho)
        g = axpby(1.0, g, 1.0, v, out=g)
        recursive = False
        if has_next and k > 0:
            recursive, _, rg = _decide(p, g, y, y_tilde, k_d, k_r)
        if recursive:
            k_d, k_r = 0, k_r + 1
            if pair is not None:
                tv_smooth(xc0, p.rho, grad=gc, scale=levels[i + 1].lam, value=False)
            else:
                xc0 = restrict(y)
                _, gc = levels[i + 1].smoothed(xc0, p.rho)
            xc, _, d = coarse_mg(levels, i + 1, xc0, axpby(1.0, rg, -1.0, gc), restrict_lower(y, lower), p,
                                 pairs)
            depth = max(depth, d)
            x = axpby(1.0, y, 1.0, prolong(axpby(1.0, xc, -1.0, xc0)))
            y_tilde = y.clone()
        else:
            k_d += 1
            x = project(axpby(1.0, y, -lv.alpha, g), lower)
        k += 1
        phi_x = phi_value(x)
        tn = _t_next(t)
        theta = (t - 1.0) / tn if p.momentum else 0.0
        y = axpby(1.0 + theta, x, -theta, x_prev)
        x_prev, t = x, tn
        if phi_prev - phi_x < p.eps_c * max(abs(phi_prev), abs(phi_x)):
            break
        phi_prev = phi_x
    return x_prev, k, depth


def mg_fista(fine: Level, coarse, x0, n_iter: int, params: MGParams = MGParams(), callback=None,
             state: Optional[IterState] = None, on_state=None):
    """Alg. FISTAMG; ``coarse`` is the next coarse level, or a list of levels
    from the next coarse one down (more than two levels).  Returns (x,
    [MGRecord]); ``callback(k, x_k, record)`` runs after every iteration.
    `n_iter`, `state` and `on_state` as in ``fista`` (the state carries the
    decision rule's K_d, K_r and y-tilde as well)."""
    levels = [fine] + (list(coarse) if isinstance(coarse, (list, tuple)) else [coarse])
    p = params
    pairs = {}
    try:
        return _mg_fista(levels, x0, n_iter, p, callback, pairs, state, on_state)
    finally:
        for pr in pairs.values():
            if pr is not None:
                pr.close()


def _mg_fista(levels, x0, n_iter: int, p: MGParams, callback, pairs, state=None, on_state=None):
    fine = levels[0]
    if state is None:
        x_prev, y, t, k_d, k_r, y_tilde, k0 = x0.clone(), x0.clone(), 1.0, 0, 0, None, 0
        hist: List[MGRecord] = []
    else:
        x_prev, y, t, k_d, k_r, k0 = state.x_prev.clone(), state.y.clone(), state.t, state.k_d, state.k_r, state.k
        y_tilde = None if state.y_tilde is None else state.y_tilde.clone()
        hist = list(state.hist)
    for k in range(k0 + 1, n_iter + 1):
        if p.eps_d is not None and len(hist) > 1 and \
                hist[-2].F - hist[-1].F < p.eps_d * max(hist[-2].F, hist[-1].F):
            break
        recursive = False
        ratio = 0.0
        rg = gf = None
        pair = _pair(pairs, levels, 0, p) if k > 1 else None
        if k > 1:
            # grad f(y) serves the decision (through grad F_rho) and a direct
            # step; with a batched pair the coarse gradient at R y comes along
            if pair is not None:
                gf, xc0, gc = pair.grads(y)
            else:
                _, gf = fine.grad_f(y)
            gF = gf.clone()
            tv_smooth(y, p.rho, grad=gF, scale=fine.lam, value=False)
            recursive, ratio, rg = _decide(p, gF, y, y_tilde, k_d, k_r)
        if recursive:
            k_d, k_r = 0, k_r + 1
            if pair is not None:
                tv_smooth(xc0, p.rho, grad=gc, scale=levels[1].lam, value=False)
            else:
                xc0 = restrict(y)
                _, gc = levels[1].smoothed(xc0, p.rho)
            v = axpby(1.0, rg, -1.0, gc)
            lower = restrict_lower(y)
            xc, nup, depth = coarse_mg(levels, 1, xc0, v, lower, p, pairs)
            x = axpby(1.0, y, 1.0, prolong(axpby(1.0, xc, -1.0, xc0)))
            y_tilde = y.clone()
            rec = MGRecord("recursive", 0.0, nup, ratio, depth)
        else:
            k_d += 1
            x = _direct(fine, y, p.prox_iter, gf)
            rec = MGRecord("direct", 0.0, 0, ratio)
        rec.F = fine.objective(x)
        rec.res = fine.res
        hist.append(rec)
        if callback is not None:
            callback(k, x, rec)
        tn = _t_next(t)
        theta = (t - 1.0) / tn if p.momentum else 0.0
        y = axpby(1.0 + theta, x, -theta, x_prev)
        x_prev, t = x, tn
        if on_state is not None:
            on_state(IterState(k, x_prev, y, t, list(hist), k_d, k_r, y_tilde))
    return x_prev, hist
