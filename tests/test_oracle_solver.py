"""Pins of the FP64 reconstruction iterations (oracle/solver.py) and of the
operators they add (smoothed TV, restricted bound): finite differences,
brute force, dense linear algebra and a library NNLS solver."""
import math

import numpy as np
import pytest
from scipy.optimize import nnls

import synth
from oracle import kspace as K
from oracle import prox, solver, transfer


def test_tv_smooth_gradient_is_the_derivative():
    rng = np.random.default_rng(11)
    for shape in [(7, 9), (4, 5, 3)]:
        x = rng.standard_normal(shape)
        rho = 0.3
        v, g = prox.tv_smooth(x, rho)
        eps = 1e-6
        fd = np.zeros_like(x)
        for idx in np.ndindex(*shape):
            e = np.zeros_like(x)
            e[idx] = eps
            fd[idx] = (prox.tv_smooth(x + e, rho)[0] - prox.tv_smooth(x - e, rho)[0]) / (2 * eps)
        assert np.max(np.abs(fd - g)) < 1e-7 * max(1.0, np.max(np.abs(g)))
        # brute-force value from the definition
        val = 0.0
        for idx in np.ndindex(*shape):
            q = rho * rho
            for a in range(len(shape)):
                if idx[a] < shape[a] - 1:
                    j = list(idx)
                    j[a] += 1
                    q += (x[idx] - x[tuple(j)]) ** 2
            val += math.sqrt(q) - rho
        assert abs(val - v) < 1e-12 * abs(val)


def test_tv_smooth_rho0_is_the_tv():
    x = np.random.default_rng(12).standard_normal((10, 12))
    assert abs(prox.tv_smooth(x, 0.0)[0] - prox.tv_value(x)) < 1e-12 * prox.tv_value(x)


def test_restrict_lower_brute_force_and_feasibility():
    rng = np.random.default_rng(13)
    for shape in [(6, 8), (4, 6, 2)]:
        y = rng.standard_normal(shape)
        lo = transfer.restrict_lower(y)
        nd = len(shape)
        for I in np.ndindex(*lo.shape):
            block = [y[tuple(2 * i + d for i, d in zip(I, delta))] for delta in np.ndindex(*([2] * nd))]
            assert abs(lo[I] - (sum(block) / len(block) - min(block))) < 1e-14
        # any coarse point above the bound keeps the prolonged correction feasible
        # even where y itself is negative (section V-C)
        for _ in range(20):
            xc = lo + np.abs(rng.standard_normal(lo.shape))
            x = y + transfer.prolong(xc - transfer.restrict(y))
            assert x.min() >= -1e-12
        x = y + transfer.prolong(lo - transfer.restrict(y))  # on the bound: each block's minimum hits 0
        assert abs(x.min()) < 1e-12


def _dense(op):
    n = int(np.prod(op.shape))
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(K.forward(op, e.reshape(op.shape)).ravel())
    return np.stack(cols, axis=1)


def _tiny(seed=21, n=(8, 8), nt=24, ns=8):
    inst = synth.small_instance(seed, n, nt=nt, ns=ns, pml=2, lossy=True)
    op = K.make_plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors)
    p_true = np.abs(np.random.default_rng(seed).standard_normal(op.shape))
    data = K.forward(op, p_true)
    return op, data


def test_power_iteration_matches_dense_eigenvalue():
    op, _ = _tiny()
    H = _dense(op)
    lmax = float(np.linalg.eigvalsh(H.T @ H).max())
    est = solver.power_iteration(op, n_iter=300, seed=1)
    assert abs(est - lmax) < 1e-6 * lmax


def test_fista_lambda0_reaches_the_nnls_minimum():
    op, data = _tiny()
    H = _dense(op)
    noise = 0.05 * np.random.default_rng(5).standard_normal(data.shape) * np.abs(data).max()
    p_hat = data + noise
    x_star, res = nnls(H, p_hat.ravel())
    f_star = 0.5 * res * res
    L = solver.power_iteration(op, n_iter=100)
    lv = solver.Level(op, p_hat, lam=0.0, alpha=1.0 / L)
    x, hist = solver.fista(lv, np.zeros(op.shape), 400)
    xi, hist_i = solver.fista(lv, np.zeros(op.shape), 400, momentum=False)
    assert x.min() >= 0 and xi.min() >= 0
    assert min(hist) >= f_star * (1 - 1e-12) and min(hist_i) >= f_star * (1 - 1e-12)
    # the convergence bounds of Beck and Teboulle from x0 = 0: FISTA
    # F(x_k) - F* <= 2 L ||x*||^2 / (k + 1)^2, ISTA <= L ||x*||^2 / (2 k)
    r2 = float(np.sum(x_star ** 2))
    for k in (50, 100, 200, 400):
        assert hist[k - 1] - f_star <= 2 * L * r2 / (k + 1) ** 2
        assert hist_i[k - 1] - f_star <= L * r2 / (2 * k)
    assert hist[-1] - f_star < 1e-4 * f_star
    assert hist_i[-1] - f_star > 2 * L * r2 / 401 ** 2  # plain ISTA is slower here: momentum matters


def test_ista_is_monotone_with_step_one_over_L():
    op, data = _tiny(seed=22)
    L = solver.power_iteration(op, n_iter=100)
    lv = solver.Level(op, data, lam=1e-3 * float(np.abs(data).max()), alpha=1.0 / L)
    _, hist = solver.fista(lv, np.zeros(op.shape), 15, momentum=False, prox_iter=200)
    assert all(b <= a * (1 + 1e-9) for a, b in zip(hist, hist[1:]))


def _two_level(seed=0, n=32, nt=40, ns=16, pml=4):
    f, c = synth.two_level(91, seed, n, 1e-4, pml, nt, ns)
    opf = K.make_plan(f.desc, f.c0, f.rho0, f.alpha0_db, f.sensors)
    opc = K.make_plan(c.desc, c.c0, c.rho0, c.alpha0_db, c.sensors)
    data = K.forward(opf, f.p0.astype(np.float64))
    return opf, opc, data, f, c


def test_mg_recursive_step_is_the_coherent_coarse_step():
    """With one coarse update and no momentum, the recursive step must be
    y + P(max(R y - alpha_c R grad F_rho,h(y), lower) - R y): the coarse
    gradient at x0 = R y is replaced by the restricted fine gradient
    (first-order coherence, equation Fourteen), then projected onto the
    restricted bound (equation constraint) and prolonged."""
    opf, opc, data, f, c = _two_level()
    Lf = solver.power_iteration(opf, n_iter=40)
    Lc = solver.power_iteration(opc, n_iter=40)
    fine = solver.Level(opf, data, lam=1e-4, alpha=1.0 / Lf)
    coarse = solver.Level(opc, data[::2], lam=1e-4, alpha=1.0 / Lc)
    prm = solver.MGParams(q_c=1, momentum=False)
    x, hist = solver.mg_fista(fine, coarse, np.zeros(opf.shape), 2, prm)
    assert [r.kind for r in hist] == ["direct", "recursive"]
    y, _ = solver.fista(fine, np.zeros(opf.shape), 1, momentum=False)  # x_1 = P_L(x_0) = y_2
    _, gf = solver.smoothed(fine, y, prm.rho)
    ry = transfer.restrict(y)
    xc = np.maximum(ry - coarse.alpha * transfer.restrict(gf), transfer.restrict_lower(y))
    expect = y + transfer.prolong(xc - ry)
    assert np.max(np.abs(x - expect)) <= 1e-12 * np.max(np.abs(expect))


def test_mg_fista_lambda0_reaches_the_nnls_minimum():
    opf, opc, data, f, c = _two_level(n=16, nt=30, ns=12, pml=2)
    H = _dense(opf)
    x_star, res = nnls(H, data.ravel())
    f_star = 0.5 * res * res
    Lf = solver.power_iteration(opf, n_iter=60)
    Lc = solver.power_iteration(opc, n_iter=60)
    fine = solver.Level(opf, data, lam=0.0, alpha=1.0 / Lf)
    coarse = solver.Level(opc, data[::2], lam=0.0, alpha=1.0 / Lc)
    x, hist = solver.mg_fista(fine, coarse, np.zeros(opf.shape), 300)
    kinds = [r.kind for r in hist]
    assert "recursive" in kinds and "direct" in kinds
    assert x.min() >= -1e-12 * np.abs(x).max()
    f0 = 0.5 * float(np.sum(data * data))
    assert hist[-1].F - f_star < 1e-4 * f0


def test_mg_first_iterations_follow_the_decision_rule():
    """k = 1 is direct; k = 2 is recursive when the restricted gradient is
    large (K_r = 0); a recursive step keeps the iterate feasible."""
    opf, opc, data, f, c = _two_level()
    Lf = solver.power_iteration(opf, n_iter=40)
    Lc = solver.power_iteration(opc, n_iter=40)
    fine = solver.Level(opf, data, lam=1e-4, alpha=1.0 / Lf)
    coarse = solver.Level(opc, data[::2], lam=1e-4, alpha=1.0 / Lc)
    x, hist = solver.mg_fista(fine, coarse, np.zeros(opf.shape), 4)
    assert hist[0].kind == "direct"
    assert hist[1].grad_ratio > 0.25 and hist[1].kind == "recursive"
    assert 1 <= hist[1].coarse_updates <= 8
    assert x.min() >= -1e-12 * np.abs(x).max()


def test_restrict_lower_with_a_fine_bound():
    """The bound of an intermediate level: lower[I] = (R y)[I] - min over
    the block of (y - l), by brute force; every coarse x >= lower keeps the
    prolonged correction above l, and x = lower touches l in every block."""
    rng = np.random.default_rng(14)
    for shape in [(6, 8), (4, 6, 2)]:
        y = rng.standard_normal(shape)
        fl = rng.standard_normal(shape)
        lo = transfer.restrict_lower(y, fl)
        nd = len(shape)
        for I in np.ndindex(*lo.shape):
            pts = [tuple(2 * i + d for i, d in zip(I, delta)) for delta in np.ndindex(*([2] * nd))]
            expect = sum(y[p] for p in pts) / len(pts) - min(y[p] - fl[p] for p in pts)
            assert abs(lo[I] - expect) < 1e-14
        for _ in range(20):
            xc = lo + np.abs(rng.standard_normal(lo.shape))
            assert (y + transfer.prolong(xc - transfer.restrict(y)) - fl).min() >= -1e-12
        gap = y + transfer.prolong(lo - transfer.restrict(y)) - fl
        assert abs(gap.min()) < 1e-12
        assert np.allclose(transfer.restrict_lower(y, np.zeros(shape)), transfer.restrict_lower(y), atol=0)


def _levels(count, seed=0, n=16, nt=30, ns=12, pml=2, lam=0.0):
    insts = synth.multi_level(91, seed, n, 1e-4, pml, nt, ns, count)
    ops = [K.make_plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors) for i in insts]
    data = K.forward(ops[0], insts[0].p0.astype(np.float64))
    lv = []
    for k, op in enumerate(ops):
        L = solver.power_iteration(op, n_iter=60)
        lv.append(solver.Level(op, data[::2 ** k][:op.nt], lam=lam, alpha=1.0 / L))
    return ops, data, lv


def test_mg_three_levels_lambda0_reaches_the_nnls_minimum():
    """Three levels (16^2, 8^2, 4^2): the recursion reaches the coarsest
    level, every iterate stays feasible, and F converges to the NNLS
    minimum of the fine problem."""
    ops, data, lv = _levels(3)
    H = _dense(ops[0])
    x_star, res = nnls(H, data.ravel())
    f_star = 0.5 * res * res
    # coarse solves stop at a 0.1 % decrease, so that they run long enough
    # to recurse themselves
    x, hist = solver.mg_fista(lv[0], lv[1:], np.zeros(ops[0].shape), 300, solver.MGParams(eps_c=1e-3))
    assert max(r.depth for r in hist) == 2
    assert x.min() >= -1e-12 * np.abs(x).max()
    f0 = 0.5 * float(np.sum(data * data))
    assert hist[-1].F - f_star < 1e-4 * f0


def test_mg_two_level_list_equals_two_level_call():
    """A list of one coarse level runs exactly the two-level algorithm."""
    ops, data, lv = _levels(2, lam=1e-4)
    x1, h1 = solver.mg_fista(lv[0], lv[1], np.zeros(ops[0].shape), 6)
    x2, h2 = solver.mg_fista(lv[0], [lv[1]], np.zeros(ops[0].shape), 6)
    assert np.array_equal(x1, x2) and [r.F for r in h1] == [r.F for r in h2]
    assert all(r.depth in (0, 1) for r in h1)


def test_mg_recursive_step_in_3d():
    """3D (16^3 -> 8^3), one coarse update, no momentum: the recursive step
    is y + P(max(R y - alpha_c R grad F_rho,h(y), lower) - R y), as in 2D."""
    f, c = synth.multi_level_3d(92, 0, 16, 2e-4, 2, 12, 2)
    opf = K.make_plan(f.desc, f.c0, f.rho0, f.alpha0_db, f.sensors)
    opc = K.make_plan(c.desc, c.c0, c.rho0, c.alpha0_db, c.sensors)
    data = K.forward(opf, f.p0.astype(np.float64))
    fine = solver.Level(opf, data, lam=1e-4, alpha=1.0 / solver.power_iteration(opf, n_iter=20))
    coarse = solver.Level(opc, data[::2], lam=1e-4, alpha=1.0 / solver.power_iteration(opc, n_iter=20))
    prm = solver.MGParams(q_c=1, momentum=False, kappa=0.125, rho=3e-2)
    x, hist = solver.mg_fista(fine, coarse, np.zeros(opf.shape), 2, prm)
    assert [r.kind for r in hist] == ["direct", "recursive"]
    y, _ = solver.fista(fine, np.zeros(opf.shape), 1, momentum=False)
    _, gf = solver.smoothed(fine, y, prm.rho)
    ry = transfer.restrict(y)
    xc = np.maximum(ry - coarse.alpha * transfer.restrict(gf), transfer.restrict_lower(y))
    expect = y + transfer.prolong(xc - ry)
    assert np.max(np.abs(x - expect)) <= 1e-12 * np.max(np.abs(expect))
