"""Pins of the adjoint-then-discretize operator (oracle/kspace.adjoint_atd):
the paper's adjoint system discretized with the forward's scheme.  It is
not the exact transpose, so it is pinned where the mathematics fixes it:
identity with the exact transpose where the scheme is time-symmetric
(homogeneous, no PML, lossless or absorption only), first-order convergence
to it in dt for a heterogeneous medium, linearity."""
from dataclasses import replace

import numpy as np

import synth
from oracle import kspace as K

T = 40 * 0.3 * 1e-4 / 1500  # 40 steps at CFL 0.3 of c = 1500 m/s, dx = 0.1 mm


def _case(cfl, **kw):
    inst = synth.small_instance(5, (32, 32), nt=2, ns=6, **kw)
    nt = int(round(T / (cfl * 1e-4 / 1500))) + 1
    desc = replace(inst.desc, cfl=cfl, nt=nt)
    a0 = None
    if kw.get("lossy", True):
        a0 = inst.alpha0_db if kw.get("hetero", True) else np.full(inst.c0.shape, 0.75, np.float32)
    op = K.make_plan(desc, inst.c0, inst.rho0, a0, inst.sensors)
    t = np.arange(nt) * op.dt
    h = np.stack([np.sin(2 * np.pi * t / T * (s + 1)) * np.exp(-((t - T / 2) / (T / 4)) ** 2)
                  for s in range(inst.ns)], axis=1)
    return op, h


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_atd_equals_the_transpose_homogeneous_lossless():
    """Data vanishing at t = 0 and t = T: the two adjoints agree to rounding
    (smooth data, and white data with the end samples zeroed); the sample at
    t = 0 -- the end of the adjoint's time integral -- enters with the
    trapezoid's half weight."""
    for cfl in (0.3, 0.15):
        op, h = _case(cfl, lossy=False, hetero=False, pml=0, pml_on=False)
        assert np.abs(h[0]).max() < 1e-12 and np.abs(h[-1]).max() < 1e-12
        assert _rel(K.adjoint_atd(op, h), K.adjoint(op, h)) < 1e-12
    op, _ = _case(0.3, lossy=False, hetero=False, pml=0, pml_on=False)
    h = np.random.default_rng(2).standard_normal((op.nt, 6))
    inner = h.copy()
    inner[0] = inner[-1] = 0.0
    assert _rel(K.adjoint_atd(op, inner), K.adjoint(op, inner)) < 1e-12
    first = np.zeros_like(h)
    first[0] = h[0]
    assert _rel(K.adjoint_atd(op, first), 0.5 * K.adjoint(op, first)) < 1e-12


def test_atd_equals_the_transpose_with_absorption_only():
    """The tau term of statea (rho0 L1[c0^2 tau d/dt (rho* / rho0)]) is the
    transpose of the forward's in a homogeneous medium: with eta set to 0
    the two adjoints agree to rounding."""
    op, h = _case(0.3, lossy=True, hetero=False, pml=0, pml_on=False)
    op.eta = np.zeros_like(op.eta)
    assert np.abs(op.tau).max() > 0
    assert _rel(K.adjoint_atd(op, h), K.adjoint(op, h)) < 1e-12


def test_atd_converges_to_the_transpose_at_first_order():
    """Heterogeneous lossless medium without PML: the difference halves
    with dt (the continuous adjoint is the limit of both)."""
    d = [_rel(K.adjoint_atd(*_case(cfl, lossy=False, hetero=True, pml=0, pml_on=False)),
              K.adjoint(*_case(cfl, lossy=False, hetero=True, pml=0, pml_on=False))) for cfl in (0.3, 0.15, 0.075)]
    assert 0 < d[0] < 1e-2
    for a, b in zip(d, d[1:]):
        assert 1.7 < a / b < 2.3, d


def test_atd_is_linear():
    op, h = _case(0.3, lossy=True, hetero=True, pml=4, pml_on=True)
    g = np.random.default_rng(3).standard_normal(h.shape)
    lhs = K.adjoint_atd(op, 2.0 * h - 0.5 * g)
    rhs = 2.0 * K.adjoint_atd(op, h) - 0.5 * K.adjoint_atd(op, g)
    assert _rel(lhs, rhs) < 1e-12
