"""GPU: the error paths of plan creation, forced from the host (sensor
positions outside the grid, a time step above the stability bound, a bad
medium); they return before any kernel runs.  The deferred non-finite check
is tested in test_gpu_batch.py (test_check_finite_flag)."""
from dataclasses import replace
import math

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1603_02329_amd as pat  # noqa: E402

DEV = "cuda"


def _create(inst, **kw):
    return pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV, **kw)


@pytest.mark.parametrize("n", [(32, 32), (16, 16, 16)])
def test_plan_create_unstable_dt(n):
    """An explicit dt above the bound c_max dt / min dx <= 1/sqrt(d) is
    PAT_EUNSTABLE; at 0.99 of the bound the plan is created."""
    inst = synth.small_instance(41, n, nt=4, ns=3)
    cmax = float(inst.c0.max())
    bound = inst.desc.dx[0] / (cmax * math.sqrt(len(n)))
    ok = synth.Instance(replace(inst.desc, dt=0.99 * bound), inst.c0, inst.rho0, inst.alpha0_db, inst.sensors,
                        inst.p0)
    _create(ok).close()
    bad = synth.Instance(replace(inst.desc, dt=1.02 * bound), inst.c0, inst.rho0, inst.alpha0_db, inst.sensors,
                         inst.p0)
    with pytest.raises(pat.PatError) as e:
        _create(bad)
    assert e.value.code == pat.PAT_EUNSTABLE
    # the same dt becomes stable with a slower medium (c_max enters the bound)
    slow = synth.Instance(bad.desc, (inst.c0 * np.float32(0.95)).astype(np.float32), inst.rho0, inst.alpha0_db,
                          inst.sensors, inst.p0)
    _create(slow).close()


@pytest.mark.parametrize("n", [(32, 32), (16, 16, 16)])
def test_plan_create_rejects_sensor_outside_grid(n):
    inst = synth.small_instance(42, n, nt=4, ns=4)
    for j in range(len(n)):
        for v in (-0.25 * inst.desc.dx[j], (inst.desc.n[j] - 0.75) * inst.desc.dx[j]):
            s = np.array(inst.sensors, dtype=np.float64)
            s[2, j] = inst.desc.origin[j] + v
            with pytest.raises(pat.PatError) as e:
                pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, s, device=DEV)
            assert e.value.code == pat.PAT_EINVAL, (j, v)
    # on the last node exactly: accepted
    s = np.array(inst.sensors, dtype=np.float64)
    s[0, :] = [inst.desc.origin[j] + (inst.desc.n[j] - 1) * inst.desc.dx[j] for j in range(len(n))]
    pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, s, device=DEV).close()


def test_plan_create_rejects_bad_medium():
    inst = synth.small_instance(43, (32, 32), nt=4, ns=3)
    for field, val in (("c0", 0.0), ("c0", np.nan), ("rho0", -1.0), ("alpha0_db", -0.1), ("alpha0_db", np.inf)):
        arrs = dict(c0=inst.c0.copy(), rho0=inst.rho0.copy(), alpha0_db=inst.alpha0_db.copy())
        arrs[field][5, 7] = val
        with pytest.raises(pat.PatError) as e:
            pat.Plan(inst.desc, arrs["c0"], arrs["rho0"], arrs["alpha0_db"], inst.sensors, device=DEV)
        assert e.value.code == pat.PAT_EINVAL, field


def _eos_contraction(inst):
    """max |eta| max_k |k|^(y-1) of a lossy instance (eq. Twelve; the bound
    the plan checks for PAT_EOS_INIT), in float64."""
    d = inst.desc
    y = d.alpha_power
    a_conv = 100.0 * (1e-6 / (2 * math.pi)) ** y / (20.0 * math.log10(math.e))
    a0 = inst.alpha0_db.astype(np.float64) * a_conv
    eta = 2.0 * a0 * inst.c0.astype(np.float64) ** y * math.tan(math.pi * y / 2)
    kmax = math.sqrt(sum((math.pi / dx) ** 2 for dx in d.dx))
    return float(np.abs(eta).max()) * kmax ** (y - 1.0)


@pytest.mark.parametrize("n", [(32, 32), (16, 16, 16)])
def test_eos_init_rejects_slow_contraction(n):
    """PAT_EOS_INIT: a medium whose max |eta| |k|^(y-1) exceeds 0.05 is
    PAT_EINVAL (six fixed-point steps would not reach float rounding); just
    below the bound the plan is created, and without the flag the strong
    absorption is accepted."""
    inst = synth.small_instance(43, n, nt=4, ns=3, lossy=True)
    q = _eos_contraction(inst)
    for f, ok in ((0.95, True), (1.05, False)):
        a = (inst.alpha0_db.astype(np.float64) * (f * 0.05 / q)).astype(np.float32)
        eos = synth.Instance(replace(inst.desc, section3_density=True), inst.c0, inst.rho0, a, inst.sensors, inst.p0)
        if ok:
            _create(eos).close()
        else:
            with pytest.raises(pat.PatError) as e:
                _create(eos)
            assert e.value.code == pat.PAT_EINVAL
            _create(synth.Instance(inst.desc, inst.c0, inst.rho0, a, inst.sensors, inst.p0)).close()
