"""GPU: the longest axes the library accepts (1024 points in 2D, 256 in 3D).

Their kernels differ from the shorter ones (a 1024-point column spans two
wavefronts, so its transforms synchronise the block; the 3D passes take
256-point axes in every position).  Thin grids with one long axis are
checked against the FP64 oracle element by element; the largest grids
(1024^2, 256^3) against what holds at any size: the exact solution of the
homogeneous lossless periodic problem (p^n = F^-1[F p0 cos(c |k| n dt)],
exact for the k-space scheme) and the dot-product identity of the adjoint.
"""
from dataclasses import replace

import numpy as np
import pytest
import scipy.fft as sfft

import synth
from oracle import kspace as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1603_02329_amd as pat  # noqa: E402

DEV = "cuda"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


LONG = [
    dict(n=(1024, 32), nt=14, ns=6, pml=8, lossy=True),
    dict(n=(32, 1024), nt=12, ns=5, pml=8, lossy=False),
    dict(n=(1024, 16), nt=10, ns=4, pml=0, lossy=True, pml_on=False),
    dict(n=(256, 16, 16), nt=8, ns=5, pml=3, lossy=True),
    dict(n=(16, 256, 16), nt=8, ns=5, pml=3, lossy=False),
    dict(n=(16, 16, 256), nt=8, ns=5, pml=3, lossy=True),
]


@pytest.mark.parametrize("case", LONG, ids=[f"{c['n']}-{'lossy' if c['lossy'] else 'll'}" for c in LONG])
def test_long_axis_parity(case):
    inst = synth.small_instance(300 + LONG.index(case), **case)
    print("case", case, flush=True)
    plan = pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV)
    d = plan.forward(torch.from_numpy(inst.p0).to(DEV)).cpu().numpy()
    h = np.random.default_rng(3).standard_normal((inst.desc.nt, inst.ns)).astype(np.float32)
    img = plan.adjoint(torch.from_numpy(h).to(DEV)).cpu().numpy()
    op = K.make_plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors)
    ed, ei = rel(d, K.forward(op, inst.p0)), rel(img, K.adjoint(op, h))
    print(f"rel forward {ed:.2e} adjoint {ei:.2e}", flush=True)
    assert ed <= 1e-5 and ei <= 1e-5


def _exact_data(inst, dt, nt):
    """Sensor data of the homogeneous lossless periodic problem, exactly:
    p^n = F^-1[F p0 cos(c |k| n dt)], sampled by the sensors' linear taps."""
    desc = inst.desc
    nd = desc.ndim
    ks = [2 * np.pi * np.fft.fftfreq(desc.n[j], desc.dx[j]) for j in range(nd)]
    mesh = np.meshgrid(*reversed(ks), indexing="ij")  # numpy axis order (z, y, x)
    kmag = np.sqrt(sum(m ** 2 for m in mesh))
    c = float(inst.c0.flat[0])
    P0 = sfft.fftn(inst.p0.astype(np.float64), workers=8)
    idx, w = K.sensor_weights(desc, inst.sensors)
    out = np.empty((nt, idx.shape[0]))
    for n in range(nt):
        p = sfft.ifftn(P0 * np.cos(c * kmag * n * dt), workers=8).real.ravel()
        out[n] = (w * p[idx]).sum(axis=1)
    return out


@pytest.mark.parametrize("n,nt", [((1024, 1024), 24), ((256, 256, 256), 6)])
def test_max_size_exact_solution(n, nt):
    """Largest grids, homogeneous lossless, no PML: the data equal the
    closed-form solution at the sensors."""
    inst = synth.small_instance(320 + len(n), n, nt=nt, ns=16, pml=0, lossy=False, hetero=False, pml_on=False)
    print("max size", n, flush=True)
    plan = pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV)
    d = plan.forward(torch.from_numpy(inst.p0).to(DEV)).cpu().numpy()
    dt = 0.3 * inst.desc.dx[0] / 1500.0
    assert plan.dt == pytest.approx(dt, rel=1e-12)
    ref = _exact_data(inst, dt, nt)
    e = rel(d, ref)
    print(f"rel to the exact solution {e:.2e}", flush=True)
    assert e <= 1e-5
    del plan
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,nt", [((1024, 1024), 16), ((256, 256, 256), 5)])
def test_max_size_dot_identity(n, nt):
    """Largest grids, lossy heterogeneous with PML: <H x, h> = <x, H^T h>
    with float64 sums, to float32 rounding."""
    inst = synth.small_instance(330 + len(n), n, nt=nt, ns=24, pml=16 if len(n) == 2 else 8, lossy=True)
    print("max size dot", n, flush=True)
    plan = pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV)
    d = plan.forward(torch.from_numpy(inst.p0).to(DEV)).cpu().numpy().astype(np.float64)
    h = np.random.default_rng(8).standard_normal((nt, inst.ns)).astype(np.float32)
    img = plan.adjoint(torch.from_numpy(h).to(DEV)).cpu().numpy().astype(np.float64)
    lhs = float((d * h).sum())
    rhs = float((inst.p0.astype(np.float64) * img).sum())
    gap = abs(lhs - rhs) / (np.linalg.norm(d) * np.linalg.norm(h))
    print(f"dot gap {gap:.2e}", flush=True)
    assert gap <= 1e-6
    assert np.isfinite(img).all() and np.linalg.norm(img) > 0
    del plan
    torch.cuda.empty_cache()
