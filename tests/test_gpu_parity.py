"""GPU parity: the HIP forward/adjoint against the FP64 oracle on the same
float32 inputs (relative L2 over all samples / all pixels)."""
from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import kspace as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1603_02329_amd as pat  # noqa: E402

DEV = "cuda"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def run_pair(inst, seed=0):
    plan = pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV)
    p0 = torch.from_numpy(inst.p0).to(DEV)
    d = plan.forward(p0).cpu().numpy()
    h = np.random.default_rng(seed).standard_normal((inst.desc.nt, inst.ns)).astype(np.float32)
    img = plan.adjoint(torch.from_numpy(h).to(DEV)).cpu().numpy()
    op = K.make_plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors)
    return plan, d, img, K.forward(op, inst.p0), K.adjoint(op, h), h


CASES = [
    dict(n=(16, 16), nt=10, ns=5, pml=3, lossy=True, hetero=True),
    dict(n=(32, 16), nt=15, ns=7, pml=2, lossy=False, hetero=True),
    dict(n=(16, 64), nt=12, ns=9, pml=4, lossy=True, hetero=True),
    dict(n=(64, 64), nt=30, ns=11, pml=6, lossy=True, hetero=True),
    dict(n=(128, 32), nt=20, ns=4, pml=8, lossy=False, hetero=False),
    dict(n=(32, 32), nt=25, ns=6, pml=0, lossy=True, hetero=True, pml_on=False),
    dict(n=(16, 16), nt=1, ns=5, pml=3, lossy=True, hetero=True),
    dict(n=(16, 16), nt=2, ns=5, pml=3, lossy=False, hetero=True),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c['n']}-nt{c['nt']}-{'lossy' if c['lossy'] else 'll'}" for c in CASES])
def test_small_parity(case):
    inst = synth.small_instance(100 + CASES.index(case), **case)
    print("case", case, flush=True)
    _, d, img, rd, ri, _ = run_pair(inst)
    assert rel(d, rd) <= 1e-5
    assert rel(img, ri) <= 1e-5


@pytest.mark.parametrize("n", [(64, 32), (512, 16)], ids=["64x32", "512x16"])
def test_line_array_parity(n):
    """A line of sensors along x, one grid spacing apart: each row it crosses
    carries more node groups of the adjoint's scatter than the row has lanes
    (4 at 64 points, 32 at 512), so a lane adds several of the step's sums;
    forward and adjoint against the oracle, eager and batched."""
    inst = synth.small_instance(140 + n[0], n, nt=12, ns=4, pml=2, lossy=True)
    dx = inst.desc.dx[0]
    k = min(n[0] - 8, 40)
    xs = 3.3 + np.arange(k, dtype=np.float64)
    inst = replace(inst, sensors=np.stack([xs * dx, np.full(k, 7.6 * dx)], axis=1))
    print("line array", n, k, flush=True)
    plan, d, img, rd, ri, h = run_pair(inst)
    assert rel(d, rd) <= 1e-5
    assert rel(img, ri) <= 1e-5
    b = pat.Batch([plan], chunk=4)
    hb = torch.from_numpy(h).to(DEV)
    assert torch.equal(b.adjoint([hb])[0].cpu(), torch.from_numpy(img))
    b.close()


def test_config1_parity_and_dot():
    inst = synth.config1()
    plan, d, img, rd, ri, h = run_pair(inst)
    print("cfg1", rel(d, rd), rel(img, ri), flush=True)
    assert rel(d, rd) <= 1e-5
    assert rel(img, ri) <= 1e-5
    # GPU dot test with float64 sums
    x = inst.p0.astype(np.float64)
    lhs = float((d.astype(np.float64) * h).sum())
    rhs = float((x * img.astype(np.float64)).sum())
    assert abs(lhs - rhs) <= 1e-6 * np.linalg.norm(d) * np.linalg.norm(h)


def test_config2_short_parity():
    inst = synth.config2()
    inst = synth.Instance(replace(inst.desc, nt=150), inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, inst.p0)
    _, d, img, rd, ri, _ = run_pair(inst)
    print("cfg2/150", rel(d, rd), rel(img, ri), flush=True)
    assert rel(d, rd) <= 1e-5
    assert rel(img, ri) <= 1e-5


CASES3 = [
    dict(n=(16, 16, 16), nt=8, ns=5, pml=2, lossy=True, hetero=True),
    dict(n=(32, 16, 64), nt=10, ns=7, pml=3, lossy=True, hetero=True),
    dict(n=(16, 32, 16), nt=9, ns=4, pml=2, lossy=False, hetero=True),
    dict(n=(32, 32, 32), nt=12, ns=6, pml=0, lossy=True, hetero=True, pml_on=False),
    dict(n=(64, 64, 64), nt=10, ns=9, pml=6, lossy=True, hetero=True),
    dict(n=(64, 128, 32), nt=8, ns=5, pml=4, lossy=False, hetero=True),
]


@pytest.mark.parametrize("case", CASES3, ids=[f"{c['n']}-nt{c['nt']}" for c in CASES3])
def test_small_parity_3d(case):
    inst = synth.small_instance(200 + CASES3.index(case), **case)
    print("case3", case, flush=True)
    _, d, img, rd, ri, _ = run_pair(inst)
    print("rel", rel(d, rd), rel(img, ri), flush=True)
    assert rel(d, rd) <= 1e-5
    assert rel(img, ri) <= 1e-5


def test_config5_short_parity():
    """128^3 lossy medium and phantom, planar 128x128 sensor moved to z = 64
    (inside the source region, so that 12 samples already carry signal)."""
    inst = synth.config5()
    d = inst.desc
    sens = synth.plane_sensors(128, 128, d.dx, d.origin, 64)
    inst = synth.Instance(replace(d, nt=12), inst.c0, inst.rho0, inst.alpha0_db, sens, inst.p0)
    _, d, img, rd, ri, _ = run_pair(inst)
    print("cfg5/12", rel(d, rd), rel(img, ri), flush=True)
    assert rel(d, rd) <= 1e-5
    assert rel(img, ri) <= 1e-5


SMOOTH_P0_CASES = [
    dict(n=(64, 32), nt=20, ns=6, pml=3, lossy=True, hetero=True),
    dict(n=(32, 128), nt=12, ns=5, pml=4, lossy=False, hetero=True),
    dict(n=(16, 16), nt=1, ns=5, pml=3, lossy=True, hetero=True),
    dict(n=(16, 32, 16), nt=10, ns=6, pml=3, lossy=True, hetero=True),
    dict(n=(32, 16, 16), nt=8, ns=4, pml=2, lossy=False, hetero=True),
]


@pytest.mark.parametrize("case", SMOOTH_P0_CASES,
                         ids=[f"{c['n']}-nt{c['nt']}-{'lossy' if c['lossy'] else 'll'}" for c in SMOOTH_P0_CASES])
def test_smoothed_p0_parity(case):
    """Plans that filter the initial pressure (H = H0 S, H^T = S H0^T, the
    window applied by a column pass between two row passes) against the
    oracle's filter (numpy FFT): forward, adjoint and the
    adjoint-then-discretize operator; the filter changes the result."""
    inst = synth.small_instance(140 + SMOOTH_P0_CASES.index(case), **case)
    sm = synth.Instance(replace(inst.desc, smooth_p0=True), inst.c0, inst.rho0, inst.alpha0_db,
                        inst.sensors, inst.p0, inst.name)
    print("case", case, flush=True)
    plan, d, img, rd, ri, h = run_pair(sm)
    assert rel(d, rd) <= 1e-5
    assert rel(img, ri) <= 1e-5
    _, d0, img0, _, _, _ = run_pair(inst)
    assert rel(d0, d) > 1e-4 and rel(img0, img) > 1e-4
    if case["nt"] > 1:
        op = K.make_plan(sm.desc, sm.c0, sm.rho0, sm.alpha0_db, sm.sensors)
        ia = plan.adjoint_atd(torch.from_numpy(h).to(DEV)).cpu().numpy()
        assert rel(ia, K.adjoint_atd(op, h)) <= 1e-5


EOS_CASES = [
    dict(n=(64, 32), nt=20, ns=6, pml=3, lossy=True, hetero=True),
    dict(n=(16, 16), nt=2, ns=5, pml=3, lossy=True, hetero=True),
    dict(n=(32, 32), nt=25, ns=6, pml=0, lossy=True, hetero=True, pml_on=False),
    dict(n=(16, 32, 16), nt=10, ns=6, pml=3, lossy=True, hetero=True),
]


@pytest.mark.parametrize("case", EOS_CASES,
                         ids=[f"{c['n']}-nt{c['nt']}{'-nopml' if c.get('pml_on') is False else ''}" for c in EOS_CASES])
def test_eos_initial_density_parity(case):
    """Plans whose density starts from the t = 0 equation of state
    (PAT_EOS_INIT: six fixed-point steps of x <- p0/c0^2 + eta L2 x on the
    GPU, their transpose in the adjoint) against the oracle's option, which
    iterates to convergence: forward and adjoint; the option changes the
    result."""
    inst = synth.small_instance(170 + EOS_CASES.index(case), **case)
    eo = synth.Instance(replace(inst.desc, section3_density=True), inst.c0, inst.rho0, inst.alpha0_db,
                        inst.sensors, inst.p0, inst.name)
    print("case", case, flush=True)
    plan, d, img, rd, ri, h = run_pair(eo)
    assert rel(d, rd) <= 1e-5
    assert rel(img, ri) <= 1e-5
    _, d0, img0, _, _, _ = run_pair(inst)
    print("change", rel(d0, d), rel(img0, img), flush=True)
    assert rel(d0, d) > 1e-5 and rel(img0, img) > 1e-5


def test_smoothed_p0_segmented_forward_is_bitwise():
    """The filter runs in the first segment of a checkpointed forward: any
    split of the time axis reproduces the unsegmented data bitwise."""
    inst = synth.small_instance(150, (64, 64), nt=24, ns=7, pml=4, lossy=True)
    desc = replace(inst.desc, smooth_p0=True)
    plan = pat.Plan(desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV)
    p0 = torch.from_numpy(inst.p0).to(DEV)
    full = plan.forward(p0).clone()
    state = torch.empty(plan.state_bytes, dtype=torch.uint8, device=DEV)
    seg = torch.full_like(full, float("nan"))
    for a, b in [(0, 7), (7, 24)]:
        plan.forward_range(p0 if a == 0 else None, seg, a, b, state)
    torch.cuda.synchronize()
    assert torch.equal(seg, full)


@pytest.mark.parametrize("case", ["2d", "2d-smooth-p0", "2d-eos", "3d", "3d-eos"])
def test_gpu_adjoint_is_dense_transpose_of_gpu_forward(case):
    """The GPU adjoint against the GPU forward itself: H built column by
    column from pat_forward on unit images, H^T row by row from pat_adjoint
    on unit data (lossy, heterogeneous, with PML); they agree entrywise to
    float32 rounding.  3D: 96 sampled columns of the 4096."""
    if case.startswith("3d"):
        inst = synth.small_instance(160, (16, 16, 16), nt=5, ns=3, pml=2, lossy=True)
    else:
        inst = synth.small_instance(161, (16, 16), nt=6, ns=3, pml=3, lossy=True)
    desc = replace(inst.desc, smooth_p0=(case == "2d-smooth-p0"), section3_density=case.endswith("eos"))
    plan = pat.Plan(desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV)
    N, M = plan.npoints, inst.desc.nt * inst.ns
    cols = np.arange(N) if not case.startswith("3d") else np.sort(np.random.default_rng(4).choice(N, 96, replace=False))
    A = np.zeros((M, len(cols)))
    for j, i in enumerate(cols):
        e = torch.zeros(N, device=DEV)
        e[i] = 1.0
        A[:, j] = plan.forward(e.reshape(plan.shape)).cpu().numpy().ravel()
    AT = np.zeros((len(cols), M))
    for m in range(M):
        h = torch.zeros(M, device=DEV)
        h[m] = 1.0
        AT[:, m] = plan.adjoint(h.reshape(inst.desc.nt, inst.ns)).cpu().numpy().ravel()[cols]
    err = np.abs(A.T - AT).max() / np.abs(A).max()
    print(case, "max |H^T - adjoint| / max |H|", err, flush=True)
    assert err <= 2e-6
