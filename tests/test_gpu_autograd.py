"""GPU: autograd wrappers -- central differences of the quadratic loss,
backward against the FP64 oracle adjoint, checkpointed forward and replay."""
from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import kspace as K

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1603_02329_amd as pat  # noqa: E402
from paper_1603_02329_amd.autograd import PatLeastSquares, PatOperator, replay_segment  # noqa: E402

DEV = "cuda"


def _setup(inst, seed=0):
    plan = pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV)
    rng = np.random.default_rng(seed)
    target = rng.standard_normal((inst.desc.nt, inst.ns)).astype(np.float32)
    return plan, torch.from_numpy(target).to(DEV)


@pytest.mark.parametrize("n", [(64, 64), (32, 32, 32)])
def test_backward_matches_oracle_and_finite_differences(n):
    inst = synth.small_instance(700, n, nt=30, ns=9, pml=4, lossy=True)
    plan, target = _setup(inst)
    x = torch.from_numpy(inst.p0).to(DEV).requires_grad_(True)
    f = PatLeastSquares.apply(x, target, plan)
    f.backward()
    g = x.grad.detach().cpu().numpy().astype(np.float64)
    # oracle: grad = H^T (H x - target)
    op = K.make_plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors)
    r = K.forward(op, inst.p0) - target.cpu().numpy()
    ref = K.adjoint(op, r)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) <= 1e-5
    # central difference along a random direction: the loss is exactly
    # quadratic, so the difference has no truncation error for any step; a
    # step of the size of x keeps float32 cancellation out of the difference
    v = torch.from_numpy(np.random.default_rng(1).standard_normal(inst.p0.shape).astype(np.float32)).to(DEV)
    eps = float(x.detach().norm()) / float(v.norm())
    with torch.no_grad():
        fp = float(PatLeastSquares.apply(x.detach() + eps * v, target, plan))
        fm = float(PatLeastSquares.apply(x.detach() - eps * v, target, plan))
    fd = (fp - fm) / (2 * eps)
    an = float((x.grad * v).double().sum())
    assert abs(fd - an) <= 1e-4 * abs(an)


def test_operator_autograd_and_checkpoints():
    inst = synth.small_instance(701, (32, 32, 16), nt=37, ns=6, pml=3, lossy=True)
    plan, target = _setup(inst)
    x = torch.from_numpy(inst.p0).to(DEV).requires_grad_(True)
    plain = plan.forward(x.detach()).clone()
    d = PatOperator.apply(x, plan, 10)
    assert torch.equal(d, plain)  # segmented forward is bitwise the plain forward
    loss = 0.5 * ((d - target) ** 2).sum()
    loss.backward()
    ref = plan.adjoint((plain - target).contiguous())
    assert torch.allclose(x.grad, ref, rtol=1e-6, atol=1e-6 * float(ref.abs().max()))


def test_replay_from_checkpoint_is_bitwise():
    inst = synth.small_instance(702, (32, 32, 32), nt=41, ns=5, pml=3, lossy=True)
    plan, _ = _setup(inst)
    x = torch.from_numpy(inst.p0).to(DEV)
    from paper_1603_02329_amd.autograd import forward_checkpointed
    data, ckpts = forward_checkpointed(plan, x, 10)
    assert [n for n, _ in ckpts] == [10, 20, 30, 40]
    assert torch.equal(data, plan.forward(x))
    seg = replay_segment(plan, ckpts, x, 23, 35)
    assert torch.equal(seg, data[23:35])
