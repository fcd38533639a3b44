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


def test_batched_autograd_matches_the_oracle():
    """Batched least squares through torch.autograd: loss and gradients of
    three uneven instances against the FP64 oracle (loss 1e-6 relative,
    gradients rel-L2 1e-5), and the gradients equal the batched adjoint of
    the residuals bitwise."""
    from paper_1603_02329_amd.autograd import PatBatchLeastSquares
    specs = [dict(n=(64, 64), nt=41, ns=9, pml=6), dict(n=(32, 32), nt=23, ns=5, pml=3),
             dict(n=(64, 32), nt=31, ns=7, pml=4)]
    insts = [synth.small_instance(900 + k, **s) for k, s in enumerate(specs)]
    plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=DEV) for i in insts]
    batch = pat.Batch(plans, chunk=8)
    rng = np.random.default_rng(9)
    targets_np = [rng.standard_normal((i.desc.nt, i.ns)).astype(np.float32) for i in insts]
    xs = [torch.from_numpy(i.p0).to(DEV).requires_grad_(True) for i in insts]
    targets = [torch.from_numpy(t).to(DEV) for t in targets_np]
    loss = PatBatchLeastSquares.apply(batch, targets, *xs)
    loss.backward()
    torch.cuda.synchronize()
    ref_loss = 0.0
    for k, inst in enumerate(insts):
        op = K.make_plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors)
        r = K.forward(op, inst.p0.astype(np.float64)) - targets_np[k]
        ref_loss += 0.5 * float(np.sum(r * r))
        g_ref = K.adjoint(op, r)
        g = xs[k].grad.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(g - g_ref) <= 1e-5 * np.linalg.norm(g_ref), k
    assert abs(float(loss.detach()) - ref_loss) <= 1e-6 * ref_loss
    datas = batch.forward([x.detach() for x in xs])
    res = [pat.residual_f64(d, t)[0] for d, t in zip(datas, targets)]
    imgs = batch.adjoint(res)
    torch.cuda.synchronize()
    for k in range(len(insts)):
        assert torch.equal(imgs[k], xs[k].grad), k
    # the loss is the sum of the per-instance residual norms in index order
    assert float(loss.detach()) == sum(pat.residual_f64(d, t)[1] for d, t in zip(datas, targets))
    batch.close()
