"""GPU parity at the workloads' full sizes against stored FP64-oracle results.

The reference files in tests/golden/ are written by make_golden.py, which
calls only the oracle on the seeded synthetic inputs.  The GPU runs the same
instances at their full time axis -- the 48-instance batch through the
batched executor with graph-captured chunks, as the benchmark runs it -- and
is compared with relative L2 error <= 1e-5 on the stored sensor subsample
(forward) and voxel set (adjoint of the stored seeded data).
"""
import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1603_02329_amd as pat  # noqa: E402

DEV = "cuda"
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-5


def _load(case):
    path = os.path.join(GOLD, f"{case}.npz")
    if not os.path.exists(path):
        pytest.skip(f"reference {case}.npz not generated")
    return np.load(path, allow_pickle=False)


def _h(g, inst):
    return np.random.default_rng(int(g["h_seed"])).standard_normal((inst.desc.nt, inst.ns)).astype(np.float32)


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _check(case, inst, data, img, g):
    ed = _rel(data[:, g["sensor_idx"]], g["data"])
    ei = _rel(img.ravel()[g["img_idx"]], g["img"])
    print(f"{case}: forward rel-L2 {ed:.3e}  adjoint rel-L2 {ei:.3e}", flush=True)
    assert ed <= TOL, (case, ed)
    assert ei <= TOL, (case, ei)


SINGLE = {
    "cfg2": lambda: synth.config2(),
    "cfg3f": lambda: synth.config3()[0],
    "cfg3c": lambda: synth.config3()[1],
    "cfg5": lambda: synth.config5(),
}


@pytest.mark.parametrize("case", list(SINGLE))
def test_fullsize_single(case):
    g = _load(case)
    inst = SINGLE[case]()
    assert int(g["nt"]) == inst.desc.nt
    plan = pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV)
    data = plan.forward(torch.from_numpy(inst.p0).to(DEV)).cpu().numpy()
    img = plan.adjoint(torch.from_numpy(_h(g, inst)).to(DEV)).cpu().numpy()
    _check(case, inst, data, img, g)


def test_fullsize_batch48():
    """All 48 uneven instances through one batch in the benchmark's launch
    configuration (default grouping and fusion, graph chunks of 64 steps,
    column variants autotuned on the batch's own buffers); the six with
    stored references are checked."""
    ids = [0, 1, 16, 17, 32, 33]
    gold = {i: _load(f"cfg4_{i}") for i in ids}
    insts = synth.config4()
    plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=DEV) for i in insts]
    batch = pat.Batch(plans)
    p0 = [torch.from_numpy(i.p0).to(DEV) for i in insts]
    batch.forward(p0)
    batch.autotune(reps=3)
    datas = batch.forward(p0)
    hs = []
    for k, inst in enumerate(insts):
        h = _h(gold[k], inst) if k in gold else np.zeros((inst.desc.nt, inst.ns), np.float32)
        hs.append(torch.from_numpy(h).to(DEV))
    imgs = batch.adjoint(hs)
    torch.cuda.synchronize()
    for k in ids:
        _check(f"cfg4_{k}", insts[k], datas[k].cpu().numpy(), imgs[k].cpu().numpy(), gold[k])
    batch.close()


def test_batch48_short_all_instances():
    """All 48 instances with the time axis cut to a third (200 / 400 / 800
    samples: the wave crosses each instance's sensor arc within that time),
    through the batched executor (default grouping, graph chunks of 64
    steps, autotuned column variants), each forward record set and each
    adjoint image checked against the oracle relative to its own norm."""
    from dataclasses import replace
    g = _load("cfg4_short")
    insts = [synth.Instance(replace(i.desc, nt=i.desc.nt // 3), i.c0, i.rho0, i.alpha0_db, i.sensors, i.p0, i.name)
             for i in synth.config4()]
    plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=DEV) for i in insts]
    batch = pat.Batch(plans)
    p0 = [torch.from_numpy(i.p0).to(DEV) for i in insts]
    batch.forward(p0)
    batch.autotune(reps=2)
    datas = batch.forward(p0)
    hs = [torch.from_numpy(np.random.default_rng(int(g[f"h_seed_{k}"])).standard_normal(
        (inst.desc.nt, inst.ns)).astype(np.float32)).to(DEV) for k, inst in enumerate(insts)]
    imgs = batch.adjoint(hs)
    torch.cuda.synchronize()
    worst = (0.0, -1, "")
    for k, inst in enumerate(insts):
        assert int(g[f"nt_{k}"]) == inst.desc.nt
        ed = _rel(datas[k].cpu().numpy()[:, g[f"sensor_idx_{k}"]], g[f"data_{k}"])
        ei = _rel(imgs[k].cpu().numpy().ravel()[g[f"img_idx_{k}"]], g[f"img_{k}"])
        for e, what in ((ed, "forward"), (ei, "adjoint")):
            if e > worst[0]:
                worst = (e, k, what)
        assert ed <= TOL and ei <= TOL, (k, ed, ei)
    print(f"cfg4_short: worst rel-L2 over 48 instances {worst[0]:.3e} (instance {worst[1]}, {worst[2]})",
          flush=True)
    batch.close()


def test_cfg5_autograd_with_checkpoints():
    """The 128^3 workload through torch.autograd with the forward run in
    checkpointed segments of 50 steps: the segmented forward equals the
    one-piece pat_forward bitwise and matches the oracle on the stored
    sensors; the backward of <H p0, h> (h the stored seeded data) is H^T h
    and matches the oracle adjoint on the stored voxels."""
    from paper_1603_02329_amd.autograd import PatOperator, replay_segment
    g = _load("cfg5")
    inst = synth.config5()
    plan = pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV)
    x = torch.from_numpy(inst.p0).to(DEV).requires_grad_(True)
    h = torch.from_numpy(_h(g, inst)).to(DEV)
    plain = plan.forward(x.detach()).clone()
    with torch.enable_grad():
        d = PatOperator.apply(x, plan, 50)
        loss = (d.double() * h.double()).sum()
    assert torch.equal(d, plain)
    loss.backward()
    torch.cuda.synchronize()
    _check("cfg5 autograd/ckpt50", inst, d.detach().cpu().numpy(), x.grad.cpu().numpy(), g)
    assert torch.equal(x.grad, plan.adjoint(h))
    # a segment replayed from the snapshot at 750 is bitwise the recorded one
    ckpts = d.grad_fn.checkpoints  # the snapshots the Function kept on its context
    assert [n for n, _ in ckpts] == list(range(50, 800, 50))
    seg = replay_segment(plan, ckpts, x.detach(), 760, 800)
    assert torch.equal(seg, plain[760:800])
