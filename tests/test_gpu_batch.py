"""GPU: the batched executor (work tables + graph-captured chunks) and the
segmented forward reproduce the eager single-instance path bitwise."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1603_02329_amd as pat  # noqa: E402

DEV = "cuda"


def _instances():
    specs = [
        dict(n=(32, 32), nt=23, ns=6, pml=4, lossy=True),
        dict(n=(32, 32), nt=23, ns=4, pml=3, lossy=True),
        dict(n=(64, 64), nt=41, ns=9, pml=6, lossy=True),
        dict(n=(16, 16), nt=9, ns=3, pml=2, lossy=False),
        dict(n=(64, 32), nt=17, ns=5, pml=4, lossy=True),
        dict(n=(32, 32), nt=1, ns=3, pml=3, lossy=True),
    ]
    return [synth.small_instance(500 + i, **s) for i, s in enumerate(specs)]


@pytest.mark.parametrize("chunk", [1, 4])
def test_batch_matches_eager_bitwise(chunk):
    insts = _instances()
    plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=DEV) for i in insts]
    p0 = [torch.from_numpy(i.p0).to(DEV) for i in insts]
    ref_d = [p.forward(x).clone() for p, x in zip(plans, p0)]
    rng = np.random.default_rng(3)
    hs = [torch.from_numpy(rng.standard_normal((i.desc.nt, i.ns)).astype(np.float32)).to(DEV) for i in insts]
    ref_i = [p.adjoint(h).clone() for p, h in zip(plans, hs)]
    b = pat.Batch(plans, chunk=chunk)
    for rep in range(2):  # graph replays across calls
        d = b.forward(p0)
        im = b.adjoint(hs)
        torch.cuda.synchronize()
        for k in range(len(insts)):
            assert torch.equal(d[k], ref_d[k]), (rep, k)
            assert torch.equal(im[k], ref_i[k]), (rep, k)
    b.close()


def test_forward_range_resume_is_bitwise():
    inst = synth.small_instance(600, (64, 64), nt=37, ns=7, pml=5, lossy=True)
    plan = pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV)
    p0 = torch.from_numpy(inst.p0).to(DEV)
    full = plan.forward(p0).clone()
    state = torch.empty(plan.state_bytes, dtype=torch.uint8, device=DEV)
    seg = torch.full_like(full, float("nan"))
    for a, b in [(0, 10), (10, 11), (11, 30), (30, 37)]:
        plan.forward_range(p0 if a == 0 else None, seg, a, b, state)
    torch.cuda.synchronize()
    assert torch.equal(seg, full)


def test_check_finite_flag():
    inst = synth.small_instance(601, (32, 32), nt=8, ns=4, pml=3, lossy=True)
    plan = pat.Plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV,
                    check_finite=True)
    p0 = torch.from_numpy(inst.p0).to(DEV)
    plan.forward(p0)
    plan.sync()
    bad = p0.clone()
    bad[5, 7] = float("inf")
    plan.forward(bad)
    with pytest.raises(pat.PatError) as e:
        plan.sync()
    assert e.value.code == pat.PAT_ENONFINITE
    plan.forward(p0)
    plan.sync()  # flag cleared
