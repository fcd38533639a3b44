"""GPU: the batched executor (work tables + graph-captured chunks) and the
segmented forward reproduce the eager single-instance path bitwise."""
from dataclasses import replace

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


@pytest.mark.parametrize("chunk,parts,lanes", [(1, 0, 0), (4, 0, 0), (4, 1, 1), (3, 3, 2)])
def test_batch_matches_eager_bitwise(chunk, parts, lanes):
    insts = _instances()
    plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=DEV) for i in insts]
    p0 = [torch.from_numpy(i.p0).to(DEV) for i in insts]
    ref_d = [p.forward(x).clone() for p, x in zip(plans, p0)]
    rng = np.random.default_rng(3)
    hs = [torch.from_numpy(rng.standard_normal((i.desc.nt, i.ns)).astype(np.float32)).to(DEV) for i in insts]
    ref_i = [p.adjoint(h).clone() for p, h in zip(plans, hs)]
    b = pat.Batch(plans, chunk=chunk, parts=parts, lanes=lanes)
    for rep in range(2):  # graph replays across calls
        d = b.forward(p0)
        im = b.adjoint(hs)
        torch.cuda.synchronize()
        for k in range(len(insts)):
            assert torch.equal(d[k], ref_d[k]), (rep, k)
            assert torch.equal(im[k], ref_i[k]), (rep, k)
    b.close()


def test_batches_sharing_lanes_match_eager_bitwise():
    """Batches alive at the same time share the device's lane streams: a
    one-lane, a two-lane and a three-lane batch (the pool grows to three),
    each over plans of its own, called on two caller streams so that their
    work interleaves on the shared lanes, each keep their results bitwise
    those of the eager path."""
    insts = _instances()
    sets = [[pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=DEV) for i in insts] for _ in range(3)]
    p0 = [torch.from_numpy(i.p0).to(DEV) for i in insts]
    ref_d = [p.forward(x).clone() for p, x in zip(sets[0], p0)]
    rng = np.random.default_rng(5)
    hs = [torch.from_numpy(rng.standard_normal((i.desc.nt, i.ns)).astype(np.float32)).to(DEV) for i in insts]
    ref_i = [p.adjoint(h).clone() for p, h in zip(sets[0], hs)]
    batches = [pat.Batch(sets[0], chunk=4, parts=1, lanes=1), pat.Batch(sets[1], chunk=4, parts=2, lanes=2),
               pat.Batch(sets[2], chunk=3, parts=3, lanes=3)]
    main, side = torch.cuda.current_stream(), torch.cuda.Stream()
    side.wait_stream(main)
    for rep in range(2):
        outs = []
        for j, b in enumerate(batches):
            with torch.cuda.stream(side if j % 2 else main):
                outs.append((b.forward(p0), b.adjoint(hs)))
        torch.cuda.synchronize()
        for j, (d, im) in enumerate(outs):
            for k in range(len(insts)):
                assert torch.equal(d[k], ref_d[k]), (rep, j, k)
                assert torch.equal(im[k], ref_i[k]), (rep, j, k)
    for b in batches:
        b.close()


def _fused_instances(lossy):
    """2D size classes with axes of 128, 256 and 512 points (fused into
    shared launches), different time axes, non-square grids, and a class of
    one instance (absent from some groups when split in three)."""
    specs = [
        dict(n=(128, 128), nt=7, ns=5, pml=6),
        dict(n=(128, 128), nt=7, ns=4, pml=5),
        dict(n=(256, 256), nt=13, ns=6, pml=8),
        dict(n=(256, 128), nt=10, ns=5, pml=6),
        dict(n=(512, 512), nt=25, ns=7, pml=10),
        dict(n=(128, 512), nt=4, ns=3, pml=5),
        dict(n=(512, 512), nt=25, ns=6, pml=10),
    ]
    return [synth.small_instance(800 + i, lossy=lossy, **s) for i, s in enumerate(specs)]


@pytest.mark.parametrize("lossy,chunk,parts,lanes,tune",
                         [(True, 1, 0, 0, False), (True, 4, 0, 0, True), (True, 4, 1, 1, False),
                          (True, 3, 3, 2, False), (False, 4, 0, 0, True)])
def test_fused_batch_matches_eager_bitwise(lossy, chunk, parts, lanes, tune):
    """Size classes fused into shared launches, each instance stepping at
    its own rate through the common loop, equal the eager path bitwise."""
    insts = _fused_instances(lossy)
    plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=DEV) for i in insts]
    p0 = [torch.from_numpy(i.p0).to(DEV) for i in insts]
    ref_d = [p.forward(x).clone() for p, x in zip(plans, p0)]
    rng = np.random.default_rng(8)
    hs = [torch.from_numpy(rng.standard_normal((i.desc.nt, i.ns)).astype(np.float32)).to(DEV) for i in insts]
    ref_i = [p.adjoint(h).clone() for p, h in zip(plans, hs)]
    b = pat.Batch(plans, chunk=chunk, parts=parts, lanes=lanes)
    if tune:
        b.forward(p0)  # captures graphs that the tuning must drop
        rep = b.autotune(reps=2)
        shapes = {(i.desc.n[0], i.desc.n[1]) for i in insts}
        assert rep and set().union(*(set(map(tuple, e["fused"])) for e in rep)) == shapes
        assert all(e["tile"] in (8, 4) for e in rep)
    for r in range(2):  # graph replays across calls
        d = b.forward(p0)
        im = b.adjoint(hs)
        torch.cuda.synchronize()
        for k in range(len(insts)):
            assert torch.equal(d[k], ref_d[k]), (r, k)
            assert torch.equal(im[k], ref_i[k]), (r, k)
    b.close()
    # the same batch unfused
    b = pat.Batch(plans, chunk=chunk, parts=parts, lanes=lanes, fuse=False)
    d = b.forward(p0)
    torch.cuda.synchronize()
    assert all(torch.equal(d[k], ref_d[k]) for k in range(len(insts)))
    b.close()


def test_fused_mixed_physics_bitwise():
    """Lossy and lossless classes in one batch: each physics fuses its own
    size classes (the pass sequences differ), a class of another size range
    (64^2) stays unfused beside them; all equal the eager path bitwise."""
    specs = [dict(n=(128, 128), nt=7, ns=5, pml=6, lossy=True), dict(n=(256, 256), nt=11, ns=6, pml=8, lossy=True),
             dict(n=(128, 128), nt=9, ns=4, pml=6, lossy=False), dict(n=(256, 128), nt=5, ns=5, pml=6, lossy=False),
             dict(n=(64, 64), nt=8, ns=4, pml=4, lossy=True)]
    insts = [synth.small_instance(880 + i, **s) for i, s in enumerate(specs)]
    plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=DEV) for i in insts]
    p0 = [torch.from_numpy(i.p0).to(DEV) for i in insts]
    ref_d = [p.forward(x).clone() for p, x in zip(plans, p0)]
    rng = np.random.default_rng(9)
    hs = [torch.from_numpy(rng.standard_normal((i.desc.nt, i.ns)).astype(np.float32)).to(DEV) for i in insts]
    ref_i = [p.adjoint(h).clone() for p, h in zip(plans, hs)]
    b = pat.Batch(plans, chunk=4)
    rep = b.autotune(reps=2)
    fused = [tuple(map(tuple, e["fused"])) for e in rep if "fused" in e]
    assert {(128, 128), (256, 256)} <= set(s for f in fused for s in f)
    for r in range(2):
        d = b.forward(p0)
        im = b.adjoint(hs)
        torch.cuda.synchronize()
        for k in range(len(insts)):
            assert torch.equal(d[k], ref_d[k]), (r, k)
            assert torch.equal(im[k], ref_i[k]), (r, k)
    b.close()


@pytest.mark.parametrize("fuse", [True, False])
def test_smoothed_p0_batch_bitwise(fuse):
    """Plans that filter p0, or start the density from the t = 0 equation of
    state, beside plans that do neither: the batch groups them apart (their
    first and last passes differ), fuses the 2D classes that agree, and
    equals the eager path bitwise; nt = 1 runs the filter after the sensor
    transpose (and has no density).  A 3D batch likewise."""
    specs2 = [dict(n=(128, 128), nt=7, ns=5, pml=6, lossy=True, sm=True),
              dict(n=(256, 256), nt=11, ns=6, pml=8, lossy=True, sm=True),
              dict(n=(128, 128), nt=9, ns=4, pml=6, lossy=True, sm=False),
              dict(n=(256, 128), nt=5, ns=5, pml=6, lossy=False, sm=True),
              dict(n=(64, 64), nt=8, ns=4, pml=4, lossy=True, sm=True),
              dict(n=(64, 64), nt=1, ns=4, pml=4, lossy=True, sm=True),
              dict(n=(128, 128), nt=7, ns=5, pml=6, lossy=True, sm=False, eos=True),
              dict(n=(256, 256), nt=5, ns=3, pml=8, lossy=True, sm=False, eos=True),
              dict(n=(128, 256), nt=6, ns=4, pml=6, lossy=True, sm=True, eos=True),
              dict(n=(64, 64), nt=1, ns=4, pml=4, lossy=True, sm=False, eos=True)]
    specs3 = [dict(n=(16, 32, 16), nt=6, ns=5, pml=3, lossy=True, sm=True),
              dict(n=(16, 32, 16), nt=6, ns=4, pml=3, lossy=True, sm=False),
              dict(n=(32, 16, 16), nt=5, ns=4, pml=2, lossy=False, sm=True),
              dict(n=(16, 32, 16), nt=6, ns=4, pml=3, lossy=True, sm=False, eos=True)]
    for specs, seed in ((specs2, 900), (specs3, 920)):
        insts, plans = [], []
        for i, sp in enumerate(specs):
            sp = dict(sp)
            sm = sp.pop("sm")
            eos = sp.pop("eos", False)
            inst = synth.small_instance(seed + i, **sp)
            desc = replace(inst.desc, smooth_p0=sm, section3_density=eos)
            insts.append(inst)
            plans.append(pat.Plan(desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=DEV))
        p0 = [torch.from_numpy(i.p0).to(DEV) for i in insts]
        ref_d = [p.forward(x).clone() for p, x in zip(plans, p0)]
        rng = np.random.default_rng(seed)
        hs = [torch.from_numpy(rng.standard_normal((i.desc.nt, i.ns)).astype(np.float32)).to(DEV) for i in insts]
        ref_i = [p.adjoint(h).clone() for p, h in zip(plans, hs)]
        b = pat.Batch(plans, chunk=4, fuse=fuse)
        print("batch", len(specs[0]["n"]), "D fuse", fuse, flush=True)
        for r in range(2):
            d = b.forward(p0)
            im = b.adjoint(hs)
            torch.cuda.synchronize()
            for k in range(len(insts)):
                assert torch.equal(d[k], ref_d[k]), (r, k)
                assert torch.equal(im[k], ref_i[k]), (r, k)
        b.close()


def test_one_call_batched_entry_points():
    """pat_forward_batched / pat_adjoint_batched: per instance bitwise the
    eager results, on the first call (batch built) and the second (kept);
    after one of its plans is destroyed, a new list with a new plan works."""
    specs = [dict(n=(128, 128), nt=7, ns=5, pml=6, lossy=True), dict(n=(256, 256), nt=9, ns=4, pml=8, lossy=True),
             dict(n=(64, 32), nt=6, ns=3, pml=4, lossy=False)]
    insts = [synth.small_instance(940 + i, **sp) for i, sp in enumerate(specs)]
    plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=DEV) for i in insts]
    p0 = [torch.from_numpy(i.p0).to(DEV) for i in insts]
    rng = np.random.default_rng(7)
    hs = [torch.from_numpy(rng.standard_normal((i.desc.nt, i.ns)).astype(np.float32)).to(DEV) for i in insts]
    ref_d = [p.forward(x).clone() for p, x in zip(plans, p0)]
    ref_i = [p.adjoint(h).clone() for p, h in zip(plans, hs)]
    for r in range(2):
        d = pat.forward_batched(plans, p0)
        im = pat.adjoint_batched(plans, hs)
        torch.cuda.synchronize()
        for k in range(len(plans)):
            assert torch.equal(d[k], ref_d[k]), (r, k)
            assert torch.equal(im[k], ref_i[k]), (r, k)
    plans[2].close()  # frees the kept batch of this list
    fresh = pat.Plan(insts[2].desc, insts[2].c0, insts[2].rho0, insts[2].alpha0_db, insts[2].sensors, device=DEV)
    d = pat.forward_batched([plans[0], fresh], [p0[0], p0[2]])
    torch.cuda.synchronize()
    assert torch.equal(d[0], ref_d[0]) and torch.equal(d[1], ref_d[2])


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


def _tunable_instances(ndim):
    """Sizes whose column passes have several compiled tile widths: 2D
    columns of 128 and 256 points; a 3D grid whose z axis (128) differs from
    its y axis (32), so y- and z-axis passes need separate tables.  (A batch
    holds one dimensionality.)"""
    if ndim == 2:
        specs = [
            dict(n=(128, 128), nt=13, ns=6, pml=6, lossy=True),
            dict(n=(128, 128), nt=13, ns=5, pml=5, lossy=True),
            dict(n=(64, 256), nt=11, ns=4, pml=4, lossy=False),
        ]
    else:
        specs = [
            dict(n=(32, 32, 128), nt=7, ns=5, pml=3, lossy=True),
            dict(n=(32, 32, 128), nt=5, ns=4, pml=3, lossy=False),
        ]
    return [synth.small_instance(700 + 10 * ndim + i, **s) for i, s in enumerate(specs)]


def _run_tune_case(insts, tune):
    plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=DEV) for i in insts]
    p0 = [torch.from_numpy(i.p0).to(DEV) for i in insts]
    ref_d = [p.forward(x).clone() for p, x in zip(plans, p0)]
    rng = np.random.default_rng(5)
    hs = [torch.from_numpy(rng.standard_normal((i.desc.nt, i.ns)).astype(np.float32)).to(DEV) for i in insts]
    ref_i = [p.adjoint(h).clone() for p, h in zip(plans, hs)]
    b = pat.Batch(plans, chunk=4)
    b.forward(p0)  # captures graphs that the tuning must drop
    rep = tune(b)
    for _ in range(2):
        d = b.forward(p0)
        im = b.adjoint(hs)
        torch.cuda.synchronize()
        for k in range(len(insts)):
            assert torch.equal(d[k], ref_d[k]), k
            assert torch.equal(im[k], ref_i[k]), k
    return b, rep


@pytest.mark.parametrize("ndim", [2, 3])
def test_autotune_keeps_results_bitwise(ndim):
    insts = _tunable_instances(ndim)
    b, rep = _run_tune_case(insts, lambda b: b.autotune(reps=3))
    assert rep == b.tuning_report()
    assert rep, "no pass was tuned"
    for e in rep:
        cands = [(c["tile"], c["fpb"]) for c in e["candidates"]]
        assert len(cands) >= 2 and (e["tile"], e["fpb"]) in cands
        assert all(c["us"] > 0 for c in e["candidates"])
        assert e["axis_len"] in (128, 256, 512)
    if ndim == 3:
        assert all(e["n"] == [32, 32, 128] and e["mode"] <= 2 for e in rep)
    # several groups: one width policy, timed in context; the first policy
    # (width 8, one field per workgroup) kept unless another beats it by
    # 0.5 %, and every pass's variant the best of its isolated timings under
    # the policy kept
    assert len({e["policy"] for e in rep}) == 1
    us = rep[0]["policy_us"]
    first = us["width=8,fpb=1"]
    if rep[0]["policy"] == "width=8,fpb=1":
        assert min(us.values()) >= 0.995 * first - 0.1
    else:
        assert us[rep[0]["policy"]] <= min(us.values()) + 0.1
        assert us[rep[0]["policy"]] <= 0.995 * first + 0.1
    rule = {"width=8,fpb=1": lambda v: v["tile"] == 8 and v["fpb"] == 1, "fastest": lambda v: True,
            "width<=8": lambda v: v["tile"] <= 8, "width<=4": lambda v: v["tile"] <= 4,
            "width=8": lambda v: v["tile"] == 8}[rep[0]["policy"]]
    for e in rep:
        allowed = [v for v in e["candidates"] if rule(v)] or e["candidates"]
        chosen = [v for v in allowed if (v["tile"], v["fpb"]) == (e["tile"], e["fpb"])]
        assert chosen and chosen[0]["us"] <= min(v["us"] for v in allowed) + 1e-3
    b.close()


@pytest.mark.parametrize("ndim,tile,fpb", [(2, 4, 1), (2, 8, 1), (2, 16, 2), (2, 4, 2), (3, 4, 1), (3, 8, 1)])
def test_forced_tile_widths_bitwise(ndim, tile, fpb):
    """Every compiled variant, forced on every pass that has it, equals eager."""
    insts = _tunable_instances(ndim)
    applied = []

    def force(b):
        rep = b.autotune(reps=1)
        for e in rep:
            if any(v["tile"] == tile and v["fpb"] == fpb for v in e["candidates"]):
                b.set_tile(e, tile, fpb)
                applied.append(e["pass"])
        return rep
    b, _ = _run_tune_case(insts, force)
    assert applied
    if ndim == 3:
        b.close()
        return
    e = dict(n=[128, 128, 1], nt=13, lossy=1, dir=0, tile=4)
    with pytest.raises(pat.PatError):
        b.set_tile(dict(e, **{"pass": 1}))            # pass 1 of the forward is a row pass
    with pytest.raises(pat.PatError):
        b.set_tile(dict(e, **{"pass": 0}), 2)         # width 2 is not compiled
    with pytest.raises(pat.PatError):
        b.set_tile(dict(e, n=[96, 96, 1], **{"pass": 0}))  # no such class
    with pytest.raises(pat.PatError):
        b.set_tile(dict(e, nt=12, **{"pass": 0}))     # no class with that time axis
    with pytest.raises(pat.PatError):
        b.set_tile(dict(e, **{"pass": 0}), 8, 2)      # the gradient pass has one input field
    b.set_tile(dict(e, **{"pass": 0}), 0, 1)          # back to the default
    b.close()


def test_autotune_cache_roundtrip(tmp_path):
    insts = _tunable_instances(2)[:2]
    cache = str(tmp_path / "tiles.json")
    b, rep = _run_tune_case(insts, lambda b: b.autotune(reps=2, cache=cache))
    b.close()
    import json
    stored = json.load(open(cache))
    assert len(stored) == 1
    (arch, by_key), = stored.items()
    assert arch.startswith("gfx")
    b2, rep2 = _run_tune_case(insts, lambda b: b.autotune(reps=2, cache=cache))
    key = [(e["dir"], e["pass"], e["tile"], e["fpb"]) for e in rep]
    assert [(e["dir"], e["pass"], e["tile"], e["fpb"]) for e in rep2] == key
    assert b2.tuning_report() == []  # applied from the cache, nothing timed
    b2.close()
