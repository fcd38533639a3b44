"""Benchmark: forward+adjoint grid-point-steps per second on one MI355X.

A step is one gradient-and-prox iteration over a whole batch of synthetic
problems: the batched forward H x for every instance, the float32 residual
with its float64 half squared norm (the least-squares objective), the
batched adjoint H^T r (the gradient), then x <- prox(x - alpha grad) with 20
FGP iterations of the TV prox.  Throughput counts 2 * N * N_t grid-point
steps per instance (forward and adjoint), over the wall time of the step.

Default workload: 48 uneven 2D instances, 16 each of 128^2 (N_t 600),
256^2 (N_t 1200) and 512^2 (N_t 2400), heterogeneous lossy media.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "forward+adjoint grid-point-steps/s, batched vs plain FP32, at rel-L2 ≤1e-5"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    import synth
    if name == "cfg4":
        return synth.config4(), "48 x 2D lossy heterogeneous: 16x128^2/Nt600 + 16x256^2/Nt1200 + 16x512^2/Nt2400"
    if name == "cfg2":
        return [synth.config2()], "2D 256^2 lossy heterogeneous, Nt 1200, 256 sensors"
    if name == "cfg3":
        f, c = synth.config3()
        return [f, c], "2D two-level: 512^2/Nt2400 + 256^2/Nt1200 lossy heterogeneous"
    if name == "cfg5":
        return [synth.config5()], "3D 128^3 lossy heterogeneous, Nt 800, 128x128 plane of sensors"
    raise SystemExit(f"unknown workload {name}")


KERNEL_SOURCES = ("paper_1603_02329_amd/csrc/passes_fused.hip", "paper_1603_02329_amd/csrc/passes_row.h",
                  "paper_1603_02329_amd/csrc/passes_col.h", "paper_1603_02329_amd/csrc/passes_common.h",
                  "paper_1603_02329_amd/csrc/fft.h", "paper_1603_02329_amd/csrc/pat_internal.h")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def scaling_probe(insts, pat, torch, dev):
    """Fixed and marginal cost of the batched step.  (1) Forward + adjoint of
    the first k instances of every size class, k = 2, 4, 8, 16, each batch
    with the default grouping (two groups on two streams), autotuned, the
    best of three timed calls.  (2) The launch time of every pass against the
    number of 512^2 instances in the launch: a one-stream batch of one group
    over the first 1, 2, 4, 8, 16 of them, each pass launched back to back
    (10 untimed, then 50 timed with HIP events)."""
    by = {}
    for i in insts:
        by.setdefault(tuple(i.desc.n), []).append(i)
    print("instances per class, ms per forward + adjoint (best of 3), G grid-point-steps/s")
    for k in (2, 4, 8, 16):
        sel = [i for n in sorted(by) for i in by[n][:k]]
        plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=dev) for i in sel]
        p0 = [torch.from_numpy(i.p0).to(dev) for i in sel]
        gps = sum(2.0 * p.npoints * p.nt for p in plans)
        b = pat.Batch(plans)
        d = b.forward(p0)
        b.autotune(reps=10)
        d = b.forward(p0)
        b.adjoint(d)
        best = float("inf")
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            d = b.forward(p0)
            b.adjoint(d)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        print(f"{k:3d}  {best:8.1f}  {gps / best / 1e6:6.2f}", flush=True)
        b.close()
        del b, plans, p0, d
    big = by[max(by)]
    names = ["c-grad", "r-vel", "c-div", "r-dens", "c-abs", "r-state", "c-aabs", "r-adens", "c-adiv", "r-avel",
             "c-agrad"]
    keys = [(0, 0), (0, 1), (0, 2), (0, 3), (0, 4), (0, 5), (1, 1), (1, 2), (1, 3), (1, 4), (1, 5)]
    n = big[0].desc.n[0]
    print(f"\n{n}^2 instances per launch, us per launch (one stream, back-to-back launches)")
    print("  k " + " ".join(f"{x:>8s}" for x in names))
    for k in (1, 2, 4, 8, 16):
        sel = big[:k]
        plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=dev) for i in sel]
        p0 = [torch.from_numpy(i.p0).to(dev) for i in sel]
        b = pat.Batch(plans, chunk=1, parts=1, lanes=1)
        b.adjoint(b.forward(p0))
        b.autotune(reps=10)
        row = []
        for d_, i_ in keys:
            b.time_pass(d_, i_, n, 10)
            row.append(b.time_pass(d_, i_, n, 50)[0])
        print(f"{k:3d} " + " ".join(f"{u:8.2f}" for u in row), flush=True)
        b.close()
        del b, plans, p0


def fused_batch(plans) -> bool:
    """Whether the library's batch of these plans fuses its size classes
    into shared launches (2D, both axes 128/256/512, nt >= 2, more than one
    size class of the same physics)."""
    classes = {}
    for p in plans:
        n = p.desc.n
        if len(n) != 2 or any(v not in (128, 256, 512) for v in n) or p.desc.nt < 2:
            continue
        classes.setdefault(p.lossy, set()).add((tuple(n), p.desc.nt))
    return any(len(v) > 1 for v in classes.values())


def row_kernel_name(plans, kind: int) -> str:
    """Kernel symbol (as rocprofv3 prints it) of row-pass kind `kind` over
    the one-stream batch of these plans."""
    if fused_batch(plans):
        return f"k_rowf<2, {kind}>"
    nx = max(p.desc.n[0] for p in plans)
    return f"k_row<{nx}, {len(plans[0].desc.n)}, {kind}>"


def _summary_fields(name: str):
    """The `- key: value` lines of a committed rocprofv3 counter summary, or
    None when it is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].strip().split(": ", 1)
            fields[k] = v.strip("` ")
    return fields if fields.get("kernel_source_sha256") == kernel_source_hash() else None


def counter_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when that summary was taken on different kernel
    sources (or is missing)."""
    fields = _summary_fields("cfg4_counters_fetch_write.md")
    key = f"traffic_bytes_per_launch[{kernel}]"
    return float(fields[key]) if fields and key in fields else None


def step_traffic(workload: str):
    """Measured HBM bytes per grid-point-step of a whole forward + adjoint of
    the workload (committed counter summary: the 48-instance 2D batch or the
    128^3 instance), or None."""
    name = {"cfg4": "cfg4_step_counters_fetch_write.md", "cfg5": "cfg5_step_counters_fetch_write.md"}.get(workload)
    fields = _summary_fields(name) if name else None
    return float(fields["traffic_bytes_per_gps"]) if fields and "traffic_bytes_per_gps" in fields else None


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), or the platform string."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(insts, seconds_target=15.0):
    """The FP64 oracle on a bounded sample: one instance of each grid size,
    a shortened time axis, forward + adjoint."""
    from dataclasses import replace

    from oracle import kspace as K
    cores = min(os.cpu_count() or 1, 16)
    K.WORKERS = cores
    seen = {}
    for inst in insts:
        seen.setdefault(inst.desc.n, inst)
    sample = list(seen.values())
    nts = 300  # about 15 s of oracle work on the box's 16 host threads
    gps = 0.0
    t_total = 0.0
    for inst in sample:
        d = replace(inst.desc, nt=nts)
        op = K.make_plan(d, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors)
        t0 = time.perf_counter()
        data = K.forward(op, inst.p0)
        K.adjoint(op, data)
        t_total += time.perf_counter() - t0
        gps += 2.0 * inst.desc.npoints * nts
    sizes = "+".join(f"{i.desc.n[0]}^2" for i in sample)
    # the same oracle on one core, on the middle-sized instance of the sample
    K.WORKERS = 1
    small = sorted(sample, key=lambda i: i.desc.npoints)[len(sample) // 2]
    d = replace(small.desc, nt=nts)
    op = K.make_plan(d, small.c0, small.rho0, small.alpha0_db, small.sensors)
    t0 = time.perf_counter()
    K.adjoint(op, K.forward(op, small.p0))
    t1 = time.perf_counter() - t0
    K.WORKERS = cores
    return {"value": gps / t_total, "unit": "grid-point-steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "cpu_count": os.cpu_count(),
            "sample": f"FP64 oracle forward+adjoint of one instance per size ({sizes}) with N_t={nts} "
                      f"instead of the full time axis; {t_total:.1f} s on {cores} threads (scipy.fft workers)",
            "single_core": {"value": 2.0 * small.desc.npoints * nts / t1, "unit": "grid-point-steps/s",
                            "sample": f"{small.desc.n[0]}^2 instance, N_t={nts}, {t1:.1f} s on 1 thread"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg4")
    ap.add_argument("--chunk", type=int, default=64, help="graph chunk (steps per captured graph; 1 = eager)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=3, help="timed steps of the plain path (after 1 warm-up)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default column tile widths")
    ap.add_argument("--parts", type=int, default=0, help="groups per size class (0: the library default)")
    ap.add_argument("--lanes", type=int, default=0, help="streams for the groups (0: one per group)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="run only the isolated kernel-timing phase (for profiling it); no JSON line")
    ap.add_argument("--passes-only", action="store_true",
                    help="run the roofline phase and the isolated timing of every pass (for profiling "
                         "them); prints the per-pass table, no JSON line")
    ap.add_argument("--time-pass", default=None,
                    help="direction:pass_index timed with HIP events (default: the forward velocity row pass, "
                         "0:1 in 2D, 0:3 in 3D)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="counter probe: a 1 GiB device copy (calibration) and a burst of the roofline "
                         "phase's launches; run under rocprofv3 --pmc")
    ap.add_argument("--sync-probe", action="store_true",
                    help="diagnostic: cost of a grid-wide barrier in a cooperative launch against a kernel "
                         "boundary (stream and graph), for several grid sizes and amounts of work; no JSON line")
    ap.add_argument("--scaling-probe", action="store_true",
                    help="diagnostic (2D): forward + adjoint time of the first k instances of every size class "
                         "(k = 2, 4, 8, 16; two groups on two streams), and the launch time of every pass "
                         "against the number of 512^2 instances in the launch (1 to 16; one stream); no JSON "
                         "line")
    ap.add_argument("--pmc-step", action="store_true",
                    help="counter probe of a whole step: the calibration copy, then one forward and one "
                         "adjoint of the workload with the time axes cut to a tenth, every pass launched "
                         "eagerly; run under rocprofv3 --pmc")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the solver runs each instance on a single device, and "
              "independent instances would be split across GPUs without communication; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1603_02329_amd as pat
    dev = torch.device("cuda:0")
    if args.sync_probe:
        import ctypes
        L = pat.lib()
        torch.zeros(1, device=dev)
        print("blocks/CU  floats/block  cg grid sync (us/iter)  atomic barrier (us/iter)  stream launch (us)  "
              "graph launch (us)")
        for bpc in (1, 2, 4):
            for fpb in (0, 2048, 16384):
                g, at, st, gr = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
                rc = L.pat_diag_sync_costs(bpc, fpb, 1000, ctypes.byref(g), ctypes.byref(at), ctypes.byref(st),
                                           ctypes.byref(gr))
                if rc:
                    print(f"{bpc:9d}  {fpb:12d}  error {rc}")
                    continue
                print(f"{bpc:9d}  {fpb:12d}  {g.value:22.2f}  {at.value:24.2f}  {st.value:18.2f}  {gr.value:17.2f}",
                      flush=True)
        return
    insts, wl_name = workload(args.workload)
    if args.scaling_probe:
        scaling_probe(insts, pat, torch, dev)
        return
    if args.pmc_step:
        # the same instances with a tenth of their time axes: the size
        # classes keep their step ratios, so each step of a fused group
        # carries the same mix of instances as at full length
        import synth
        from dataclasses import replace
        insts = [synth.Instance(replace(i.desc, nt=max(2, i.desc.nt // 10)), i.c0, i.rho0, i.alpha0_db, i.sensors,
                                i.p0, i.name) for i in insts]
    if args.pmc_probe:
        # same instances and launch geometry, 9 time samples: the per-launch
        # traffic of a pass does not depend on the length of the time axis
        import synth
        from dataclasses import replace
        insts = [synth.Instance(replace(i.desc, nt=min(i.desc.nt, 9)), i.c0, i.rho0, i.alpha0_db, i.sensors,
                                i.p0, i.name) for i in insts]
    log(f"workload: {wl_name} ({len(insts)} instances)")
    ndim = insts[0].desc.ndim
    if args.time_pass is None:
        args.time_pass = "0:1" if ndim == 2 else "0:3"
    # algorithmic bytes per grid-point-step (float32): 2D lossy 152; 3D lossy
    # with homogeneous rho0 184 (the y-z spectral operators as two plane passes)
    b_alg = 152.0 if ndim == 2 else 184.0
    plans = [pat.Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=dev) for i in insts]
    x_true = [torch.from_numpy(i.p0).to(dev) for i in insts]
    if args.pmc_probe:
        # counter calibration: an elementwise kernel that reads and writes
        # exactly 1 GiB of data not resident in any cache (a second 1 GiB
        # fill in between evicts it from L2 and the Infinity Cache)
        a = torch.ones(256 * 1024 * 1024, device=dev)
        flush = torch.zeros(256 * 1024 * 1024, device=dev)
        b = torch.add(a, 1.0)
        del flush, b
        probe = pat.Batch(plans, chunk=1, parts=1, lanes=1)
        tdir, tidx = (int(v) for v in args.time_pass.split(":"))
        probe.time_pass(tdir, tidx, max(p.desc.n[0] for p in plans), 20)  # the roofline phase's launches
        torch.cuda.synchronize()
        log("pmc probe done")
        return
    if args.pmc_step:
        a = torch.ones(256 * 1024 * 1024, device=dev)
        flush = torch.zeros(256 * 1024 * 1024, device=dev)
        b = torch.add(a, 1.0)
        del flush, b, a
        bs = pat.Batch(plans, chunk=1)
        d = bs.forward(x_true)
        bs.adjoint(d)
        torch.cuda.synchronize()
        gps = sum(float(p.desc.npoints) * p.desc.nt for p in plans)
        log(f"pmc step done: {len(plans)} instances, {gps:.6e} grid-point-steps per direction")
        return
    tdir, tidx = (int(v) for v in args.time_pass.split(":"))
    nx_dom = max(p.desc.n[0] for p in plans)  # time the largest grids' launches only

    def isolated_kernel(reps=200):
        """The selected pass on its own: `reps` back-to-back launches over a
        one-stream batch with one group (size classes fused into one launch
        where the library fuses them, else the largest size's launch), every
        launch having the GPU to itself, timed with HIP events around the
        burst.  Returns (ms total, launches, algorithmic bytes total)."""
        b1 = pat.Batch(plans, chunk=1, parts=1, lanes=1)
        b1.time_pass(tdir, tidx, nx_dom, 100)  # untimed warm-up burst: clocks settle
        us, by = b1.time_pass(tdir, tidx, nx_dom, reps)
        b1.close()
        return us * reps / 1e3, reps, by * reps

    # the roofline phase runs first, so that `--roofline-only` (the profiled
    # command) repeats it exactly
    k_ms, k_n, k_bytes = isolated_kernel()
    log(f"isolated pass {tdir}:{tidx}: {k_n} launches, {k_ms / k_n * 1e3:.2f} us/launch, "
        f"{k_bytes / (k_ms / 1e3) / 1e9:.0f} GB/s")
    if args.roofline_only:
        return

    def every_pass(reps=50):
        """Every pass of a forward and an adjoint step timed on its own the
        same way, the column passes in the widths the autotuner picks for
        this one-stream batch (after the roofline phase, untimed for the
        benchmark): {(dir, pass): (us per launch, algorithmic bytes per
        launch)}."""
        out = {}
        b1 = pat.Batch(plans, chunk=1, parts=1, lanes=1)
        b1.autotune(reps=10)  # the column passes in their tuned launch shapes
        for d in (0, 1):
            for k in range(16):
                try:
                    b1.time_pass(d, k, nx_dom, 10)
                    out[(d, k)] = b1.time_pass(d, k, nx_dom, reps)
                except pat.PatError:
                    continue  # no such pass (or not timeable alone)
        b1.close()
        return out

    pass_times = every_pass() if ndim == 2 else {}
    if args.passes_only:
        for (d, k), (us, by) in sorted(pass_times.items()):
            log(f"pass {d}:{k}: {us:.2f} us/launch, {by / 1e6:.1f} MB, {by / (us * 1e-6) / 1e9:.0f} GB/s")
        return
    batch = pat.Batch(plans, chunk=args.chunk, parts=args.parts, lanes=args.lanes)
    targets = [d.clone() for d in batch.forward(x_true)]
    tiles = []
    if not args.no_autotune:
        # untimed: pick the column tile widths on the batch's own buffers
        # (the targets are already copied out)
        t0 = time.perf_counter()
        tiles = batch.autotune(reps=10)
        log(f"autotune: {len(tiles)} passes in {time.perf_counter() - t0:.1f} s: " +
            ", ".join(f"{e['n'][0]}:{e['dir']}:{e['pass']}->{e['tile']}" for e in tiles))
    xs = [0.5 * x for x in x_true]
    total_gps = sum(2.0 * p.npoints * p.nt for p in plans)
    tvw = [torch.empty(max(1, pat.lib().pat_tv_prox_work_bytes(x.dim(), pat._i32x3(list(reversed(x.shape))))),
                       dtype=torch.uint8, device=dev) for x in xs]
    alpha = 1e-3
    lam = 1e-3

    from paper_1603_02329_amd.autograd import PatBatchLeastSquares, PatLeastSquares

    def step(loss_fn):
        """One gradient-and-prox iteration: the least-squares loss through
        torch.autograd (forward in the Function, the adjoint as its
        backward), then x <- prox(x - alpha grad), the proxes of all
        instances in one batched call."""
        leaves = [x.detach().requires_grad_(True) for x in xs]
        loss = loss_fn(leaves)
        loss.backward()
        zs = [x.detach() - alpha * x.grad for x in leaves]
        xs[:] = pat.tv_prox_batched(zs, [alpha * lam] * len(zs), 20, works=tvw)
        return loss

    def batched(leaves):
        return PatBatchLeastSquares.apply(batch, targets, *leaves)

    def plain(leaves):
        return sum(PatLeastSquares.apply(x, t, p) for x, t, p in zip(leaves, targets, plans))

    def timed(fns, steps, warmup, label):
        """Mean ms per step over `steps` steps between two synchronisations
        (the value the benchmark reports), and the per-step times from HIP
        events between the steps (their median is reported beside it)."""
        for _ in range(warmup):
            step(fns)
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        evs[0].record()
        for i in range(steps):
            step(fns)
            evs[i + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
        ms = evs[0].elapsed_time(evs[steps]) / steps
        med = float(np.median(per))
        log(f"{label}: {ms:.1f} ms/step (median {med:.1f}, host wall {wall / steps * 1e3:.1f} ms/step), "
            f"{total_gps / (ms / 1e3) / 1e9:.2f} G gps/s")
        return ms, med, per


    # main timed region: the batched executor (graph-captured chunks; the
    # steps left over by the chunking run eagerly between the chunks and
    # are event-timed there, sharing the GPU with the other streams)
    pat.timing_begin(tdir, tidx, nx_dom)
    ms, ms_med, ms_all = timed(batched, args.steps, args.warmup, f"batched(chunk={args.chunk})")
    s_ms, s_n, s_bytes = pat.timing_end()
    plain_ms = plain_med = None
    if not args.no_plain:
        plain_ms, plain_med, _ = timed(plain, args.plain_steps, 1, "plain (one instance at a time, eager)")
    value = total_gps / (ms / 1e3)
    achieved = k_bytes / (k_ms / 1e3) / 1e9 if k_ms > 0 else 0.0
    # adjoint passes are named for the forward pass they transpose (the
    # divergence's transpose carries the a_j multipliers, the gradient's b_j)
    names = {(0, 0): "col gradient", (0, 1): "row velocity", (0, 2): "col divergence", (0, 3): "row density",
             (0, 4): "col absorption", (0, 5): "row state+gather", (1, 0): "row adj-state+scatter",
             (1, 1): "col adj-absorption", (1, 2): "row adj-density", (1, 3): "col adj-divergence",
             (1, 4): "row adj-velocity", (1, 5): "col adj-gradient"}
    if ndim == 3:
        names = {(0, 3): "row velocity", (0, 7): "row density", (0, 11): "row state+gather"}
    step_bytes = value * b_alg / 1e9  # algorithmic GB/s of the whole step
    st_bpg = step_traffic(args.workload)
    dom_name = names.get((tdir, tidx), f"{tdir}:{tidx}")
    dominant = {
        "kernel": dom_name,
        "kernel_symbol": row_kernel_name(plans, 1) if dom_name == "row velocity" else None,
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": counter_traffic(row_kernel_name(plans, 1)) if dom_name == "row velocity" else None,
        "launches": k_n,
        "avg_launch_us": (k_ms / k_n * 1e3) if k_n else None,
        "measured_in": "back-to-back launches of the pass over a one-stream batch before the timed region, "
                       "after an untimed burst of 100 (each launch: " +
                       ("every instance of the batch, its size classes fused" if fused_batch(plans)
                        else "every instance of the largest size") + "; GPU to itself)",
        "in_timed_region": {
            "launches": s_n,
            "avg_launch_us": (s_ms / s_n * 1e3) if s_n else None,
            "achieved": (s_bytes / (s_ms / 1e3) / 1e9) if s_ms > 0 else None,
            "note": "eager steps between graph chunks, concurrent with the other streams' passes",
        },
    }
    passes = {}
    for (d, k), (us, by) in sorted(pass_times.items()):
        gbs = by / us * 1e-3
        passes[names.get((d, k), f"{d}:{k}")] = {"avg_launch_us": us, "achieved": gbs,
                                                  "frac": gbs / HBM_PEAK_GBS, "bytes_per_launch": by}
    cols = {k: v for k, v in passes.items() if k.startswith("col")}
    worst_col = min(cols.items(), key=lambda kv: kv[1]["frac"]) if cols else None
    roofline = {
        # headline: the whole gradient step (forward + adjoint of every
        # instance, all passes, both streams) against the algorithmic bytes
        # per grid-point-step
        "bound": "hbm",
        "kernel": "whole step: batched forward + adjoint, every pass of every instance",
        "achieved": step_bytes,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": step_bytes / HBM_PEAK_GBS,
        "bytes_per_gps": b_alg,
        "traffic": (st_bpg * total_gps) if st_bpg else None,
        "traffic_bytes_per_gps": st_bpg,
        "target_frac": 0.60,
        "target_met": step_bytes / HBM_PEAK_GBS >= 0.60,
        "dominant_kernel": dominant,
        "worst_column_pass": ({"pass": worst_col[0], **worst_col[1]} if worst_col else None),
        "passes_isolated": passes,
    }
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": wl_name,
            "instances": len(plans),
            "gps_per_step": total_gps,
            "executor": f"batched, graph chunk {args.chunk}; least squares through torch.autograd "
                        "(backward = batched adjoint)",
            "col_tiles": {f"{e['n'][0]}x{e['n'][1]}x{e['n'][2]}:{e['dir']}:{e['pass']}": e["tile"] for e in tiles},
            "col_tile_policy": (tiles[0].get("policy") if tiles else None),
            "col_tile_policy_us": (tiles[0].get("policy_us") if tiles else None),
            "ms_per_step_median": ms_med,
            "ms_per_step_all": ms_all,
            "plain_ms_per_step": plain_ms,
            "plain_ms_per_step_median": plain_med,
            "plain_steps": (args.plain_steps if plain_ms else None),
            "batched_over_plain": (plain_ms / ms) if plain_ms else None,
        },
        "roofline": roofline,
    }
    if not args.no_cpu:
        log("timing the FP64 oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(insts)
    batch.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
