"""The paper's adjoint-then-discretize operator against the exact transpose
on the GPU (section III's adjoint system, discretized with the forward
scheme, against pat_adjoint): dot-test gaps, the difference of the two
gradients of the least-squares objective, and the time per call.

    python -m paper_1603_02329_amd.adjoint_ablation [--workload cfg2|cfg3f|cfg5] [--init default|eos|both]
                                                   [--json out.json]

For x the workload's phantom, d = H x its data and r = H(x/2) - d the
residual at x/2: gap(A) = |<H x, h> - <x, A h>| / |<H x, h>| for white
data h (seeded) and h = r; the gradients A r compared by relative L2
difference and cosine.  --init picks the forward's initial density:
p0 / c0^2 (default) or section III's equation of state at t = 0
(PAT_EOS_INIT), of which the paper's adjoint system is the transpose in
the continuum; "both" reports the two.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--init", default="both", choices=("default", "eos", "both"))
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)

    import torch
    from dataclasses import replace

    import synth
    from . import Plan

    if args.workload == "cfg2":
        inst = synth.config2()
    elif args.workload == "cfg3f":
        inst = synth.config3()[0]
    elif args.workload == "cfg5":
        inst = synth.config5()
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    dev = torch.device("cuda:0")

    def dot(a, b):
        return float((a.double() * b.double()).sum())

    out = {"workload": args.workload, "n": list(inst.desc.n), "nt": inst.desc.nt}
    inits = ("default", "eos") if args.init == "both" else (args.init,)
    for init in inits:
        desc = replace(inst.desc, section3_density=(init == "eos"))
        plan = Plan(desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors, device=dev)
        x = torch.from_numpy(inst.p0).to(dev)
        d = plan.forward(x).clone()
        r = (plan.forward(0.5 * x) - d).contiguous()
        h = torch.from_numpy(np.random.default_rng(11).standard_normal(tuple(d.shape)).astype(np.float32)).to(dev)
        res = {}
        for name, fn in (("exact", plan.adjoint), ("atd", plan.adjoint_atd)):
            fn(h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ah = fn(h).clone()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            ar = fn(r).clone()
            res[name] = {
                "ms_per_call": ms,
                "dot_gap_white": abs(dot(d, h) - dot(x, ah)) / abs(dot(d, h)),
                "dot_gap_residual": abs(dot(d, r) - dot(x, ar)) / abs(dot(d, r)),
            }
            res[name + "_grad"] = ar
        ge, ga = res.pop("exact_grad"), res.pop("atd_grad")
        res["grad_rel_diff"] = math.sqrt(dot(ga - ge, ga - ge) / dot(ge, ge))
        res["grad_cosine"] = dot(ga, ge) / math.sqrt(dot(ga, ga) * dot(ge, ge))
        out["init_" + init] = res
        plan.close()
    print(json.dumps(out), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
