"""Reconstruction of a synthetic multi-level 2D or 3D problem on the GPU: ISTA,
FISTA and their multi-grid variants (Alg. ISTA, Alg. FISTA, Alg. FISTAMG),
with the objective F, the relative error RE and the residual norm RES
(section VI) and the elapsed time after every iteration.

    python -m paper_1603_02329_amd.reconstruct [--dim 2|3] [--n 512] [--iters 20]
        [--methods ista,mg-ista,fista,mg-fista] [--lam 1e-2] [--levels 2]
        [--eps-c 1e-2] [--smooth-p0] [--json out.json]

The problem: the seeded two-level medium and vessel phantom of the
synthetic workloads (512^2 / 256^2 by default, N_t 2400 / 1200), data = the
GPU forward of the phantom plus white Gaussian noise at 40 dB SNR (the
noise standard deviation is the data's rms times 10^(-40/20)); the data of
coarse level l (grid n/2^l, N_t / 2^l) are the fine data at every 2^l-th
sample.  Step sizes from the power
method on each level: 2/L_f for ISTA (as in section VI-A), 1/L_f for FISTA;
the two-level parameters are the paper's 2D values (kappa 1/4, vartheta
0.1, q_d 3, q_c 8, eps_c 1e-2, rho 1e-2).  The data are generated on the
reconstruction grid itself, so this shows convergence against time, not
the paper's inverse-crime-free errors.  --dim 3: the 3D workload's medium
and ellipsoid phantom (128^3 / 64^3 by default, N_t 800 / 400, planar
sensor at the PML), with the paper's 3D parameters (kappa 1/8, rho 3e-2;
section VI-B).  With --smooth-p0 every level's
operators filter the initial pressure (H = H0 S, H^T = S H0^T).
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--dim", type=int, default=2, choices=(2, 3), help="2D (default) or 3D problem")
    ap.add_argument("--n", type=int, default=0,
                    help="fine grid size (power of two; default 512 in 2D, 128 in 3D)")
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--methods", default="ista,mg-ista,fista,mg-fista")
    ap.add_argument("--lam", type=float, default=1e-2)
    ap.add_argument("--kappa", type=float, default=0.0, help="decision threshold (default 1/4 in 2D, 1/8 in 3D)")
    ap.add_argument("--rho", type=float, default=0.0, help="TV smoothing (default 1e-2 in 2D, 3e-2 in 3D)")
    ap.add_argument("--power-iters", type=int, default=20)
    ap.add_argument("--levels", type=int, default=2, help="grid levels of the MG variants (2: the paper's)")
    ap.add_argument("--eps-c", type=float, default=1e-2, help="coarse-solve termination (relative decrease)")
    ap.add_argument("--no-batch-levels", action="store_true",
                    help="run the fine and coarse gradients one after the other instead of in one batch")
    ap.add_argument("--smooth-p0", action="store_true",
                    help="filter the initial pressure inside H and H^T on every level (section VI-A)")
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)

    import torch

    import synth
    from . import Plan
    from . import solver as S

    dev = torch.device("cuda:0")
    nd = args.dim
    n = args.n or (512 if nd == 2 else 128)
    kappa = args.kappa or (0.25 if nd == 2 else 0.125)
    rho = args.rho or (1e-2 if nd == 2 else 3e-2)
    if nd == 2:
        pml = max(4, 20 * n // 512)
        nt = max(64, 2400 * n // 512)
        # the first two levels are those of the two-level workload (same draws)
        insts = synth.multi_level(3, 0, n, 1e-4, pml, nt, 256, max(2, args.levels))
    else:
        # the 128^3 workload's grid, PML and time axis; planar sensor at the PML
        pml = max(2, 16 * n // 128)
        nt = max(32, 800 * n // 128)
        insts = synth.multi_level_3d(5, 0, n, 2e-4, pml, nt, max(2, args.levels))
    if args.smooth_p0:
        from dataclasses import replace
        insts = [synth.Instance(replace(i.desc, smooth_p0=True), i.c0, i.rho0, i.alpha0_db, i.sensors, i.p0, i.name)
                 for i in insts]
    plans = [Plan(i.desc, i.c0, i.rho0, i.alpha0_db, i.sensors, device=dev) for i in insts]
    pf = plans[0]
    fine_i = insts[0]
    p_exact = torch.from_numpy(fine_i.p0).to(dev)
    clean = pf.forward(p_exact)
    rms = math.sqrt(float((clean.double() ** 2).mean()))
    noise = np.random.default_rng(4242).standard_normal(tuple(clean.shape)) * rms * 10.0 ** (-40.0 / 20.0)
    data = (clean + torch.from_numpy(noise.astype(np.float32)).to(dev)).contiguous()
    datas = [data] + [data[::2 ** l][:insts[l].desc.nt].contiguous() for l in range(1, len(insts))]
    v = torch.from_numpy(np.random.default_rng(7).standard_normal(fine_i.p0.shape).astype(np.float32)).to(dev)
    t0 = time.perf_counter()
    from . import restrict
    Ls = []
    for l, p in enumerate(plans):
        Ls.append(S.power_iteration(p, v, args.power_iters))
        v = restrict(v)
    print("grids " + " / ".join(f"{i.desc.n[0]}^{nd}" for i in insts) + ", N_t " +
          " / ".join(str(i.desc.nt) for i in insts) + "; L_f " + ", ".join(f"{x:.4e}" for x in Ls) +
          f" ({time.perf_counter() - t0:.1f} s)", flush=True)
    norm_exact = math.sqrt(float((p_exact.double() ** 2).sum()))

    def re(x):
        return 100.0 * math.sqrt(float(((x.double() - p_exact.double()) ** 2).sum())) / norm_exact

    results = {}
    for method in [m.strip() for m in args.methods.split(",") if m.strip()]:
        momentum = "fista" in method
        scale = 1.0 if momentum else 2.0
        levels = [S.Level(p, d, args.lam, scale / L) for p, d, L in zip(plans, datas, Ls)]
        fine = levels[0]
        x0 = torch.zeros_like(p_exact)
        rows = []
        torch.cuda.synchronize()
        start = time.perf_counter()

        def log(k, x, rec):
            torch.cuda.synchronize()
            F = rec if isinstance(rec, float) else rec.F
            kind = "direct" if isinstance(rec, float) else rec.kind
            row = {"k": k, "kind": kind, "F": F, "RE": re(x), "RES": fine.res, "seconds": time.perf_counter() - start}
            if not isinstance(rec, float) and rec.depth > 1:
                kind = f"{kind}{rec.depth}"
                row["depth"] = rec.depth
            rows.append(row)
            print(f"{method:9s} k={k:3d} {kind:9s} F={F:.6e} RE={row['RE']:7.3f}% RES={row['RES']:.4e} "
                  f"t={row['seconds']:7.2f}s", flush=True)

        if method.startswith("mg-"):
            S.mg_fista(fine, levels[1:args.levels], x0, args.iters,
                       S.MGParams(momentum=momentum, eps_c=args.eps_c, kappa=kappa, rho=rho,
                                  batch_levels=not args.no_batch_levels), callback=log)
        else:
            S.fista(fine, x0, args.iters, momentum=momentum, callback=log)
        results[method] = rows
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"dim": nd, "n": n, "nt": nt, "lam": args.lam, "kappa": kappa, "rho": rho, "levels": args.levels,
                       "L_f": Ls, "results": results}, f, indent=1)


if __name__ == "__main__":
    main()
