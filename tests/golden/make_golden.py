"""Write the full-size oracle results the GPU parity tests compare against.

Every value stored here is computed by the FP64 oracle (``oracle/``) from the
seeded synthetic inputs (``synth/``) and rounded to float32 once; nothing
comes from the GPU library.  For each case the file holds:

  data       oracle forward H p0 on the sensors listed in ``sensor_idx``
             (a fixed subsample of the sensors, all time samples), (nt, k)
  sensor_idx the sensor indices kept
  h_seed     seed of the standard-normal float32 data h fed to the adjoint
  img        oracle adjoint H^T h on the voxels listed in ``img_idx``
             (flat indices; all voxels for 2D cases, a subsample in 3D)
  img_idx    flat voxel indices kept

Usage:  python tests/golden/make_golden.py [case ...]   (default: all)
Cases: cfg2, cfg3f, cfg3c, cfg4_<i> (i = 0, 1, 16, 17, 32, 33), cfg5, and
cfg4_short: all 48 instances of the batch workload with the time axis cut to
a third (200 / 400 / 800 samples: long enough for the wave to cross each
instance's sensor arc, so that every record carries its phantom's signal),
one file with arrays per instance (``data_<i>``, ``img_<i>``; sensors every
8th, voxels on a stride-8 lattice).
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import kspace as K  # noqa: E402

CFG4_IDS = (0, 1, 16, 17, 32, 33)


def instance(case: str):
    if case == "cfg2":
        return synth.config2()
    if case == "cfg3f":
        return synth.config3()[0]
    if case == "cfg3c":
        return synth.config3()[1]
    if case.startswith("cfg4_"):
        return synth.config4()[int(case.split("_")[1])]
    if case == "cfg5":
        return synth.config5()
    raise KeyError(case)


def subsample(case: str, inst):
    ns = inst.ns
    if case == "cfg5":
        sens = np.arange(0, ns, 16)
        n = int(np.prod(inst.desc.shape))
        grid = np.arange(n).reshape(inst.desc.shape)[::4, ::4, ::4]
        return sens, grid.ravel()
    return np.arange(0, ns, 4), np.arange(int(np.prod(inst.desc.shape)))


def h_for(case: str, inst):
    seed = 97 + sum(ord(ch) for ch in case)
    h = np.random.default_rng(seed).standard_normal((inst.desc.nt, inst.ns)).astype(np.float32)
    return seed, h


def make(case: str, workers: int) -> None:
    K.WORKERS = workers
    inst = instance(case)
    t0 = time.time()
    op = K.make_plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors)
    data = K.forward(op, inst.p0)
    seed, h = h_for(case, inst)
    img = K.adjoint(op, h)
    sidx, iidx = subsample(case, inst)
    out = os.path.join(HERE, f"{case}.npz")
    np.savez_compressed(out, data=data[:, sidx].astype(np.float32), sensor_idx=sidx.astype(np.int32),
                        h_seed=np.int64(seed), img=img.ravel()[iidx].astype(np.float32),
                        img_idx=iidx.astype(np.int64), nt=np.int64(inst.desc.nt))
    print(f"{case}: {time.time() - t0:.1f} s -> {out} ({os.path.getsize(out) / 1e6:.2f} MB)", flush=True)


SHORT_DIV = 3  # time axes of the cfg4_short case: N_t / SHORT_DIV


def short_instances():
    """The 48 batch instances with N_t cut to a third."""
    from dataclasses import replace
    return [synth.Instance(replace(i.desc, nt=i.desc.nt // SHORT_DIV), i.c0, i.rho0, i.alpha0_db, i.sensors, i.p0,
                           i.name) for i in synth.config4()]


_SHORT = None


def _short_one(args):
    global _SHORT
    k, workers = args
    K.WORKERS = workers
    if _SHORT is None:  # once per worker process
        _SHORT = short_instances()
    inst = _SHORT[k]
    op = K.make_plan(inst.desc, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors)
    data = K.forward(op, inst.p0)
    seed, h = h_for(f"cfg4_short_{k}", inst)
    img = K.adjoint(op, h)
    sidx = np.arange(0, inst.ns, 8)
    iidx = np.arange(int(np.prod(inst.desc.shape))).reshape(inst.desc.shape)[::8, ::8].ravel()
    return k, {f"data_{k}": data[:, sidx].astype(np.float32), f"sensor_idx_{k}": sidx.astype(np.int32),
               f"h_seed_{k}": np.int64(seed), f"img_{k}": img.ravel()[iidx].astype(np.float32),
               f"img_idx_{k}": iidx.astype(np.int64), f"nt_{k}": np.int64(inst.desc.nt)}


def make_short(workers: int) -> None:
    """The 48 instances in a pool of processes (ORACLE_PROCS, default 1),
    each running the oracle with `workers` FFT threads."""
    from concurrent.futures import ProcessPoolExecutor
    procs = int(os.environ.get("ORACLE_PROCS", "1"))
    t0 = time.time()
    out = {}
    sizes = [int(np.prod(i.desc.shape)) for i in short_instances()]
    order = sorted(range(len(sizes)), key=lambda k: -sizes[k])  # largest first
    with ProcessPoolExecutor(procs) as ex:
        for k, arrs in ex.map(_short_one, [(k, workers) for k in order]):
            out.update(arrs)
            print(f"cfg4_short {k}: {time.time() - t0:.1f} s", flush=True)
    path = os.path.join(HERE, "cfg4_short.npz")
    np.savez_compressed(path, **out)
    print(f"cfg4_short -> {path} ({os.path.getsize(path) / 1e6:.2f} MB)", flush=True)


def main():
    cases = sys.argv[1:] or (["cfg2", "cfg3c", "cfg3f"] + [f"cfg4_{i}" for i in CFG4_IDS] + ["cfg5", "cfg4_short"])
    workers = int(os.environ.get("ORACLE_WORKERS", os.cpu_count() or 1))
    for c in cases:
        if c == "cfg4_short":
            make_short(workers)
        else:
            make(c, workers)


if __name__ == "__main__":
    main()
