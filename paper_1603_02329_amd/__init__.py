"""Python binding of libpat (gfx950): argument marshalling only.

Every operator runs in the HIP kernels of ``libpat.so``; this module only
checks tensors, allocates outputs with torch and forwards device pointers and
the current HIP stream to the C ABI declared in ``include/pat.h``.  It fails
loudly when the library is missing or a tensor is not on the GPU: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Optional, Sequence

import numpy as np

__all__ = ["lib", "PatError", "Plan", "Batch", "tv_prox", "restrict", "prolong", "dot_f64", "residual_f64", "residual_f64_batched",
           "tv_smooth", "restrict_lower", "axpby", "project", "tv_prox_batched", "forward_batched",
           "adjoint_batched",
           "LIB_PATH", "EXPORTED"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpat.so")

PAT_OK, PAT_EINVAL, PAT_EUNSTABLE, PAT_ENOMEM, PAT_EHIP, PAT_ENONFINITE, PAT_ENOSYS, PAT_ETOOBIG = range(8)
PAT_NO_PML = 0x1
PAT_CHECK_FINITE = 0x2
PAT_SMOOTH_P0 = 0x8
PAT_EOS_INIT = 0x10
PAT_BATCH_NO_FUSE = 0x1
PAT_BATCH_NO_STAGGER = 0x2

#: every symbol include/pat.h declares
EXPORTED = [
    "pat_plan_create", "pat_plan_destroy", "pat_plan_info", "pat_forward", "pat_adjoint", "pat_adjoint_atd",
    "pat_forward_range", "pat_batch_create", "pat_batch_create_ex", "pat_batch_destroy", "pat_batch_forward",
    "pat_batch_adjoint", "pat_tv_prox_work_bytes", "pat_tv_prox", "pat_tv_prox_batched", "pat_restrict",
    "pat_prolong",
    "pat_dot_f64", "pat_residual_f64", "pat_residual_f64_batched", "pat_residual_batched_work_bytes", "pat_plan_sync", "pat_strerror", "pat_timing_begin",
    "pat_timing_end", "pat_batch_autotune", "pat_tuning_report", "pat_batch_set_tile", "pat_batch_time_pass",
    "pat_tv_smooth", "pat_restrict_lower", "pat_axpby", "pat_project", "pat_forward_batched",
    "pat_adjoint_batched", "pat_desc_check", "pat_tv_prox_noalloc", "pat_diag_sync_costs",
]


class PatError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.pat_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


class CDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double * 3),
        ("origin", ctypes.c_double * 3), ("nt", ctypes.c_int32), ("dt", ctypes.c_double),
        ("cfl", ctypes.c_double), ("pml_size", ctypes.c_int32 * 3), ("pml_alpha", ctypes.c_double),
        ("alpha_power", ctypes.c_double), ("n_sensors", ctypes.c_int32), ("flags", ctypes.c_uint32),
    ]


class CInfo(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double), ("c_ref", ctypes.c_double), ("npoints", ctypes.c_int64),
        ("lossy", ctypes.c_int32), ("n_slots", ctypes.c_int32), ("device_bytes", ctypes.c_size_t),
        ("state_bytes", ctypes.c_size_t),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libpat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libpat.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "pat_plan_create": (ctypes.c_int, [pp, ctypes.POINTER(CDesc), vp, vp, vp, vp, vp]),
        "pat_plan_destroy": (None, [vp]),
        "pat_desc_check": (ctypes.c_int, [ctypes.POINTER(CDesc), i32, vp, f64]),
        "pat_plan_info": (ctypes.c_int, [vp, ctypes.POINTER(CInfo)]),
        "pat_forward": (ctypes.c_int, [vp, vp, vp, vp]),
        "pat_adjoint": (ctypes.c_int, [vp, vp, vp, vp]),
        "pat_adjoint_atd": (ctypes.c_int, [vp, vp, vp, vp]),
        "pat_forward_range": (ctypes.c_int, [vp, vp, vp, i32, i32, vp, vp]),
        "pat_batch_create": (ctypes.c_int, [pp, pp, i32, i32]),
        "pat_batch_create_ex": (ctypes.c_int, [pp, pp, i32, i32, i32, i32, ctypes.c_uint32]),
        "pat_batch_destroy": (None, [vp]),
        "pat_batch_forward": (ctypes.c_int, [vp, pp, pp, vp]),
        "pat_batch_adjoint": (ctypes.c_int, [vp, pp, pp, vp]),
        "pat_forward_batched": (ctypes.c_int, [pp, i32, pp, pp, vp]),
        "pat_adjoint_batched": (ctypes.c_int, [pp, i32, pp, pp, vp]),
        "pat_tv_prox_work_bytes": (sz, [i32, ctypes.POINTER(i32)]),
        "pat_tv_prox": (ctypes.c_int, [i32, ctypes.POINTER(i32), vp, vp, f64, i32, vp, vp, sz, vp]),
        "pat_diag_sync_costs": (ctypes.c_int, [i32, i32, i32, ctypes.POINTER(f64), ctypes.POINTER(f64),
                                                ctypes.POINTER(f64), ctypes.POINTER(f64)]),
        "pat_tv_prox_noalloc": (ctypes.c_int, [i32, ctypes.POINTER(i32), vp, vp, f64, i32, vp, vp]),
        "pat_tv_prox_batched": (ctypes.c_int, [i32, i32, ctypes.POINTER(i32), pp, pp, ctypes.POINTER(f64), i32, pp,
                                               pp, ctypes.POINTER(sz), vp]),
        "pat_restrict": (ctypes.c_int, [i32, ctypes.POINTER(i32), vp, vp, vp]),
        "pat_prolong": (ctypes.c_int, [i32, ctypes.POINTER(i32), vp, vp, vp]),
        "pat_dot_f64": (ctypes.c_int, [vp, vp, i64, ctypes.POINTER(f64), vp]),
        "pat_residual_f64": (ctypes.c_int, [vp, vp, vp, i64, ctypes.POINTER(f64), vp]),
        "pat_residual_f64_batched": (ctypes.c_int, [i32, vp, vp, vp, vp, vp, vp, vp]),
        "pat_residual_batched_work_bytes": (ctypes.c_size_t, [i32]),
        "pat_plan_sync": (ctypes.c_int, [vp, vp]),
        "pat_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "pat_timing_begin": (ctypes.c_int, [i32, i32, i32]),
        "pat_timing_end": (ctypes.c_int, [ctypes.POINTER(f64), ctypes.POINTER(i64), ctypes.POINTER(f64)]),
        "pat_batch_autotune": (ctypes.c_int, [vp, i32, vp]),
        "pat_tv_smooth": (ctypes.c_int, [i32, ctypes.POINTER(i32), vp, f64, f64, vp, ctypes.POINTER(f64), vp]),
        "pat_restrict_lower": (ctypes.c_int, [i32, ctypes.POINTER(i32), vp, vp, vp, vp]),
        "pat_axpby": (ctypes.c_int, [i64, f64, vp, f64, vp, vp, vp]),
        "pat_project": (ctypes.c_int, [i64, vp, vp, vp, vp]),
        "pat_batch_time_pass": (ctypes.c_int, [vp, i32, i32, i32, i32, vp, ctypes.POINTER(f64), ctypes.POINTER(f64)]),
        "pat_tuning_report": (ctypes.c_int, [vp, ctypes.c_char_p, sz, ctypes.POINTER(sz)]),
        "pat_batch_set_tile": (ctypes.c_int, [vp, ctypes.POINTER(i32), i32, i32, i32, i32, i32, i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(code: int, where: str) -> None:
    if code != PAT_OK:
        raise PatError(code, where)


def _torch():
    import torch
    return torch


def _stream(stream=None) -> ctypes.c_void_p:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(t, name: str, numel: Optional[int] = None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the HIP device")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _i32x3(v: Sequence[int]):
    a = (ctypes.c_int32 * 3)(*([int(x) for x in v] + [1] * (3 - len(v))))
    return a


def make_desc(desc, n_sensors: int, check_finite: bool = False) -> CDesc:
    """C descriptor from any object with the GridDesc attributes."""
    nd = int(desc.ndim)
    c = CDesc()
    c.ndim = nd
    for j in range(3):
        c.n[j] = int(desc.n[j]) if j < nd else 1
        c.dx[j] = float(desc.dx[j]) if j < nd else 1.0
        c.origin[j] = float(desc.origin[j]) if j < nd else 0.0
        c.pml_size[j] = int(desc.pml_size[j]) if j < len(desc.pml_size) else 0
    c.nt = int(desc.nt)
    c.dt = float(desc.dt)
    c.cfl = float(desc.cfl)
    c.pml_alpha = float(desc.pml_alpha)
    c.alpha_power = float(desc.alpha_power)
    c.n_sensors = int(n_sensors)
    c.flags = ((0 if getattr(desc, "pml", True) else PAT_NO_PML) | (PAT_CHECK_FINITE if check_finite else 0) |
               (PAT_SMOOTH_P0 if getattr(desc, "smooth_p0", False) else 0) |
               (PAT_EOS_INIT if getattr(desc, "section3_density", False) else 0))
    return c


class Plan:
    """One solver instance (a grid level) resident on the GPU.

    ``c0``, ``rho0`` and ``alpha0_db`` are float32 tensors (or arrays, copied
    to the device) of the grid's shape; ``sensors`` is an (ns, ndim) array of
    physical positions.  ``alpha0_db=None`` selects a lossless medium."""

    def __init__(self, desc, c0, rho0, alpha0_db, sensors, *, device="cuda", check_finite=False):
        torch = _torch()
        L = lib()
        self.desc = desc
        self.ndim = int(desc.ndim)
        self.shape = tuple(int(v) for v in reversed(desc.n[: self.ndim]))
        self.npoints = int(np.prod(self.shape))
        sens = np.ascontiguousarray(np.asarray(sensors, dtype=np.float64).reshape(-1, self.ndim))
        self.ns = sens.shape[0]
        self.nt = int(desc.nt)

        def dev(a):
            if a is None:
                return None
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a, np.float32))
            return t.to(device=device, dtype=torch.float32).contiguous()

        c0t, r0t, a0t = dev(c0), dev(rho0), dev(alpha0_db)
        cd = make_desc(desc, self.ns, check_finite)
        h = ctypes.c_void_p()
        rc = L.pat_plan_create(ctypes.byref(h), ctypes.byref(cd), _dev_f32(c0t, "c0", self.npoints),
                               _dev_f32(r0t, "rho0", self.npoints),
                               None if a0t is None else _dev_f32(a0t, "alpha0_db", self.npoints),
                               sens.ctypes.data_as(ctypes.c_void_p), _stream())
        _check(rc, "pat_plan_create")
        self._h = h
        self._device = device
        info = CInfo()
        _check(L.pat_plan_info(h, ctypes.byref(info)), "pat_plan_info")
        self.dt = info.dt
        self.c_ref = info.c_ref
        self.lossy = bool(info.lossy)
        self.device_bytes = int(info.device_bytes)
        self.state_bytes = int(info.state_bytes)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pat_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, p0, data=None):
        """data[n, s] = (H p0) sampled at t = n dt (shape (nt, ns))."""
        torch = _torch()
        if data is None:
            data = torch.empty((self.nt, self.ns), device=p0.device, dtype=torch.float32)
        _check(lib().pat_forward(self._h, _dev_f32(p0, "p0", self.npoints),
                                 _dev_f32(data, "data", self.nt * self.ns), _stream()), "pat_forward")
        return data

    def adjoint(self, data, img=None):
        """img = H^T data (shape of the grid)."""
        torch = _torch()
        if img is None:
            img = torch.empty(self.shape, device=data.device, dtype=torch.float32)
        _check(lib().pat_adjoint(self._h, _dev_f32(data, "data", self.nt * self.ns),
                                 _dev_f32(img, "img", self.npoints), _stream()), "pat_adjoint")
        return img

    def adjoint_atd(self, data, img=None):
        """The paper's adjoint-then-discretize operator applied to data
        (pat_adjoint_atd); for comparison with the exact transpose."""
        torch = _torch()
        if img is None:
            img = torch.empty(self.shape, device=data.device, dtype=torch.float32)
        _check(lib().pat_adjoint_atd(self._h, _dev_f32(data, "data", self.nt * self.ns),
                                     _dev_f32(img, "img", self.npoints), _stream()), "pat_adjoint_atd")
        return img

    def forward_range(self, p0, data, n_begin: int, n_end: int, state):
        """Samples n_begin..n_end-1 into data; state (uint8 tensor of
        state_bytes) is read when n_begin > 0 and receives the end state."""
        torch = _torch()
        if state.dtype != torch.uint8 or state.numel() < self.state_bytes or not state.is_cuda:
            raise ValueError("state must be a uint8 device tensor of state_bytes")
        _check(lib().pat_forward_range(self._h, None if p0 is None else _dev_f32(p0, "p0", self.npoints),
                                       _dev_f32(data, "data", self.nt * self.ns), int(n_begin), int(n_end),
                                       ctypes.c_void_p(state.data_ptr()), _stream()), "pat_forward_range")
        return data

    def sync(self):
        """Wait for the plan's work; raises PatError(ENONFINITE) if flagged."""
        _check(lib().pat_plan_sync(self._h, _stream()), "pat_plan_sync")


class Batch:
    """Many plans run together (one launch per pass over all instances)."""

    def __init__(self, plans: Sequence[Plan], chunk: int = 0, parts: int = 0, lanes: int = 0, fuse: bool = True,
                 stagger: bool = True):
        """chunk: steps per captured graph (0: 64; 1: eager); parts: groups
        per size class (0: 2); lanes: streams (0: one per group; fewer:
        groups placed heaviest first on the least-loaded stream); fuse: 2D
        size classes of axes 128/256/512 share their launches; stagger: odd
        groups start one pass after the first (see pat_batch_create_ex)."""
        self.plans = list(plans)
        self._opts = (int(chunk), int(parts), int(lanes), bool(fuse), bool(stagger))
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        flags = (0 if fuse else PAT_BATCH_NO_FUSE) | (0 if stagger else PAT_BATCH_NO_STAGGER)
        _check(lib().pat_batch_create_ex(ctypes.byref(h), arr, len(self.plans), int(chunk), int(parts), int(lanes),
                                         flags),
               "pat_batch_create_ex")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pat_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, p0s, datas=None):
        torch = _torch()
        if datas is None:
            datas = [torch.empty((p.nt, p.ns), device=x.device, dtype=torch.float32) for p, x in zip(self.plans, p0s)]
        a = (ctypes.c_void_p * len(self.plans))(*[_dev_f32(x, "p0", p.npoints).value for p, x in zip(self.plans, p0s)])
        b = (ctypes.c_void_p * len(self.plans))(*[_dev_f32(d, "data", p.nt * p.ns).value
                                                  for p, d in zip(self.plans, datas)])
        _check(lib().pat_batch_forward(self._h, a, b, _stream()), "pat_batch_forward")
        return datas

    def adjoint(self, datas, imgs=None):
        torch = _torch()
        if imgs is None:
            imgs = [torch.empty(p.shape, device=d.device, dtype=torch.float32) for p, d in zip(self.plans, datas)]
        a = (ctypes.c_void_p * len(self.plans))(*[_dev_f32(d, "data", p.nt * p.ns).value
                                                  for p, d in zip(self.plans, datas)])
        b = (ctypes.c_void_p * len(self.plans))(*[_dev_f32(x, "img", p.npoints).value for p, x in zip(self.plans, imgs)])
        _check(lib().pat_batch_adjoint(self._h, a, b, _stream()), "pat_batch_adjoint")
        return imgs

    def time_pass(self, direction: int, pass_index: int, nx: int = 0, reps: int = 100):
        """(microseconds, algorithmic bytes) per launch of one pass, from
        back-to-back launches (pat_batch_time_pass)."""
        us, by = ctypes.c_double(), ctypes.c_double()
        _check(lib().pat_batch_time_pass(self._h, int(direction), int(pass_index), int(nx), int(reps), _stream(),
                                         ctypes.byref(us), ctypes.byref(by)), "pat_batch_time_pass")
        return us.value, by.value

    def tuning_report(self) -> list:
        """The autotuner's choices (list of dicts, see pat_tuning_report)."""
        need = ctypes.c_size_t()
        _check(lib().pat_tuning_report(self._h, None, 0, ctypes.byref(need)), "pat_tuning_report")
        buf = ctypes.create_string_buffer(need.value + 1)
        _check(lib().pat_tuning_report(self._h, buf, need.value + 1, ctypes.byref(need)), "pat_tuning_report")
        return json.loads(buf.value.decode())

    def set_tile(self, entry: dict, tile: Optional[int] = None, fpb: Optional[int] = None) -> None:
        """Apply one stored choice: a report entry (keys n, nt, lossy, dir,
        pass, tile, fpb); ``tile`` / ``fpb`` override the entry's."""
        t = entry["tile"] if tile is None else tile
        f = entry.get("fpb", 1) if fpb is None else fpb
        _check(lib().pat_batch_set_tile(self._h, _i32x3(list(entry["n"])), int(entry["nt"]), int(entry["lossy"]),
                                        int(entry["dir"]), int(entry["pass"]), int(t), int(f)),
               "pat_batch_set_tile")

    def autotune(self, reps: int = 20, cache: Optional[str] = None) -> list:
        """Pick the column tile widths by timing (pat_batch_autotune).

        With ``cache`` (a JSON file), the choices stored there for this
        device architecture and this batch composition (size classes with
        their instance counts, grouping options) are applied without timing;
        otherwise the batch is timed and its report stored in the file.
        Returns the report entries in force."""
        arch = _arch()
        key = self._batch_key()
        if cache and os.path.exists(cache):
            with open(cache) as f:
                entries = json.load(f).get(arch, {}).get(key)
            if entries is not None:
                for e in entries:
                    self.set_tile(e)
                return entries
        _check(lib().pat_batch_autotune(self._h, int(reps), _stream()), "pat_batch_autotune")
        rep = self.tuning_report()
        if cache:
            data = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    data = json.load(f)
            data.setdefault(arch, {})[key] = rep
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1)
            os.replace(tmp, cache)
        return rep

    def _batch_key(self) -> str:
        """Cache key of the batch: every size class (grid, time samples,
        physics, instance count) and the grouping options -- the timings of
        one class depend on what runs beside it."""
        count = {}
        for p in self.plans:
            n = _grid3(p)
            k = f"{n[0]}x{n[1]}x{n[2]}/nt{p.nt}/{'lossy' if p.lossy else 'lossless'}"
            count[k] = count.get(k, 0) + 1
        chunk, parts, lanes, fuse, stagger = self._opts
        return ";".join(f"{k}/i{v}" for k, v in sorted(count.items())) + \
            f"|chunk{chunk}/parts{parts}/lanes{lanes}/{'fused' if fuse else 'unfused'}" + \
            ("/staggered" if stagger else "")


def _grid3(plan) -> list:
    """(nx, ny, nz) of a plan, nz = 1 in 2D."""
    n = list(reversed(plan.shape))
    return n + [1] * (3 - len(n))


def _arch() -> str:
    torch = _torch()
    return str(torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName).split(":")[0]


def timing_begin(direction: int, pass_index: int, nx: int = 0) -> None:
    """Start HIP-event timing of one pass of the time step (see pat.h)."""
    _check(lib().pat_timing_begin(int(direction), int(pass_index), int(nx)), "pat_timing_begin")


def timing_end():
    """(total milliseconds, launches, algorithmic bytes) of the timed pass."""
    ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(lib().pat_timing_end(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)), "pat_timing_end")
    return ms.value, n.value, b.value


def tv_prox(z, lam: float, n_iter: int = 20, lower=None, out=None, work=None):
    """argmin_x lam TV(x) + 1/2||x - z||^2 s.t. x >= lower (FGP, n_iter steps)."""
    torch = _torch()
    nd = z.dim()
    n = _i32x3(list(reversed(z.shape)))
    nbytes = lib().pat_tv_prox_work_bytes(nd, n)
    if out is None:
        out = torch.empty_like(z)
    if work is None:
        work = torch.empty(max(1, nbytes), dtype=torch.uint8, device=z.device)
    _check(lib().pat_tv_prox(nd, n, _dev_f32(z, "z"), _dev_f32(out, "x", z.numel()), float(lam), int(n_iter),
                             None if lower is None else _dev_f32(lower, "lower", z.numel()),
                             ctypes.c_void_p(work.data_ptr()), ctypes.c_size_t(work.numel()), _stream()),
           "pat_tv_prox")
    return out


def forward_batched(plans, p0s, datas=None):
    """H of several plans in one call (pat_forward_batched: the library keeps
    one batch per distinct plan list); returns the list of data tensors."""
    torch = _torch()
    if datas is None:
        datas = [torch.empty((p.nt, p.ns), device=x.device, dtype=torch.float32) for p, x in zip(plans, p0s)]
    k = len(plans)
    hs = (ctypes.c_void_p * k)(*[p.handle.value for p in plans])
    a = (ctypes.c_void_p * k)(*[_dev_f32(x, "p0", p.npoints).value for p, x in zip(plans, p0s)])
    b = (ctypes.c_void_p * k)(*[_dev_f32(d, "data", p.nt * p.ns).value for p, d in zip(plans, datas)])
    _check(lib().pat_forward_batched(hs, k, a, b, _stream()), "pat_forward_batched")
    return datas


def adjoint_batched(plans, datas, imgs=None):
    """H^T of several plans in one call (pat_adjoint_batched); returns the
    list of images."""
    torch = _torch()
    if imgs is None:
        imgs = [torch.empty(p.shape, device=d.device, dtype=torch.float32) for p, d in zip(plans, datas)]
    k = len(plans)
    hs = (ctypes.c_void_p * k)(*[p.handle.value for p in plans])
    a = (ctypes.c_void_p * k)(*[_dev_f32(d, "data", p.nt * p.ns).value for p, d in zip(plans, datas)])
    b = (ctypes.c_void_p * k)(*[_dev_f32(x, "img", p.npoints).value for p, x in zip(plans, imgs)])
    _check(lib().pat_adjoint_batched(hs, k, a, b, _stream()), "pat_adjoint_batched")
    return imgs


def tv_prox_batched(zs, lams, n_iter: int = 20, lowers=None, outs=None, works=None):
    """``tv_prox`` of several images of one dimensionality in one set of
    launches (pat_tv_prox_batched); returns the list of outputs."""
    torch = _torch()
    k = len(zs)
    nd = zs[0].dim()
    dims = (ctypes.c_int32 * (3 * k))(*[v for z in zs for v in list(_i32x3(list(reversed(z.shape))))])
    if outs is None:
        outs = [torch.empty_like(z) for z in zs]
    if works is None:
        works = [torch.empty(max(1, lib().pat_tv_prox_work_bytes(nd, _i32x3(list(reversed(z.shape))))),
                             dtype=torch.uint8, device=z.device) for z in zs]
    ptr = lambda xs: (ctypes.c_void_p * k)(*xs)  # noqa: E731
    zp = ptr([_dev_f32(z, "z").value for z in zs])
    xp = ptr([_dev_f32(o, "x", z.numel()).value for o, z in zip(outs, zs)])
    lp = None if lowers is None else ptr([None if lo is None else _dev_f32(lo, "lower", z.numel()).value
                                          for lo, z in zip(lowers, zs)])
    wp = ptr([w.data_ptr() for w in works])
    wb = (ctypes.c_size_t * k)(*[w.numel() for w in works])
    lam = (ctypes.c_double * k)(*[float(v) for v in lams])
    _check(lib().pat_tv_prox_batched(k, nd, dims, zp, xp, lam, int(n_iter), lp, wp, wb, _stream()),
           "pat_tv_prox_batched")
    return outs


def restrict(fine, out=None):
    torch = _torch()
    nd = fine.dim()
    if out is None:
        out = torch.empty(tuple(s // 2 for s in fine.shape), device=fine.device, dtype=torch.float32)
    _check(lib().pat_restrict(nd, _i32x3(list(reversed(fine.shape))), _dev_f32(fine, "fine"),
                              _dev_f32(out, "coarse", fine.numel() >> nd), _stream()), "pat_restrict")
    return out


def prolong(coarse, out=None):
    torch = _torch()
    nd = coarse.dim()
    if out is None:
        out = torch.empty(tuple(2 * s for s in coarse.shape), device=coarse.device, dtype=torch.float32)
    _check(lib().pat_prolong(nd, _i32x3(list(reversed(coarse.shape))), _dev_f32(coarse, "coarse"),
                             _dev_f32(out, "fine", coarse.numel() << nd), _stream()), "pat_prolong")
    return out


def dot_f64(a, b=None) -> float:
    """sum a*b of float32 device tensors with float64 accumulation."""
    b = a if b is None else b
    out = ctypes.c_double()
    _check(lib().pat_dot_f64(_dev_f32(a, "a"), _dev_f32(b, "b", a.numel()), a.numel(), ctypes.byref(out),
                             _stream()), "pat_dot_f64")
    return out.value


def residual_f64(a, b, r=None):
    """(r = a - b, 1/2 ||a - b||^2 in float64)."""
    torch = _torch()
    if r is None:
        r = torch.empty_like(a)
    out = ctypes.c_double()
    _check(lib().pat_residual_f64(_dev_f32(a, "a"), _dev_f32(b, "b", a.numel()), _dev_f32(r, "r", a.numel()),
                                  a.numel(), ctypes.byref(out), _stream()), "pat_residual_f64")
    return r, out.value


def residual_f64_batched(As, Bs, Rs=None, work=None, out=None):
    """(list of r_i = a_i - b_i, device float64 tensor out of len(As) + 1:
    out[i] = 1/2 ||a_i - b_i||^2, out[-1] their sum), with no host
    synchronisation (pat_residual_f64_batched).  work: a uint8 device
    tensor of at least pat_residual_batched_work_bytes(len(As)) bytes
    (allocated when None)."""
    torch = _torch()
    count = len(As)
    if Rs is None:
        Rs = [torch.empty_like(a) for a in As]
    need = int(lib().pat_residual_batched_work_bytes(count))
    if work is None or work.numel() < need:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=As[0].device)
    if out is None:
        out = torch.empty(count + 1, dtype=torch.float64, device=As[0].device)
    vpa = ctypes.c_void_p * count
    pa = vpa(*[_dev_f32(a, "a").value for a in As])
    pb = vpa(*[_dev_f32(b, "b", a.numel()).value for a, b in zip(As, Bs)])
    pr = vpa(*[_dev_f32(r, "r", a.numel()).value for a, r in zip(As, Rs)])
    ns = (ctypes.c_int64 * count)(*[a.numel() for a in As])
    _check(lib().pat_residual_f64_batched(count, pa, pb, pr, ns, ctypes.c_void_p(work.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), _stream()), "pat_residual_f64_batched")
    return Rs, out


def tv_smooth(x, rho: float, grad=None, scale: float = 1.0, value: bool = True):
    """Smoothed TV J_rho(x) (float64, or None with value=False); with `grad`
    given, grad += scale * grad J_rho(x) in place."""
    out = ctypes.c_double()
    _check(lib().pat_tv_smooth(x.dim(), _i32x3(list(reversed(x.shape))), _dev_f32(x, "x"), float(rho), float(scale),
                               None if grad is None else _dev_f32(grad, "grad", x.numel()),
                               ctypes.byref(out) if value else None, _stream()), "pat_tv_smooth")
    return out.value if value else None


def restrict_lower(fine, fine_lower=None, out=None):
    """R(y) - blockmin(y - l): the coarse bound that keeps a prolonged
    correction of y above the fine bound l (None: 0)."""
    torch = _torch()
    nd = fine.dim()
    if out is None:
        out = torch.empty(tuple(s // 2 for s in fine.shape), device=fine.device, dtype=torch.float32)
    fl = None if fine_lower is None else _dev_f32(fine_lower, "fine_lower", fine.numel())
    _check(lib().pat_restrict_lower(nd, _i32x3(list(reversed(fine.shape))), _dev_f32(fine, "fine"), fl,
                                    _dev_f32(out, "lower", fine.numel() >> nd), _stream()), "pat_restrict_lower")
    return out


def axpby(a: float, x, b: float, y, out=None):
    """out = a x + b y."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(x)
    n = x.numel()
    _check(lib().pat_axpby(n, float(a), _dev_f32(x, "x"), float(b), _dev_f32(y, "y", n), _dev_f32(out, "out", n),
                           _stream()), "pat_axpby")
    return out


def project(x, lower=None, out=None):
    """out = max(x, lower) (lower None: 0)."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(x)
    n = x.numel()
    _check(lib().pat_project(n, _dev_f32(x, "x"), None if lower is None else _dev_f32(lower, "lower", n),
                             _dev_f32(out, "out", n), _stream()), "pat_project")
    return out
