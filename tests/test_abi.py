"""Host-side checks of the C ABI: the library loads and exports every
declared symbol, and the pure-host entry points validate their arguments
(no kernel is launched by any of these)."""
import ctypes
import os
import re

import pytest

import paper_1603_02329_amd as pat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pat.h")).read()
    return sorted(set(re.findall(r"\b(pat_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = pat.lib()
    declared = _declared()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(pat.EXPORTED) == declared


def test_strerror_codes():
    L = pat.lib()
    for code in range(8):
        assert L.pat_strerror(code) and L.pat_strerror(code) != b"unknown error"
    assert L.pat_strerror(99) == b"unknown error"


def test_prox_work_bytes():
    L = pat.lib()
    n = (ctypes.c_int32 * 3)(512, 256, 1)
    assert L.pat_tv_prox_work_bytes(2, n) == 5 * 512 * 256 * 4
    n3 = (ctypes.c_int32 * 3)(8, 8, 8)
    assert L.pat_tv_prox_work_bytes(3, n3) == 7 * 512 * 4
    assert L.pat_tv_prox_work_bytes(4, n3) == 0


def test_plan_create_rejects_bad_descriptors_on_host():
    """Descriptor validation happens before any device access."""
    L = pat.lib()
    import synth
    base = synth.small_instance(1, (16, 16), nt=4).desc
    cd4 = pat.make_desc(base, 3)
    cd4.ndim = 4
    h0 = ctypes.c_void_p()
    assert L.pat_plan_create(ctypes.byref(h0), ctypes.byref(cd4), ctypes.c_void_p(16), ctypes.c_void_p(16), None,
                             (ctypes.c_double * 6)(), None) == pat.PAT_EINVAL
    bad = [
        dict(n=(24, 16)), dict(n=(8, 16)), dict(n=(2048, 16)), dict(nt=0),
        dict(pml_size=(8, 2, 0)), dict(dx=(0.0, 1e-4)), dict(dt=0.0, cfl=0.0),
    ]
    from dataclasses import replace
    for kw in bad:
        d = replace(base, **kw)
        cd = pat.make_desc(d, 3)
        h = ctypes.c_void_p()
        dummy = ctypes.c_void_p(16)
        pos = (ctypes.c_double * 6)()
        rc = L.pat_plan_create(ctypes.byref(h), ctypes.byref(cd), dummy, dummy, None, pos, None)
        assert rc == pat.PAT_EINVAL, kw
    # bad power-law exponent only matters for a lossy medium
    d = replace(base, alpha_power=1.0)
    cd = pat.make_desc(d, 3)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    assert L.pat_plan_create(ctypes.byref(h), ctypes.byref(cd), dummy, dummy, dummy, (ctypes.c_double * 6)(),
                             None) == pat.PAT_EINVAL
    # unknown plan flags (0x4 and 0x20 are undefined)
    for bad in (0x4, pat.PAT_EOS_INIT << 1):
        cd = pat.make_desc(base, 3)
        cd.flags = bad
        assert L.pat_plan_create(ctypes.byref(h), ctypes.byref(cd), dummy, dummy, None, (ctypes.c_double * 6)(),
                                 None) == pat.PAT_EINVAL
        assert L.pat_desc_check(ctypes.byref(cd), 0, (ctypes.c_double * 6)(), 0.0) == pat.PAT_EINVAL
    assert pat.make_desc(replace(base, smooth_p0=True), 3).flags == pat.PAT_SMOOTH_P0
    cd = pat.make_desc(replace(base, section3_density=True), 3)
    assert cd.flags == pat.PAT_EOS_INIT
    assert L.pat_desc_check(ctypes.byref(cd), 0, (ctypes.c_double * 6)(), 0.0) == pat.PAT_OK
    # NULL arguments
    cd = pat.make_desc(base, 3)
    assert L.pat_plan_create(ctypes.byref(h), ctypes.byref(cd), None, dummy, None, (ctypes.c_double * 6)(),
                             None) == pat.PAT_EINVAL
    assert L.pat_plan_create(None, ctypes.byref(cd), dummy, dummy, None, (ctypes.c_double * 6)(),
                             None) == pat.PAT_EINVAL


def test_null_plan_calls_are_rejected():
    L = pat.lib()
    assert L.pat_forward(None, None, None, None) == pat.PAT_EINVAL
    assert L.pat_adjoint(None, None, None, None) == pat.PAT_EINVAL
    assert L.pat_plan_info(None, None) == pat.PAT_EINVAL
    assert L.pat_plan_sync(None, None) == pat.PAT_EINVAL
    L.pat_plan_destroy(None)
    n = (ctypes.c_int32 * 3)(16, 16, 1)
    assert L.pat_restrict(2, n, None, None, None) == pat.PAT_EINVAL
    assert L.pat_prolong(5, n, None, None, None) == pat.PAT_EINVAL
    assert L.pat_tv_prox(2, n, None, None, 0.1, 20, None, None, 0, None) == pat.PAT_EINVAL
    out = ctypes.c_double(7.0)
    assert L.pat_dot_f64(None, None, 0, ctypes.byref(out), None) == pat.PAT_OK and out.value == 0.0
    assert L.pat_dot_f64(None, None, 5, ctypes.byref(out), None) == pat.PAT_EINVAL
    # batched residuals: rejected before any device access
    assert L.pat_residual_batched_work_bytes(48) == 48 * 512 * 8 and L.pat_residual_batched_work_bytes(0) == 0
    ptrs = (ctypes.c_void_p * 2)(None, None)
    ns = (ctypes.c_int64 * 2)(0, 0)
    w = ctypes.c_void_p(8)  # never dereferenced: every call below fails its checks first
    assert L.pat_residual_f64_batched(0, ptrs, ptrs, ptrs, ns, w, w, None) == pat.PAT_EINVAL
    assert L.pat_residual_f64_batched(4097, ptrs, ptrs, ptrs, ns, w, w, None) == pat.PAT_EINVAL
    assert L.pat_residual_f64_batched(2, None, ptrs, ptrs, ns, w, w, None) == pat.PAT_EINVAL
    assert L.pat_residual_f64_batched(2, ptrs, ptrs, ptrs, ns, None, w, None) == pat.PAT_EINVAL
    bad = (ctypes.c_int64 * 2)(0, -1)
    assert L.pat_residual_f64_batched(2, ptrs, ptrs, ptrs, bad, w, w, None) == pat.PAT_EINVAL
    some = (ctypes.c_int64 * 2)(0, 5)  # n > 0 with NULL pointers
    assert L.pat_residual_f64_batched(2, ptrs, ptrs, ptrs, some, w, w, None) == pat.PAT_EINVAL


def test_batch_entry_points_validate_on_host():
    """Argument checks that return before any plan or device access."""
    L = pat.lib()
    h = ctypes.c_void_p()
    one = (ctypes.c_void_p * 1)(None)
    assert L.pat_batch_create(None, one, 1, 0) == pat.PAT_EINVAL
    assert L.pat_batch_create(ctypes.byref(h), None, 1, 0) == pat.PAT_EINVAL
    assert L.pat_batch_create(ctypes.byref(h), one, 0, 0) == pat.PAT_EINVAL
    assert L.pat_batch_create(ctypes.byref(h), one, 1, -1) == pat.PAT_EINVAL
    assert L.pat_batch_create_ex(ctypes.byref(h), one, 1, 0, -1, 0, 0) == pat.PAT_EINVAL
    assert L.pat_batch_create_ex(ctypes.byref(h), one, 1, 0, 0, -1, 0) == pat.PAT_EINVAL
    assert L.pat_batch_create_ex(ctypes.byref(h), one, 1, 0, 0, 0, 0x4) == pat.PAT_EINVAL  # unknown flag
    assert L.pat_batch_create(ctypes.byref(h), one, 1, 0) == pat.PAT_EINVAL  # null plan pointer
    assert h.value is None
    assert L.pat_batch_autotune(None, 1, None) == pat.PAT_EINVAL
    ptrs = (ctypes.c_void_p * 1)(None)
    for fn in (L.pat_forward_batched, L.pat_adjoint_batched):
        assert fn(None, 1, ptrs, ptrs, None) == pat.PAT_EINVAL     # no plan array
        assert fn(one, 0, ptrs, ptrs, None) == pat.PAT_EINVAL      # nb < 1
        assert fn(one, 1, ptrs, ptrs, None) == pat.PAT_EINVAL      # null plan entry
        assert fn(one, 1, None, ptrs, None) == pat.PAT_EINVAL      # no input array
    need = ctypes.c_size_t()
    assert L.pat_tuning_report(None, None, 0, ctypes.byref(need)) == pat.PAT_EINVAL
    n = (ctypes.c_int32 * 3)(16, 16, 1)
    assert L.pat_batch_set_tile(None, n, 1, 1, 0, 0, 16, 1) == pat.PAT_EINVAL


def _check_desc(desc, sensors, c_max, lossy=True):
    L = pat.lib()
    import numpy as np
    pos = np.ascontiguousarray(np.asarray(sensors, dtype=np.float64))
    cd = pat.make_desc(desc, pos.shape[0])
    return L.pat_desc_check(ctypes.byref(cd), 1 if lossy else 0, pos.ctypes.data_as(ctypes.c_void_p), c_max)


def test_desc_check_stability_bound():
    """PAT_EUNSTABLE above c_max dt / min dx = 1/sqrt(d), on the host, for an
    explicit dt and for the CFL rule; exactly at the bound is accepted."""
    import math
    from dataclasses import replace

    import synth
    for n in ((16, 16), (16, 16, 16)):
        inst = synth.small_instance(3, n, nt=4)
        d = inst.desc
        nd = len(n)
        dx = d.dx[0]
        c = 1600.0
        bound = dx / (c * math.sqrt(nd))
        assert _check_desc(replace(d, dt=0.99 * bound), inst.sensors, c) == pat.PAT_OK
        assert _check_desc(replace(d, dt=bound), inst.sensors, c) == pat.PAT_OK
        assert _check_desc(replace(d, dt=1.01 * bound), inst.sensors, c) == pat.PAT_EUNSTABLE
        assert _check_desc(replace(d, dt=0.0, cfl=0.3), inst.sensors, c) == pat.PAT_OK
        assert _check_desc(replace(d, dt=0.0, cfl=1.02 / math.sqrt(nd)), inst.sensors, c) == pat.PAT_EUNSTABLE
        # c_max <= 0: the stability check is skipped
        assert _check_desc(replace(d, dt=10 * bound), inst.sensors, 0.0) == pat.PAT_OK
        assert _check_desc(replace(d, dt=bound), inst.sensors, float("inf")) == pat.PAT_EINVAL


def test_desc_check_rejects_sensors_outside_the_grid():
    """Every grid coordinate (pos - origin)/dx must lie in [0, n - 1]: the
    edges themselves are accepted, a step beyond either edge, a NaN or an
    infinite coordinate is PAT_EINVAL, on every axis, 2D and 3D."""
    import numpy as np

    import synth
    for n in ((16, 32), (16, 16, 32)):
        inst = synth.small_instance(4, n, nt=4, ns=3)
        d = inst.desc
        nd = len(n)
        assert _check_desc(d, inst.sensors, 1500.0) == pat.PAT_OK
        for j in range(nd):
            lo = d.origin[j]
            hi = d.origin[j] + (d.n[j] - 1) * d.dx[j]
            for v, ok in ((lo, True), (hi, True), (lo - 1e-3 * d.dx[j], False), (hi + 1e-3 * d.dx[j], False),
                          (float("nan"), False), (float("inf"), False)):
                s = np.array(inst.sensors, dtype=np.float64)
                s[1, j] = v
                rc = _check_desc(d, s, 1500.0)
                assert rc == (pat.PAT_OK if ok else pat.PAT_EINVAL), (n, j, v, rc)
    assert pat.lib().pat_desc_check(ctypes.byref(pat.make_desc(inst.desc, 3)), 1, None, 1500.0) == pat.PAT_EINVAL
