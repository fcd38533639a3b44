"""GPU: pat_tv_prox_noalloc (the prox with its workspace in the library's
fixed device array) against pat_tv_prox with a caller workspace, through the
C ABI: two calls in a row, the second on a smaller grid, each bitwise equal
to the workspace entry point's result (same kernels, same order of
operations); a grid too large for the array is refused on the host."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1603_02329_amd as pat  # noqa: E402

DEV = "cuda"


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _prox_pair(shape, lam, n_iter, lower, seed):
    L = pat.lib()
    rng = np.random.default_rng(seed)
    z = torch.from_numpy(rng.standard_normal(shape).astype(np.float32)).to(DEV)
    lo = torch.from_numpy((0.2 * rng.standard_normal(shape)).astype(np.float32)).to(DEV) if lower else None
    n = pat._i32x3(list(reversed(shape)))
    nd = len(shape)
    x_ref = torch.empty_like(z)
    x_na = torch.full_like(z, float("nan"))
    work = torch.empty(L.pat_tv_prox_work_bytes(nd, n), dtype=torch.uint8, device=DEV)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.pat_tv_prox(nd, n, _ptr(z), _ptr(x_ref), lam, n_iter, _ptr(lo), _ptr(work), work.numel(), stream)
    assert rc == pat.PAT_OK
    rc = L.pat_tv_prox_noalloc(nd, n, _ptr(z), _ptr(x_na), lam, n_iter, _ptr(lo), stream)
    assert rc == pat.PAT_OK
    torch.cuda.synchronize()
    return x_ref, x_na


@pytest.mark.parametrize("first,second", [((512, 512), (256, 128)), ((64, 64, 64), (32, 16, 16))])
def test_noalloc_prox_equals_workspace_prox(first, second):
    for shape, lower, seed in ((first, False, 1), (second, True, 2)):
        x_ref, x_na = _prox_pair(shape, 1e-2, 20, lower, seed)
        assert torch.isfinite(x_na).all()
        assert torch.equal(x_na, x_ref), shape
        # the prox did something: the output is not the projection of z
        print(f"noalloc prox {shape}: bitwise equal, max |x| {float(x_ref.abs().max()):.3f}", flush=True)


def test_noalloc_prox_projection_and_size_limit():
    x_ref, x_na = _prox_pair((128, 64), 0.0, 20, True, 3)  # lambda 0: the projection only
    assert torch.equal(x_na, x_ref)
    L = pat.lib()
    big = pat._i32x3([1024, 1024])  # 5 * 2^20 floats > 2^22
    dummy = ctypes.c_void_p(16)
    assert L.pat_tv_prox_noalloc(2, big, dummy, ctypes.c_void_p(32), 1e-2, 20, None, None) == pat.PAT_ETOOBIG
    assert L.pat_tv_prox_noalloc(3, pat._i32x3([128, 128, 64]), dummy, ctypes.c_void_p(32), 1e-2, 20, None,
                                 None) == pat.PAT_ETOOBIG
    assert L.pat_tv_prox_noalloc(2, big, None, None, 1e-2, 20, None, None) == pat.PAT_EINVAL
