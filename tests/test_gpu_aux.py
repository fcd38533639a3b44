"""GPU parity of the TV prox, the transfers and the FP64 reductions."""
import math

import numpy as np
import pytest

from oracle import prox as OP
from oracle import transfer as OT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1603_02329_amd as pat  # noqa: E402

DEV = "cuda"


@pytest.mark.parametrize("shape,lam", [((64, 48), 0.05), ((512, 512), 1e-3), ((17, 9), 0.3), ((16, 12, 10), 0.1)])
def test_tv_prox_parity(shape, lam):
    rng = np.random.default_rng(1)
    z = (rng.standard_normal(shape) * 0.1 + 0.3).astype(np.float32)
    lo = (rng.uniform(-0.2, 0.2, size=shape)).astype(np.float32)
    for lower in (None, lo):
        ref = OP.tv_prox(z, lam, 20, lower)
        got = pat.tv_prox(torch.from_numpy(z).to(DEV), lam, 20,
                          None if lower is None else torch.from_numpy(lower).to(DEV)).cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= 1e-5, err


def test_tv_prox_zero_lambda_is_projection():
    rng = np.random.default_rng(2)
    z = rng.standard_normal((32, 32)).astype(np.float32)
    lo = rng.standard_normal((32, 32)).astype(np.float32)
    got = pat.tv_prox(torch.from_numpy(z).to(DEV), 0.0, 20, torch.from_numpy(lo).to(DEV)).cpu().numpy()
    assert np.array_equal(got, np.maximum(z, lo))


@pytest.mark.parametrize("shape", [(512, 512), (16, 32), (8, 16, 32)])
def test_transfers(shape):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(shape).astype(np.float32)
    r = pat.restrict(torch.from_numpy(x).to(DEV)).cpu().numpy()
    ref = OT.restrict(x)
    assert np.abs(r - ref).max() <= 1e-6 * np.abs(ref).max()
    c = rng.standard_normal(tuple(s // 2 for s in shape)).astype(np.float32)
    p = pat.prolong(torch.from_numpy(c).to(DEV)).cpu().numpy()
    assert np.array_equal(p, OT.prolong(c).astype(np.float32))


@pytest.mark.parametrize("n", [1, 1000, 262144, 3_000_001])
def test_dot_f64(n):
    rng = np.random.default_rng(4)
    a = rng.standard_normal(n).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    ta, tb = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
    got = pat.dot_f64(ta, tb)
    ref = OT.dot(a, b)
    scale = math.sqrt(OT.dot(a, a) * OT.dot(b, b))
    assert abs(got - ref) <= 1e-14 * scale
    assert pat.dot_f64(ta, tb) == got  # deterministic
    r, half = pat.residual_f64(ta, tb)
    assert np.array_equal(r.cpu().numpy(), a - b)
    assert abs(half - 0.5 * OT.norm2(a - b)) <= 1e-13 * half


def test_residual_f64_batched_equals_single_calls():
    """70 pairs (two launches of at most 64) of uneven sizes, empty ones
    included: every r_i and 1/2 ||a_i - b_i||^2 equals pat_residual_f64's
    bitwise, the last entry is their sum in index order, and nothing is
    read back in between (one synchronisation at the end)."""
    rng = np.random.default_rng(12)
    sizes = [0, 1, 7, 511, 512, 513, 100_000, 614_400] + [int(x) for x in rng.integers(1, 200_000, size=62)]
    As = [torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(DEV) for n in sizes]
    Bs = [torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(DEV) for n in sizes]
    Rs, out = pat.residual_f64_batched(As, Bs)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    total = 0.0
    for k, (a, b) in enumerate(zip(As, Bs)):
        r, half = pat.residual_f64(a, b)
        assert torch.equal(Rs[k], r), k
        assert out[k] == half, (k, out[k], half)
        total += half
    assert out[len(sizes)] == total
    # a second call reuses a caller-provided workspace and output
    work = torch.empty(pat.lib().pat_residual_batched_work_bytes(len(sizes)), dtype=torch.uint8, device=DEV)
    _, out2 = pat.residual_f64_batched(As, Bs, work=work)
    assert np.array_equal(out2.cpu().numpy(), out)


@pytest.mark.parametrize("ndim", [2, 3])
def test_tv_prox_batched_equals_single(ndim):
    """The batched prox (more images than one launch takes, mixed sizes,
    some with a lower bound, one with lambda = 0) equals per-image calls
    bitwise."""
    rng = np.random.default_rng(40 + ndim)
    shapes = [(16, 16), (32, 16), (8, 24), (64, 32)] if ndim == 2 else [(4, 8, 8), (8, 8, 16), (6, 4, 10)]
    count = 27 if ndim == 2 else 5
    zs, lams, lowers = [], [], []
    for k in range(count):
        sh = shapes[k % len(shapes)]
        zs.append(torch.from_numpy(rng.standard_normal(sh).astype(np.float32)).to(DEV))
        lams.append(0.0 if k == 3 else float(rng.uniform(0.05, 0.5)))
        lowers.append(torch.from_numpy((0.3 * rng.standard_normal(sh)).astype(np.float32)).to(DEV)
                      if k % 3 == 0 else None)
    outs = pat.tv_prox_batched(zs, lams, 20, lowers=lowers)
    for k in range(count):
        ref = pat.tv_prox(zs[k], lams[k], 20, lower=lowers[k])
        assert torch.equal(outs[k], ref), k
