"""Pins of the FP64 k-space oracle against closed forms, invariants and brute force.

None of these re-types the oracle's formulas: each checks a consequence that
the paper or the mathematics fixes (the exact homogeneous solution, energy
conservation, the explicit DFT, the dense transpose, the per-mode recurrence,
linearity, reversibility, the lossless limit, the physical decay rate).
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import kspace as K


def _plan(inst, **kw):
    d = replace(inst.desc, **kw) if kw else inst.desc
    return K.make_plan(d, inst.c0, inst.rho0, inst.alpha0_db, inst.sensors)


def _kgrid(desc):
    """|k| from numpy's fftfreq (independent of the oracle's construction)."""
    ks = [2 * np.pi * np.fft.fftfreq(desc.n[j], desc.dx[j]) for j in range(desc.ndim)]
    mesh = np.meshgrid(*reversed(ks), indexing="ij")  # numpy axis order
    return mesh[::-1]  # physical order: kx, ky[, kz]


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("n", [(16, 12), (8, 8, 8)])
def test_p1_homogeneous_lossless_is_exact_cosine(n):
    """Homogeneous, lossless, periodic: p^n = F^-1[F(p0) cos(c|k| n dt)] (the
    k-space corrected leapfrog with the symmetric start is exact)."""
    inst = synth.small_instance(11, n, nt=25, lossy=False, hetero=False, pml_on=False)
    plan = _plan(inst)
    kk = _kgrid(inst.desc)
    kmag = np.sqrt(sum(k ** 2 for k in kk))
    P0 = np.fft.fftn(inst.p0.astype(np.float64))
    worst = 0.0
    for st in K.forward_states(plan, inst.p0):
        exact = np.fft.ifftn(P0 * np.cos(1500.0 * kmag * st.n * plan.dt)).real
        worst = max(worst, np.abs(st.p - exact).max() / np.abs(exact).max())
    assert worst < 1e-12


# ---------------------------------------------------------------- P2
@pytest.mark.parametrize("n", [(16, 16), (8, 8, 8)])
def test_p2_energy_invariant_heterogeneous_lossless(n):
    """Without absorption or PML, E_n = 1/2 sum p^2/(rho0 c0^2)
    + 1/2 sum_j sum rho0_sg u_j^{n-1/2} u_j^{n+1/2} is exactly conserved for
    any positive maps (the staggered pair satisfies (D+)^T = -D-)."""
    inst = synth.small_instance(12, n, nt=40, lossy=False, hetero=True, pml_on=False)
    plan = _plan(inst)
    st = K.ForwardState(plan, inst.p0)
    E = []
    for _ in range(35):
        p_n = st.p.copy()
        u_prev = [x.copy() for x in st.u]
        K.step(plan, st)
        e = 0.5 * np.sum(p_n ** 2 / (plan.rho0 * plan.c0 ** 2))
        e += 0.5 * sum(np.sum(plan.rho0_sg[j] * u_prev[j] * st.u[j]) for j in range(plan.ndim))
        E.append(e)
    E = np.array(E)
    assert np.abs(E - E[0]).max() / abs(E[0]) < 1e-12


def test_p2_energy_decays_with_pml():
    """With the PML on (lossless medium) energy can only leave the grid."""
    inst = synth.small_instance(13, (32, 32), nt=200, lossy=False, hetero=False, pml=6)
    plan = _plan(inst)
    st = K.ForwardState(plan, inst.p0)
    E = []
    for _ in range(150):
        p_n = st.p.copy()
        u_prev = [x.copy() for x in st.u]
        K.step(plan, st)
        e = 0.5 * np.sum(p_n ** 2 / (plan.rho0 * plan.c0 ** 2))
        e += 0.5 * sum(np.sum(plan.rho0_sg[j] * u_prev[j] * st.u[j]) for j in range(2))
        E.append(e)
    assert E[-1] < 0.5 * E[0]


# ---------------------------------------------------------------- P3
def _dft_matrix(n):
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


@pytest.mark.parametrize("n", [(8, 8), (16, 8), (8, 8, 8)])
def test_p3_spectral_operator_matches_explicit_dft(n):
    """The FFT plumbing of every spectral operator equals explicit O(N^2) DFT
    matrices (Kronecker product over axes), Nyquist bins included."""
    inst = synth.small_instance(14, n, nt=3, lossy=True, hetero=True)
    plan = _plan(inst)
    f = np.random.default_rng(0).standard_normal(plan.shape)
    Fm = np.ones((1, 1))
    for s in plan.shape:  # numpy axis order, last axis fastest
        Fm = np.kron(Fm, _dft_matrix(s))
    Fi = np.conj(Fm) / Fm.shape[0]
    for mult in plan.a + plan.b + [plan.L1, plan.L2]:
        m = np.broadcast_to(mult, plan.shape).ravel()
        ref = (Fi @ (m * (Fm @ f.ravel()))).real.reshape(plan.shape)
        got = K.spectral(mult, f)
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_p3_staggered_derivative_of_single_mode():
    """For f = cos(k x): D+ f = -k kappa sin(k (x + dx/2)) and
    D- f = -k kappa sin(k (x - dx/2)), kappa = sinc(c_ref |k| dt / 2):
    pins the shift direction and the k-space correction."""
    inst = synth.small_instance(15, (32, 16), nt=3, lossy=False, hetero=False)
    plan = _plan(inst)
    nx, dx = 32, inst.desc.dx[0]
    x = np.arange(nx) * dx
    for m in (1, 5, 11, 15):
        k = 2 * np.pi * m / (nx * dx)
        f = np.tile(np.cos(k * x), (16, 1))
        th = 1500.0 * k * plan.dt / 2
        kap = math.sin(th) / th
        dplus = K.spectral(plan.a[0], f)
        dminus = K.spectral(plan.b[0], f)
        assert np.allclose(dplus, np.tile(-k * kap * np.sin(k * (x + dx / 2)), (16, 1)), atol=1e-9 * k)
        assert np.allclose(dminus, np.tile(-k * kap * np.sin(k * (x - dx / 2)), (16, 1)), atol=1e-9 * k)
        # y derivative of an x-only field vanishes
        assert np.abs(K.spectral(plan.a[1], f)).max() < 1e-9 * k


def test_p3_nyquist_mode_is_real_and_antisymmetric():
    """The Nyquist mode (-1)^i is mapped to -pi kappa/dx (-1)^i by D+ and to
    +pi kappa/dx (-1)^i by D-: real multipliers, so (D+)^T = -D- holds there."""
    inst = synth.small_instance(16, (16, 8), nt=3, lossy=False, hetero=False)
    plan = _plan(inst)
    dx = inst.desc.dx[0]
    f = np.tile((-1.0) ** np.arange(16), (8, 1))
    th = 1500.0 * (np.pi / dx) * plan.dt / 2
    kap = math.sin(th) / th
    assert np.allclose(K.spectral(plan.a[0], f), -np.pi * kap / dx * f, rtol=1e-12)
    assert np.allclose(K.spectral(plan.b[0], f), np.pi * kap / dx * f, rtol=1e-12)


# ---------------------------------------------------------------- P4
def _dense(plan, shape, nt, ns):
    N = int(np.prod(shape))
    M = nt * ns
    A = np.zeros((M, N))
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1.0
        A[:, i] = K.forward(plan, e.reshape(shape)).ravel()
    AT = np.zeros((N, M))
    for i in range(M):
        e = np.zeros(M)
        e[i] = 1.0
        AT[:, i] = K.adjoint(plan, e.reshape(nt, ns)).ravel()
    return A, AT


@pytest.mark.parametrize("n,nt,ns", [((8, 8), 12, 5), ((8, 6), 9, 4), ((4, 4, 4), 6, 3)])
def test_p4_adjoint_is_dense_transpose(n, nt, ns):
    """Column-by-column dense H from `forward` and H^T from `adjoint`, with
    PML, absorption and heterogeneity, agree entrywise."""
    inst = synth.small_instance(17, n, nt=nt, ns=ns, pml=1 if len(n) == 3 else 2, lossy=True, hetero=True)
    plan = _plan(inst)
    A, AT = _dense(plan, plan.shape, nt, ns)
    assert np.abs(A.T - AT).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("n,nt,ns", [((8, 8), 12, 5), ((4, 4, 4), 6, 3)])
def test_p4_section3_density_pair_is_dense_transpose(n, nt, ns):
    """The forward started at section III's initial density (1 - eta L2)^-1
    p0 / c0^2 and its adjoint, with PML, absorption and heterogeneity, are
    exact transposes (dense, column by column); the start differs from the
    build's p0 / c0^2 (the option is applied)."""
    inst = synth.small_instance(19, n, nt=nt, ns=ns, pml=1 if len(n) == 3 else 2, lossy=True, hetero=True)
    plan = _plan(inst, section3_density=True)
    A, AT = _dense(plan, plan.shape, nt, ns)
    assert np.abs(A.T - AT).max() <= 1e-13 * np.abs(A).max()
    A0, _ = _dense(_plan(inst), plan.shape, nt, ns)
    assert np.abs(A - A0).max() > 1e-6 * np.abs(A).max()
    assert np.abs(A[:ns] - A0[:ns]).max() <= 1e-13 * np.abs(A).max()  # the first sample is p0 in both


def test_p4_nt1_is_sensor_transpose():
    """nt = 1: H = W and H^T = W^T."""
    inst = synth.small_instance(18, (8, 8), nt=1, ns=4)
    plan = _plan(inst)
    A, AT = _dense(plan, plan.shape, 1, 4)
    assert np.abs(A.T - AT).max() <= 1e-15


# ---------------------------------------------------------------- P5
def test_p5_dot_test_config2_geometry():
    """<H x, y> = <x, H^T y> at the 256^2 lossy heterogeneous geometry."""
    inst = synth.config2()
    plan = _plan(inst, nt=30)
    x = inst.p0.astype(np.float64)
    y = np.random.default_rng(5).standard_normal((30, inst.ns))
    Hx = K.forward(plan, x)
    HTy = K.adjoint(plan, y)
    lhs = float((Hx * y).sum())
    rhs = float((x * HTy).sum())
    scale = np.linalg.norm(Hx) * np.linalg.norm(y)
    assert abs(lhs - rhs) <= 1e-13 * scale


# ---------------------------------------------------------------- P6
@pytest.mark.parametrize("n", [(16, 16), (8, 8, 8)])
def test_p6_lossy_homogeneous_follows_modal_recurrence(n):
    """Homogeneous, lossy, periodic: every Fourier mode obeys the scalar
    recurrence S+ = S- + (dt/rho0) K^2 P, R+ = R - dt rho0 S+,
    P+ = c^2 [(1 - eta L2) R+ + tau L1 rho0 S+] with K = kappa|k|, built here
    from the paper's tau, eta (equation Twelve) and the power law."""
    inst = synth.small_instance(19, n, nt=30, lossy=True, hetero=False, pml_on=False)
    a0db = np.full(inst.p0.shape, 0.75, dtype=np.float32)
    inst = synth.Instance(inst.desc, inst.c0, inst.rho0, a0db, inst.sensors, inst.p0)
    plan = _plan(inst)
    c, rho0, y, dt = 1500.0, 1000.0, 1.5, plan.dt
    a0 = 0.75 * 100 * (1e-6 / (2 * np.pi)) ** y / 8.685889638065037  # Np/((rad/s)^y m)
    tau = -2 * a0 * c ** (y - 1)
    eta = 2 * a0 * c ** y * np.tan(np.pi * y / 2)
    kk = _kgrid(inst.desc)
    k = np.sqrt(sum(q ** 2 for q in kk))
    th = c * k * dt / 2
    kap = np.where(th == 0, 1.0, np.sin(th) / np.where(th == 0, 1, th))
    K2 = (kap * k) ** 2
    with np.errstate(divide="ignore"):
        L1 = np.where(k == 0, 0.0, k ** (y - 2))
        L2 = np.where(k == 0, 0.0, k ** (y - 1))
    P = np.fft.fftn(inst.p0.astype(np.float64))
    R = P / c ** 2
    S = -(dt / (2 * rho0)) * K2 * P
    worst = 0.0
    for st in K.forward_states(plan, inst.p0):
        if st.n > 0:
            S = S + (dt / rho0) * K2 * P
            R = R - dt * rho0 * S
            P = c ** 2 * ((1 - eta * L2) * R + tau * L1 * rho0 * S)
        ref = np.fft.ifftn(P).real
        worst = max(worst, np.abs(st.p - ref).max() / np.abs(ref).max())
    assert worst < 1e-12


# ---------------------------------------------------------------- P7
def test_p7_linearity():
    inst = synth.small_instance(20, (16, 16), nt=25, ns=6)
    plan = _plan(inst)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal((2,) + plan.shape)
    a, b = 0.7, -1.9
    lhs = K.forward(plan, a * x + b * y)
    rhs = a * K.forward(plan, x) + b * K.forward(plan, y)
    assert np.abs(lhs - rhs).max() <= 1e-12 * 25 * np.abs(lhs).max()


def test_p7_reversibility_lossless():
    """Lossless, no PML: each step can be undone (rho_j += dt rho0 D-_j u,
    p = c0^2 sum rho_j, u_j += dt/rho0_sg D+_j p), recovering p0 and the
    symmetric start after nt-1 forward steps."""
    inst = synth.small_instance(21, (16, 16), nt=40, lossy=False, hetero=True, pml_on=False)
    plan = _plan(inst)
    st = K.ForwardState(plan, inst.p0)
    u_init = [x.copy() for x in st.u]
    for _ in range(39):
        K.step(plan, st)
    u = [x.copy() for x in st.u]
    rho = [x.copy() for x in st.rho]
    for _ in range(39):
        for j in range(2):
            rho[j] = rho[j] + plan.dt * plan.rho0 * K.spectral(plan.b[j], u[j])
        p = plan.c0 ** 2 * sum(rho)
        for j in range(2):
            u[j] = u[j] + plan.dt / plan.rho0_sg[j] * K.spectral(plan.a[j], p)
    p0 = inst.p0.astype(np.float64)
    assert np.abs(p - p0).max() <= 1e-12 * 40 * np.abs(p0).max()
    for j in range(2):
        assert np.abs(u[j] - u_init[j]).max() <= 1e-10 * np.abs(u_init[j]).max()


# ---------------------------------------------------------------- P8
def test_p8_modal_decay_matches_power_law():
    """A single plane wave decays at the temporal rate alpha(omega) c with
    alpha = alpha0 omega^y (section II-A-2), within a few percent."""
    n, dx = 64, 1e-4
    desc = synth.GridDesc(ndim=2, n=(n, 4), dx=(dx, dx), origin=(0, 0), nt=2000, cfl=0.2, pml=False,
                          alpha_power=1.5)
    shape = desc.shape
    c0 = np.full(shape, 1500.0, np.float32)
    rho0 = np.full(shape, 1000.0, np.float32)
    a0db = np.full(shape, 3.0, np.float32)
    m = 8
    kx = 2 * np.pi * m / (n * dx)
    x = np.arange(n) * dx
    p0 = np.tile(np.cos(kx * x), (4, 1)).astype(np.float32)
    sens = np.array([[0.0, 0.0]])
    plan = K.make_plan(desc, c0, rho0, a0db, sens)
    amps = []
    for st in K.forward_states(plan, p0):
        amps.append(np.abs(np.fft.fft(st.p[0])[m]))
    amps = np.array(amps)
    t = np.arange(len(amps)) * plan.dt
    # envelope: local maxima of |P_m(t)|
    pk = [i for i in range(1, len(amps) - 1) if amps[i] >= amps[i - 1] and amps[i] >= amps[i + 1]]
    slope = np.polyfit(t[pk], np.log(amps[pk]), 1)[0]
    omega = 1500.0 * kx
    a0 = 3.0 * 100 * (1e-6 / (2 * np.pi)) ** 1.5 / 8.685889638065037
    expect = a0 * omega ** 1.5 * 1500.0
    assert abs(-slope - expect) / expect < 0.05


# ---------------------------------------------------------------- P9
def test_p9_zero_absorption_is_bitwise_lossless():
    inst = synth.small_instance(22, (16, 16), nt=20, ns=5, lossy=False)
    zero = np.zeros(inst.p0.shape, np.float32)
    pl = K.make_plan(inst.desc, inst.c0, inst.rho0, None, inst.sensors)
    pz = K.make_plan(inst.desc, inst.c0, inst.rho0, zero, inst.sensors)
    assert np.array_equal(K.forward(pl, inst.p0), K.forward(pz, inst.p0))
    h = np.random.default_rng(3).standard_normal((20, 5))
    assert np.array_equal(K.adjoint(pl, h), K.adjoint(pz, h))


# ---------------------------------------------------------------- sensors, PML, units
def test_sensor_interpolation_exact_for_affine_fields():
    """Bilinear/trilinear interpolation reproduces affine fields exactly,
    and a sensor on a node returns that node's value."""
    for n in [(16, 12), (8, 6, 5)]:
        inst = synth.small_instance(23, n, nt=1, ns=20)
        d = inst.desc
        idx, w = K.sensor_weights(d, inst.sensors)
        coeff = [0.3, -1.7, 2.2][: d.ndim]
        grids = np.indices(d.shape).astype(float)[::-1]
        field = 0.5 + sum(coeff[j] * grids[j] * d.dx[j] for j in range(d.ndim))
        got = (w * field.ravel()[idx]).sum(1)
        ref = 0.5 + inst.sensors @ np.array(coeff)
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)
    d = synth.small_instance(24, (8, 8), nt=1).desc
    on = np.array([[3 * d.dx[0], 5 * d.dx[1]], [7 * d.dx[0], 7 * d.dx[1]], [0.0, 0.0]])
    idx, w = K.sensor_weights(d, on)
    f = np.arange(64.0).reshape(8, 8)
    assert np.allclose((w * f.ravel()[idx]).sum(1), [f[5, 3], f[7, 7], f[0, 0]], rtol=0, atol=1e-12)


def test_sensor_outside_grid_rejected():
    d = synth.small_instance(25, (8, 8), nt=1).desc
    with pytest.raises(ValueError):
        K.sensor_weights(d, np.array([[8 * d.dx[0], 1e-4]]))
    with pytest.raises(ValueError):
        K.sensor_weights(d, np.array([[-1e-9, 1e-4]]))


def test_pml_profile_shape():
    """exp(-sigma dt/2) with sigma = alpha (c/dx) (depth/L)^4: 1 in the
    interior, strongest at the edges, symmetric between nodes, 2 Np/point."""
    n, L, alpha, c, dx, dt = 40, 8, 2.0, 1500.0, 1e-4, 2e-8
    q = K.pml_profile(n, L, alpha, c, dx, dt, False)
    qs = K.pml_profile(n, L, alpha, c, dx, dt, True)
    assert np.all(q[L:n - L] == 1.0)
    assert math.isclose(q[0], math.exp(-alpha * c / dx * dt / 2), rel_tol=1e-14)
    assert np.allclose(q, q[::-1], rtol=1e-14)
    # staggered point i+1/2 mirrors staggered point (n-2-i)+1/2
    assert np.allclose(qs[: n - 1], qs[: n - 1][::-1], rtol=1e-14)
    assert np.all(np.diff(q[: L + 1]) > 0)
    assert np.all(K.pml_profile(n, 0, alpha, c, dx, dt, True) == 1.0)


def test_absorption_unit_conversion():
    """1 dB/(MHz cm) at y = 1 is 100/8.6859 Np/m per MHz = 1.8323e-6 Np/((rad/s) m)."""
    v = K.db_to_neper(np.array(1.0), 1.0)
    assert math.isclose(float(v), 100 / 8.685889638065037 / (2 * math.pi * 1e6), rel_tol=1e-12)
    assert math.isclose(float(v), 1.8323e-6, rel_tol=1e-4)


# ---------------------------------------------------------------------------
# the spectral window of the p0 smoothing
# ---------------------------------------------------------------------------

def test_window_filter_by_brute_force_and_modes():
    """The window filter of the initial-pressure smoothing against an
    explicit circular convolution with the window's inverse DFT kernel
    (O(n^2) per axis, no FFT); a constant field is unchanged; a single
    Fourier mode is scaled by the window and the Nyquist mode removed."""
    rng = np.random.default_rng(17)
    f = rng.standard_normal((8, 12))
    out = K.window_filter(f)
    ref = f.copy()
    for ax, n in enumerate(f.shape):
        w = K.blackman_k(n)
        m = np.arange(n)
        kern = np.array([np.sum(w * np.cos(2 * np.pi * m * x / n)) / n for x in range(n)])  # real, even
        conv = np.zeros_like(ref)
        for x in range(n):
            for s in range(n):
                src = np.take(ref, [s], axis=ax)
                dst = [slice(None)] * ref.ndim
                dst[ax] = slice(x, x + 1)
                conv[tuple(dst)] += kern[(x - s) % n] * src
        ref = conv
    assert np.max(np.abs(out - ref)) < 1e-12
    assert np.max(np.abs(K.window_filter(np.full((8, 16), 1500.0)) - 1500.0)) < 1e-10
    x = np.arange(16)
    for mode in (0, 3, 8):
        g = np.cos(2 * np.pi * mode * x / 16)[None, :] * np.ones((4, 1))
        expect = K.blackman_k(16)[mode] * K.blackman_k(4)[0] * g
        assert np.max(np.abs(K.window_filter(g) - expect)) < 1e-12
    assert K.blackman_k(16)[8] == pytest.approx(0.0, abs=1e-15) and K.blackman_k(16)[0] == pytest.approx(1.0)


# ---------------------------------------------------------------------------
# smoothing of the initial pressure inside H and H^T (plan option)
# ---------------------------------------------------------------------------

def _conv_window(f):
    """Explicit circular convolution, axis by axis, with the inverse DFT of
    the window (a real, even kernel): O(n^2) per line, no FFT."""
    out = np.asarray(f, dtype=np.float64).copy()
    for ax, n in enumerate(out.shape):
        w = K.blackman_k(n)
        m = np.arange(n)
        kern = np.array([np.sum(w * np.cos(2 * np.pi * m * x / n)) / n for x in range(n)])
        mat = np.array([[kern[(x - s) % n] for s in range(n)] for x in range(n)])
        out = np.moveaxis(np.tensordot(mat, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    return out


@pytest.mark.parametrize("n,lossy", [((16, 12), True), ((16, 16), False), ((8, 8, 8), True)])
def test_smoothed_p0_forward_and_adjoint_by_convolution(n, lossy):
    """With the option, H p0 is the plain H applied to the explicitly
    convolved p0, and H^T h the convolved plain H^T h (also for the
    adjoint-then-discretize operator): the filter acts on the initial
    pressure alone, before every use of it (density, velocity start,
    sample 0), and the adjoint applies it last."""
    inst = synth.small_instance(23, n, nt=7, ns=5, pml=2, lossy=lossy, hetero=True)
    plain = _plan(inst)
    sm = _plan(inst, smooth_p0=True)
    assert sm.smooth_p0 and not plain.smooth_p0
    d_s = K.forward(sm, inst.p0)
    d_ref = K.forward(plain, _conv_window(inst.p0))
    assert np.max(np.abs(d_s - d_ref)) <= 1e-12 * np.max(np.abs(d_ref))
    assert np.max(np.abs(d_s - K.forward(plain, inst.p0))) > 1e-3 * np.max(np.abs(d_ref))  # not a no-op
    h = np.random.default_rng(5).standard_normal(d_s.shape)
    for op in (K.adjoint, K.adjoint_atd):
        a_s = op(sm, h)
        a_ref = _conv_window(op(plain, h))
        assert np.max(np.abs(a_s - a_ref)) <= 1e-12 * np.max(np.abs(a_ref))


@pytest.mark.parametrize("n,nt,ns", [((8, 8), 9, 4), ((4, 4, 4), 5, 3)])
def test_smoothed_p0_dense_transpose(n, nt, ns):
    """The filtered pair stays exactly transposed (S is symmetric): dense H
    and H^T built column by column agree entrywise."""
    inst = synth.small_instance(29, n, nt=nt, ns=ns, pml=1 if len(n) == 3 else 2, lossy=True, hetero=True)
    plan = _plan(inst, smooth_p0=True)
    A, AT = _dense(plan, plan.shape, nt, ns)
    assert np.abs(A.T - AT).max() <= 1e-13 * np.abs(A).max()


def test_smoothed_p0_single_mode_and_constant():
    """Periodic homogeneous grid: a single Fourier mode of p0 reaches the
    sensors scaled by the window's value at its bins; a constant p0 is left
    unchanged (the window is 1 at k = 0); the Nyquist mode is removed."""
    inst = synth.small_instance(31, (16, 16), nt=6, ns=4, pml=0, lossy=False, hetero=False)
    plain = _plan(inst, pml=False)
    sm = _plan(inst, pml=False, smooth_p0=True)
    x = np.arange(16)
    for mx, my in ((3, 0), (2, 5), (8, 1)):
        p0 = np.cos(2 * np.pi * mx * x / 16)[None, :] * np.cos(2 * np.pi * my * x / 16)[:, None]
        scale = K.blackman_k(16)[mx] * K.blackman_k(16)[my]
        ref = scale * K.forward(plain, p0)
        assert np.max(np.abs(K.forward(sm, p0) - ref)) <= 1e-12 * max(1.0, np.max(np.abs(K.forward(plain, p0))))
    c = np.full((16, 16), 0.7)
    assert np.max(np.abs(K.forward(sm, c) - K.forward(plain, c))) <= 1e-12


# ---------------------------------------------------------------------------
# PML: reflection and one-way attenuation of a plane pulse (section VI-A)
# ---------------------------------------------------------------------------

def _pml_pulse_energies(alpha, L=20, nx=256, ny=8, steps=(100, 450, 800)):
    """Interior sum of p^2 at the given steps for a plane Gaussian pulse
    (width 4 points, centred) in a homogeneous medium with a PML of L points
    and alpha nepers per point on the x ends only.  At step 100 the two
    halves travel in the interior; by 450 they are inside the layers (what
    the interior holds then is reflection); by 800 each has crossed its
    layer, wrapped around the periodic grid and crossed the opposite layer,
    and is back in the interior."""
    dx = 1e-4
    x = np.arange(nx)
    p0 = np.exp(-((x - nx / 2) / 4.0) ** 2)[None, :] * np.ones((ny, 1))
    desc = synth.GridDesc(ndim=2, n=(nx, ny), dx=(dx, dx), origin=(0.0, 0.0), nt=2, dt=0.0, cfl=0.3,
                          pml_size=(L, 0, 0), pml_alpha=alpha, alpha_power=1.5, pml=True)
    c0 = np.full((ny, nx), 1500.0, np.float32)
    op = K.make_plan(desc, c0, np.full((ny, nx), 1000.0, np.float32), None, np.array([[nx / 2 * dx, 4 * dx]]))
    out = {}
    for st in K.forward_states(op, p0, nsteps=max(steps)):
        if st.n in steps:
            out[st.n] = float((st.p[:, L:nx - L] ** 2).sum())
    return out


def test_pml_reflection_below_bound():
    """Normal incidence on 20 points at 2 Np per point: the reflected energy
    is far below 1 % of the incident one."""
    e = _pml_pulse_energies(2.0)
    assert e[450] / e[100] < 1e-6


@pytest.mark.parametrize("alpha", [0.05, 0.2])
def test_pml_one_way_attenuation_brackets_the_profile_integral(alpha):
    """A plane wave crossing a layer with sigma = alpha (c/dx)(depth/L)^4 loses
    the amplitude factor exp(-int sigma/c dx) = exp(-alpha L/5) in the
    continuum; on the grid the integral becomes a sum over the points
    crossed, which for this increasing profile lies between its midpoint sum
    (about L/5) and its right-end sum S = sum_{d=1..L} (d/L)^4.  The pulses
    cross two layers and their energy goes as the amplitude squared, so
    -ln(E_800 / E_100) / (4 alpha) must lie in [L/5 - 0.1, S + 0.1].  (A
    square profile gives L/3, a factor Q applied once per step half the
    rate, sigma per metre instead of per point a value 10^4 off.)"""
    L = 20
    e = _pml_pulse_energies(alpha, L=L)
    s_right = sum((d / L) ** 4 for d in range(1, L + 1))
    k = -math.log(e[800] / e[100]) / (4.0 * alpha)
    assert L / 5 - 0.1 <= k <= s_right + 0.1, (k, L / 5, s_right)


@pytest.mark.parametrize("m1,m2", [((1500.0, 1000.0), (1800.0, 1200.0)), ((1500.0, 1000.0), (1500.0, 1600.0)),
                                   ((1600.0, 1100.0), (1450.0, 950.0))])
def test_interface_reflection_matches_impedance_contrast(m1, m2):
    """Heterogeneous propagation: a plane pulse meeting, at normal incidence,
    the step from medium 1 to medium 2 (sound speed and density each change;
    one case changes the density alone, one lowers both) reflects the
    pressure amplitude R = (Z2 - Z1) / (Z2 + Z1), Z = rho c, so the reflected
    pulse carries R^2 of the incident sum of p^2 (both in medium 1).  The
    pulse's other half has by then left through the PML."""
    (c1, r1), (c2, r2) = m1, m2
    nx, ny, L, dx = 512, 8, 20, 1e-4
    x = np.arange(nx)
    c = (np.where(x < 300, c1, c2)[None, :] * np.ones((ny, 1))).astype(np.float32)
    rho = (np.where(x < 300, r1, r2)[None, :] * np.ones((ny, 1))).astype(np.float32)
    p0 = np.exp(-((x - 200) / 4.0) ** 2)[None, :] * np.ones((ny, 1))
    desc = synth.GridDesc(ndim=2, n=(nx, ny), dx=(dx, dx), origin=(0.0, 0.0), nt=2, dt=0.0, cfl=0.3,
                          pml_size=(L, 0, 0), pml_alpha=2.0, alpha_power=1.5, pml=True)
    op = K.make_plan(desc, c, rho, None, np.array([[200 * dx, 4 * dx]]))
    v1 = c1 * op.dt / dx                       # grid points per step in medium 1
    n_inc, n_ref = int(50 / v1), int(200 / v1)  # incident half at 250; reflection back at 200
    e = {}
    for st in K.forward_states(op, p0, nsteps=n_ref):
        if st.n == n_inc:
            e["inc"] = float((st.p[:, 201:299] ** 2).sum())
        if st.n == n_ref:
            e["ref"] = float((st.p[:, 101:299] ** 2).sum())
            e["left"] = float((st.p[:, L:101] ** 2).sum())
    z1, z2 = r1 * c1, r2 * c2
    R = (z2 - z1) / (z2 + z1)
    assert abs(e["ref"] / e["inc"] / (R * R) - 1.0) < 0.03, (e, R * R)
    assert e["left"] < 1e-9 * e["inc"]
