"""FP64 reference of the forward operator H and its exact transpose H^T.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain CPU oracle against
which the GPU library is checked.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the GPU library never
does, and this module imports nothing from it.

What it computes
----------------
The forward model is the lossy first-order acoustic system of section II-A:
the equation of motion, the equation of continuity and the equation of state
with two fractional-Laplacian terms (equations mom, mass, state), with the
coefficients tau and eta of equation Twelve and the initial conditions of
equation initial.  The paper solves it with a k-space pseudospectral scheme
(section I and II-A; the scheme itself is not written out).  The discrete
scheme used here is the standard first-order k-space scheme on a staggered
grid:

* spatial derivatives are taken in the Fourier domain with the k-space
  correction kappa = sinc(c_ref |k| dt / 2) and a half-cell shift,
  a_j = i k_j kappa exp(+i k_j dx_j / 2) (to staggered points) and
  b_j = i k_j kappa exp(-i k_j dx_j / 2) (back to nodes);
* the fractional Laplacians are |k|^(y-2) and |k|^(y-1), zero at k = 0;
* the density is split per axis, rho = sum_j rho_j, so that a per-axis PML
  can act on each part (PML inside the grid, fourth-power profile,
  pml_alpha nepers per grid point, section VI-A);
* velocities live at t = (n + 1/2) dt, pressure and density at t = n dt;
  u(0) = 0 is imposed in the mean by a symmetric half-step start.

The sensor operator is linear (bilinear in 2D, trilinear in 3D)
interpolation of the pressure to each detector, sampled at every time step
including t = 0 (section III, operator M w; section VI-A).

The adjoint is the exact transpose of that discrete forward map (the
discrete counterpart of the time-reversed adjoint system moma/massa/statea
with the data injected as a mass source and the output rho*(T)/rho0 of
equation adjj); its defining property is equation adj2, the dot-product
identity, which the tests pin.

Initial density.  By default the lossy start is rho_j(0) = p0 / (d c0^2).
With ``section3_density`` the start follows section III's equation of state
at t = 0 instead, c0^2 (1 - eta L2) rho(0) = p0, solved by a fixed-point
iteration (``solve_dispersion``); the paper's adjoint-then-discretize system
is the transpose of that forward up to O(dt).

Array layout: numpy C order with x fastest, shape (ny, nx) or (nz, ny, nx).
Physical axis j (x=0, y=1, z=2) is numpy axis ndim-1-j.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np
import scipy.fft as sfft

__all__ = ["OraclePlan", "make_plan", "forward", "adjoint", "forward_states", "db_to_neper",
           "sensor_weights", "pml_profile", "solve_dispersion", "WORKERS"]

#: threads handed to scipy.fft (set by callers that time the oracle)
WORKERS = 1


def _fft(f):
    return sfft.fftn(f, workers=WORKERS)


def _ifft(F):
    return sfft.ifftn(F, workers=WORKERS)


def db_to_neper(alpha0_db: np.ndarray, y: float) -> np.ndarray:
    """Absorption coefficient from dB/(MHz^y cm) to Np/((rad/s)^y m).

    alpha(f) = alpha0_db * f_MHz^y dB/cm with f_MHz = omega / (2 pi 1e6);
    one neper is 20 log10(e) dB and one centimetre is 1e-2 m (section II-A-2,
    power law alpha = alpha0 w^y with w the angular frequency)."""
    return alpha0_db * 100.0 * (1e-6 / (2.0 * math.pi)) ** y / (20.0 * math.log10(math.e))


def pml_profile(n: int, L: int, alpha: float, c_ref: float, dx: float, dt: float,
                staggered: bool) -> np.ndarray:
    """Per-axis PML damping factor exp(-sigma dt / 2) on nodes or staggered points.

    The layer occupies the first and last L points of the axis (inside the
    grid).  At position s (s = i on nodes, i + 1/2 on staggered points) the
    depth into the layer is L - s on the low side and s - (n - 1 - L) on the
    high side; sigma = alpha (c_ref / dx) (depth / L)^4, i.e. alpha nepers per
    grid point at full depth (section VI-A: 2 Np per point)."""
    if L <= 0:
        return np.ones(n)
    s = np.arange(n, dtype=np.float64) + (0.5 if staggered else 0.0)
    depth = np.zeros(n)
    lo = s < L
    depth[lo] = L - s[lo]
    hi = s > (n - 1 - L)
    depth[hi] = s[hi] - (n - 1 - L)
    sigma = alpha * (c_ref / dx) * (depth / L) ** 4
    return np.exp(-sigma * dt / 2.0)


def sensor_weights(desc, sensors: np.ndarray):
    """Linear-interpolation taps of each sensor: (flat indices, weights).

    Grid coordinate g_j = (r_j - origin_j) / dx_j must lie in [0, n_j - 1];
    the lower node is min(floor(g_j), n_j - 2) so a sensor on the last node
    uses weight 1 there.  Returns arrays of shape (ns, 2^ndim)."""
    nd = desc.ndim
    sensors = np.asarray(sensors, dtype=np.float64).reshape(-1, nd)
    ns = sensors.shape[0]
    lo = np.zeros((ns, nd), dtype=np.int64)
    fr = np.zeros((ns, nd))
    for j in range(nd):
        g = (sensors[:, j] - desc.origin[j]) / desc.dx[j]
        if np.any(g < 0) or np.any(g > desc.n[j] - 1):
            raise ValueError("sensor outside the grid")
        i0 = np.minimum(np.floor(g), desc.n[j] - 2).astype(np.int64)
        lo[:, j] = i0
        fr[:, j] = g - i0
    ntap = 2 ** nd
    idx = np.zeros((ns, ntap), dtype=np.int64)
    w = np.ones((ns, ntap))
    strides = [int(np.prod(desc.n[:j])) for j in range(nd)]  # x stride 1, y stride nx, ...
    for t in range(ntap):
        for j in range(nd):
            bit = (t >> j) & 1
            idx[:, t] += (lo[:, j] + bit) * strides[j]
            w[:, t] *= fr[:, j] if bit else (1.0 - fr[:, j])
    return idx, w


@dataclass
class OraclePlan:
    desc: object
    ndim: int
    shape: tuple
    dt: float
    c_ref: float
    lossy: bool
    c0: np.ndarray
    rho0: np.ndarray
    c0sq: np.ndarray
    tau: Optional[np.ndarray]
    eta: Optional[np.ndarray]
    rho0_sg: List[np.ndarray]
    a: List[np.ndarray]          # a_j multipliers (to staggered points)
    b: List[np.ndarray]          # b_j multipliers (to nodes)
    L1: Optional[np.ndarray]     # |k|^(y-2)
    L2: Optional[np.ndarray]     # |k|^(y-1)
    Q: List[np.ndarray]          # node PML factor per axis, broadcastable
    Qsg: List[np.ndarray]        # staggered PML factor per axis
    idx: np.ndarray
    w: np.ndarray
    nt: int
    smooth_p0: bool = False      # S in H = H0 S and H^T = S H0^T (``smooth_initial``)
    section3_density: bool = False  # initial density from section III's t = 0 relation


def _bcast(v: np.ndarray, ndim: int, j: int) -> np.ndarray:
    sh = [1] * ndim
    sh[ndim - 1 - j] = v.size
    return v.reshape(sh)


def blackman_k(n: int) -> np.ndarray:
    """The Blackman window over the n wavenumber bins of one axis, centred
    on the zero wavenumber: 0.42 + 0.5 cos(2 pi m / n) + 0.08 cos(4 pi m / n)
    (1 at m = 0, 0 at the Nyquist bin m = n / 2)."""
    m = np.arange(n)
    return 0.42 + 0.5 * np.cos(2.0 * math.pi * m / n) + 0.08 * np.cos(4.0 * math.pi * m / n)


def window_filter(f: np.ndarray) -> np.ndarray:
    """The field's spectrum times the product over the axes of ``blackman_k``,
    back-transformed (real part)."""
    f = np.asarray(f, dtype=np.float64)
    W = np.ones(f.shape)
    for ax, n in enumerate(f.shape):
        sh = [1] * f.ndim
        sh[ax] = n
        W = W * blackman_k(n).reshape(sh)
    return np.fft.ifftn(W * np.fft.fftn(f)).real


def smooth_initial(f: np.ndarray) -> np.ndarray:
    """The smoothing S of the initial pressure (section VI-A: the forward
    model filters the high frequencies of p0 with a self-adjoint operator,
    which the adjoint then includes).  Reading (the paper names neither the
    filter nor its cut-off): ``window_filter``, a spectral window real and
    even in k, so that S is a real symmetric matrix and the operator pair
    stays exactly transposed: H = H0 S, H^T = S H0^T."""
    return window_filter(f)


def make_plan(desc, c0, rho0, alpha0_db, sensors) -> OraclePlan:
    """Derive every coefficient of the scheme in FP64 from the float32 inputs."""
    nd = desc.ndim
    c0 = np.asarray(c0, dtype=np.float64)
    rho0 = np.asarray(rho0, dtype=np.float64)
    shape = c0.shape
    assert shape == tuple(reversed(desc.n[:nd]))
    c_ref = float(c0.max())
    dt = float(desc.dt) if desc.dt > 0 else float(desc.cfl) * min(desc.dx[:nd]) / c_ref

    # wavenumbers: k_j[m] = 2 pi m~ / (n_j dx_j), m~ = m (m < n/2) else m - n
    k = []
    for j in range(nd):
        n = desc.n[j]
        m = np.arange(n)
        mt = np.where(m < n // 2, m, m - n)
        k.append(_bcast(2.0 * math.pi * mt / (n * desc.dx[j]), nd, j))
    kmag = np.sqrt(sum(kj ** 2 for kj in k))
    arg = c_ref * kmag * dt / 2.0
    kappa = np.where(arg == 0, 1.0, np.sin(arg) / np.where(arg == 0, 1.0, arg))
    a = [1j * k[j] * kappa * np.exp(1j * k[j] * desc.dx[j] / 2.0) for j in range(nd)]
    b = [1j * k[j] * kappa * np.exp(-1j * k[j] * desc.dx[j] / 2.0) for j in range(nd)]

    lossy = alpha0_db is not None
    y = float(desc.alpha_power)
    if lossy:
        a0 = db_to_neper(np.asarray(alpha0_db, dtype=np.float64), y)
        tau = -2.0 * a0 * c0 ** (y - 1.0)                       # equation Twelve
        eta = 2.0 * a0 * c0 ** y * math.tan(math.pi * y / 2.0)  # equation Twelve
        safe = np.where(kmag == 0, 1.0, kmag)
        L1 = np.where(kmag == 0, 0.0, safe ** (y - 2.0))
        L2 = np.where(kmag == 0, 0.0, safe ** (y - 1.0))
    else:
        tau = eta = L1 = L2 = None

    # ambient density on the staggered points: mean of the two neighbours,
    # the last index keeps its own value
    rho0_sg = []
    for j in range(nd):
        ax = nd - 1 - j
        nxt = np.concatenate([np.take(rho0, np.arange(1, shape[ax]), axis=ax),
                              np.take(rho0, [shape[ax] - 1], axis=ax)], axis=ax)
        rho0_sg.append(0.5 * (rho0 + nxt))

    Q, Qsg = [], []
    for j in range(nd):
        L = int(desc.pml_size[j]) if desc.pml else 0
        Q.append(_bcast(pml_profile(desc.n[j], L, desc.pml_alpha, c_ref, desc.dx[j], dt, False), nd, j))
        Qsg.append(_bcast(pml_profile(desc.n[j], L, desc.pml_alpha, c_ref, desc.dx[j], dt, True), nd, j))

    idx, w = sensor_weights(desc, sensors)
    return OraclePlan(desc=desc, ndim=nd, shape=shape, dt=dt, c_ref=c_ref, lossy=lossy, c0=c0,
                      rho0=rho0, c0sq=c0 ** 2, tau=tau, eta=eta, rho0_sg=rho0_sg, a=a, b=b, L1=L1,
                      L2=L2, Q=Q, Qsg=Qsg, idx=idx, w=w, nt=int(desc.nt),
                      smooth_p0=bool(getattr(desc, "smooth_p0", False)),
                      section3_density=bool(getattr(desc, "section3_density", False)))


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def spectral(mult: np.ndarray, f: np.ndarray) -> np.ndarray:
    """F^-1 [ mult * F f ] for a real field f (the real part is kept; every
    multiplier used here is Hermitian, so the imaginary part is rounding)."""
    return _ifft(mult * _fft(f)).real


def gather(plan: OraclePlan, p: np.ndarray) -> np.ndarray:
    """Sensor samples sum_q W[s, q] p[q]."""
    return (plan.w * p.ravel()[plan.idx]).sum(axis=1)


def scatter(plan: OraclePlan, h: np.ndarray) -> np.ndarray:
    """Transposed sensor operator W^T h (accumulated in FP64)."""
    out = np.zeros(int(np.prod(plan.shape)))
    np.add.at(out, plan.idx.ravel(), (plan.w * np.asarray(h, np.float64)[:, None]).ravel())
    return out.reshape(plan.shape)


def solve_dispersion(plan: OraclePlan, b: np.ndarray, transpose: bool = False) -> np.ndarray:
    """x = (I - eta L2)^-1 b, or with transpose (I - L2 eta)^-1 b (L2 is real
    and symmetric, eta diagonal), by the fixed-point iteration
    x <- b + eta L2 x (resp. b + L2 (eta x)), iterated to a relative change
    below 1e-15.  It converges because |eta| |k|^(y-1) << 1 on any grid the
    stability bound admits (1e-2 on the test grids); a slower contraction
    raises."""
    b = np.asarray(b, dtype=np.float64)
    x = b.copy()
    prev = np.inf
    for _ in range(200):
        ex = plan.eta * spectral(plan.L2, x) if not transpose else spectral(plan.L2, plan.eta * x)
        nx = b + ex
        d = float(np.linalg.norm(nx - x))
        x = nx
        if d <= 1e-15 * float(np.linalg.norm(x)):
            return x
        if d > 0.5 * prev:
            raise ValueError("dispersion solve does not contract")
        prev = d
    raise ValueError("dispersion solve did not converge")


# --------------------------------------------------------------------------
# forward
# --------------------------------------------------------------------------

class ForwardState:
    """Fields of the forward scheme between two steps: u_j at t-(1/2)dt...
    after a step u_j holds the newest half-step velocity and p, rho_j the
    newest full-step values."""

    def __init__(self, plan: OraclePlan, p0: np.ndarray):
        nd = plan.ndim
        p0 = np.asarray(p0, dtype=np.float64)
        if plan.smooth_p0:
            p0 = smooth_initial(p0)                 # the model's initial pressure is S p0
        P = _fft(p0)
        self.n = 0
        self.p = p0.copy()
        if plan.section3_density and plan.lossy:
            # section III's t = 0 relation c0^2 (1 - eta L2) rho(0) = p0 (the tau
            # term vanishes with u(0) = 0), split equally over the axes
            r0 = solve_dispersion(plan, p0 / plan.c0sq)
            self.rho = [r0 / nd for _ in range(nd)]
        else:
            # rho_j = p0 / (d c0^2): the split densities add up to p0 / c0^2
            self.rho = [p0 / (nd * plan.c0sq) for _ in range(nd)]
        # symmetric start: u_j(-dt/2) = (dt/2) (1/rho0_sg) D+_j p0, so that the
        # first update gives u_j(+dt/2) = -u_j(-dt/2) (u = 0 at t = 0 in the mean)
        self.u = [(plan.dt / 2.0) / plan.rho0_sg[j] * _ifft(plan.a[j] * P).real for j in range(nd)]


def step(plan: OraclePlan, st: ForwardState) -> None:
    """Advance the state by one time step (p^n -> p^{n+1})."""
    nd, dt = plan.ndim, plan.dt
    P = _fft(st.p)
    for j in range(nd):
        dp = _ifft(plan.a[j] * P).real                         # grad p at staggered points
        st.u[j] = plan.Qsg[j] * (plan.Qsg[j] * st.u[j] - dt / plan.rho0_sg[j] * dp)  # eq. mom
    g = [spectral(plan.b[j], st.u[j]) for j in range(nd)]      # components of div u
    for j in range(nd):
        st.rho[j] = plan.Q[j] * (plan.Q[j] * st.rho[j] - dt * plan.rho0 * g[j])     # eq. mass
    rho = sum(st.rho)
    if plan.lossy:
        # eq. state: -tau d/dt (-lap)^(y/2-1) rho = +tau (-lap)^(y/2-1) (rho0 div u)
        div = sum(g)
        A1 = spectral(plan.L1, plan.rho0 * div)
        A2 = spectral(plan.L2, rho)
        st.p = plan.c0sq * (rho + plan.tau * A1 - plan.eta * A2)
    else:
        st.p = plan.c0sq * rho                                  # eq. estate
    st.n += 1


def forward_states(plan: OraclePlan, p0: np.ndarray, nsteps: Optional[int] = None):
    """Yield the state after 0, 1, ..., nsteps steps (default nt - 1)."""
    st = ForwardState(plan, p0)
    yield st
    for _ in range(plan.nt - 1 if nsteps is None else nsteps):
        step(plan, st)
        yield st


def forward(plan: OraclePlan, p0: np.ndarray, callback: Optional[Callable] = None) -> np.ndarray:
    """H p0: sensor data of shape (nt, ns), sample n at t = n dt."""
    data = np.empty((plan.nt, plan.idx.shape[0]))
    for st in forward_states(plan, p0):
        data[st.n] = gather(plan, st.p)
        if callback is not None:
            callback(st)
    return data


# --------------------------------------------------------------------------
# adjoint (exact transpose of `forward`)
# --------------------------------------------------------------------------

def adjoint(plan: OraclePlan, h: np.ndarray, nsteps_done: Optional[Callable] = None) -> np.ndarray:
    """H^T h for data h of shape (nt, ns): an image of the grid's shape.

    Each forward step is transposed in reverse order.  With q = c0^2 pbar the
    transposed equation of state feeds rho_j-bar with q - L2(eta q) and the
    divergence with rho0 L1(tau q): the fractional Laplacians act after tau
    and eta and rho0 after them, the order of equation statea."""
    nd, dt = plan.ndim, plan.dt
    h = np.asarray(h, dtype=np.float64)
    nt = plan.nt
    pbar = scatter(plan, h[nt - 1])
    rbar = [np.zeros(plan.shape) for _ in range(nd)]
    ubar = [np.zeros(plan.shape) for _ in range(nd)]
    for n in range(nt - 2, -1, -1):
        q = plan.c0sq * pbar
        if plan.lossy:
            A2 = spectral(plan.L2, plan.eta * q)
            gsh = plan.rho0 * spectral(plan.L1, plan.tau * q)
        else:
            A2 = 0.0
            gsh = 0.0
        for j in range(nd):
            rbar[j] = rbar[j] + (q - A2)
        for j in range(nd):
            gj = gsh - dt * plan.rho0 * plan.Q[j] * rbar[j]
            rbar[j] = plan.Q[j] * plan.Q[j] * rbar[j]
            ubar[j] = ubar[j] - spectral(plan.a[j], gj)
        s = sum(spectral(plan.b[j], (1.0 / plan.rho0_sg[j]) * plan.Qsg[j] * ubar[j]) for j in range(nd))
        pbar = scatter(plan, h[n]) + dt * s
        for j in range(nd):
            ubar[j] = plan.Qsg[j] * plan.Qsg[j] * ubar[j]
        if nsteps_done is not None:
            nsteps_done(n)
    if plan.section3_density and plan.lossy:
        # transpose of rho_j(0) = (1 - eta L2)^-1 (p0 / c0^2) / d
        img = pbar + solve_dispersion(plan, sum(rbar) / nd, transpose=True) / plan.c0sq
    else:
        img = pbar + sum(rbar) / (nd * plan.c0sq)
    img = img - (dt / 2.0) * sum(spectral(plan.b[j], ubar[j] / plan.rho0_sg[j]) for j in range(nd))
    return smooth_initial(img) if plan.smooth_p0 else img     # S^T = S


# --------------------------------------------------------------------------
# adjoint-then-discretize (the paper's adjoint system, for comparison)
# --------------------------------------------------------------------------

def adjoint_atd(plan: OraclePlan, h: np.ndarray) -> np.ndarray:
    """The adjoint system of section III (eq. moma, massa, statea with eq.
    initial2, image rho*(T) / rho0 by eq. adjj) discretized with the scheme
    of ``forward`` -- the paper's "adjoint-then-discretize" operator, not
    the exact transpose (``adjoint``).  For data vanishing at the first and
    last samples it equals the transpose in a homogeneous lossless or
    absorption-only medium without PML and converges to it in dt otherwise
    (dispersion and data inside the PML aside); the end samples differ.

    Readings (the paper gives the continuous system only):
    * the fields are scaled by dV/dt so that the data enter without grid
      factors: over the adjoint step from t_n to t_n+1 (forward times T - t)
      the density gains rho0 sigma, sigma = (W^T h[N-1-n] + W^T h[N-2-n]) / 2
      (trapezoid rule on the time-reversed data), split equally over the d
      axis components and inside the PML factor like the divergence term;
    * the time derivative in eq. statea is taken through eq. massa:
      d/dt (c0^2 / rho0 rho*) = c0^2 (sigma / dt - sum_j g_j);
    * leapfrog as the forward: u* at half steps from p* = 0, u* = 0, rho* = 0;
    * p* = c0^2 rho* - rho0 L1[tau c0^2 (sigma / dt - div u*)]
           - rho0 L2[eta c0^2 / rho0 rho*], the operators in statea's order.
    """
    nd, dt = plan.ndim, plan.dt
    h = np.asarray(h, dtype=np.float64)
    nt = plan.nt
    u = [np.zeros(plan.shape) for _ in range(nd)]
    rho = [np.zeros(plan.shape) for _ in range(nd)]
    p = np.zeros(plan.shape)
    for n in range(nt - 1):
        sigma = 0.5 * (scatter(plan, h[nt - 1 - n]) + scatter(plan, h[nt - 2 - n]))
        P = _fft(p)
        for j in range(nd):
            dp = _ifft(plan.a[j] * P).real
            u[j] = plan.Qsg[j] * (plan.Qsg[j] * u[j] - dt / plan.rho0_sg[j] * dp)        # eq. moma
        g = [spectral(plan.b[j], u[j]) for j in range(nd)]
        for j in range(nd):
            rho[j] = plan.Q[j] * (plan.Q[j] * rho[j] + plan.rho0 * (sigma / nd - dt * g[j]))  # eq. massa
        rs = sum(rho)
        if plan.lossy:
            A1 = spectral(plan.L1, plan.tau * plan.c0sq * (sigma / dt - sum(g)))
            A2 = spectral(plan.L2, plan.eta * plan.c0sq / plan.rho0 * rs)
            p = plan.c0sq * rs - plan.rho0 * (A1 + A2)                                      # eq. statea
        else:
            p = plan.c0sq * rs
    img = sum(rho) / plan.rho0                                                              # eq. adjj
    return smooth_initial(img) if plan.smooth_p0 else img
