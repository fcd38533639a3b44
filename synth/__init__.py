"""Seeded synthetic workloads for the photoacoustic k-space solver.

This module only *describes and draws inputs*: grid descriptors, medium maps
(sound speed, ambient density, absorption coefficient), initial pressure
phantoms and sensor positions.  It contains none of the solver's arithmetic
(no wavenumbers, no operators, no coefficient conversion), so both the FP64
oracle and the GPU library can consume what it produces without sharing any
method code.

Every array is drawn in float64 from ``numpy.random.default_rng(seed)`` and
rounded once to float32; the same float32 arrays are handed to the oracle
(upcast) and to the GPU.

Arrays are row-major with x fastest: shape ``(ny, nx)`` in 2D and
``(nz, ny, nx)`` in 3D.  Descriptors list per-axis quantities in physical
axis order ``(x, y[, z])``.

The paper measured on its own vessel phantom and layered tissue maps (section
VI, figures 1, 2, 6, 7), which are not available; these generators stand in
for them with the paper's value ranges: sound speed 1450-1730 m/s, density
950-1150 kg/m^3, absorption 0.75 dB/(MHz^y cm) with y = 1.5, and vessel-like
initial pressure of amplitude up to 1 (section VI-A).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "GridDesc", "Instance", "rng_for", "circle_sensors", "half_circle_sensors",
    "plane_sensors", "blob_medium", "disc_phantom", "vessel_phantom",
    "ellipsoid_phantom", "config1", "config2", "config3", "config4", "config5",
    "small_instance", "CONFIG_NAMES",
]

CONFIG_NAMES = {
    1: "2D 64^2 homogeneous lossless, Nt=300, 64 circle sensors",
    2: "2D 256^2 heterogeneous lossy, Nt=1200, 256 half-circle sensors",
    3: "2D MG pair 512^2 (Nt=2400) + 256^2 (Nt=1200), 256 half-circle sensors",
    4: "batch of 48 2D instances: 16 x 128^2/600, 16 x 256^2/1200, 16 x 512^2/2400",
    5: "3D 128^3 heterogeneous lossy, Nt=800, 128x128 planar sensor",
}


@dataclass(frozen=True)
class GridDesc:
    """Computational grid and time axis of one solver instance.

    ``n``, ``dx``, ``origin`` and ``pml_size`` are given per physical axis
    (x, y[, z]).  Node ``i`` along axis ``j`` sits at ``origin[j] + i*dx[j]``.
    ``nt`` samples are recorded at ``t = n*dt`` for ``n = 0..nt-1``; a
    non-positive ``dt`` asks the solver to derive it from ``cfl``.
    The PML lies inside the grid; ``pml=False`` switches it off (periodic).
    """

    ndim: int
    n: Tuple[int, ...]
    dx: Tuple[float, ...]
    origin: Tuple[float, ...]
    nt: int
    dt: float = 0.0
    cfl: float = 0.3
    pml_size: Tuple[int, ...] = (0, 0, 0)
    pml_alpha: float = 2.0
    alpha_power: float = 1.5
    pml: bool = True
    smooth_p0: bool = False  # smooth the initial pressure inside H (and H^T)
    section3_density: bool = False  # initial density from section III's t = 0 relation

    @property
    def shape(self) -> Tuple[int, ...]:
        """numpy array shape (reversed axis order, x fastest)."""
        return tuple(int(v) for v in reversed(self.n[: self.ndim]))

    @property
    def npoints(self) -> int:
        return int(np.prod(self.n[: self.ndim]))


@dataclass
class Instance:
    """One synthetic forward/adjoint problem: descriptor + float32 inputs."""

    desc: GridDesc
    c0: np.ndarray
    rho0: np.ndarray
    alpha0_db: Optional[np.ndarray]
    sensors: np.ndarray  # (ns, ndim) float64 physical positions [m]
    p0: np.ndarray
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def ns(self) -> int:
        return int(self.sensors.shape[0])


def rng_for(config: int, instance: int = 0) -> np.random.Generator:
    """The seeding rule: seed = 1000*config + instance."""
    return np.random.default_rng(1000 * int(config) + int(instance))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _coords(shape: Sequence[int]) -> List[np.ndarray]:
    """Index grids in physical axis order (ix, iy[, iz]) broadcast to shape."""
    nd = len(shape)
    idx = np.indices(shape, dtype=np.float64)
    return [idx[nd - 1 - j] for j in range(nd)]


# --------------------------------------------------------------------------
# sensors
# --------------------------------------------------------------------------

def circle_sensors(n: int, dx: float, origin: float, radius_pts: float, count: int) -> np.ndarray:
    """Full circle around the grid centre, theta_s = 2*pi*s/count."""
    c = origin + (n / 2) * dx
    th = 2.0 * np.pi * np.arange(count) / count
    return np.stack([c + radius_pts * dx * np.cos(th), c + radius_pts * dx * np.sin(th)], axis=1)


def half_circle_sensors(n: int, dx: float, origin: float, radius_pts: float, count: int) -> np.ndarray:
    """Left half of a circle about the grid centre (section VI-A geometry):
    theta_s = pi/2 + pi*s/(count-1)."""
    c = origin + (n / 2) * dx
    th = np.pi / 2 + np.pi * np.arange(count) / max(count - 1, 1)
    return np.stack([c + radius_pts * dx * np.cos(th), c + radius_pts * dx * np.sin(th)], axis=1)


def plane_sensors(nx: int, ny: int, dx: Sequence[float], origin: Sequence[float], z_index: int) -> np.ndarray:
    """Every (x, y) node of the plane z = z_index (planar detector)."""
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([
        origin[0] + ix.ravel() * dx[0],
        origin[1] + iy.ravel() * dx[1],
        np.full(ix.size, origin[2] + z_index * dx[2]),
    ], axis=1)
    return pos


# --------------------------------------------------------------------------
# media
# --------------------------------------------------------------------------

def _blob_params(rng, k: int, nd: int, lo: Sequence[float], hi: Sequence[float], amp: float,
                 sig_lo: float, sig_hi: float):
    centres = np.stack([rng.uniform(lo[j], hi[j], size=k) for j in range(nd)], axis=1)
    amps = rng.uniform(-amp, amp, size=k)
    sig = rng.uniform(sig_lo, sig_hi, size=k)
    return centres, amps, sig


def _blob_field(shape, centres_idx, amps, sig_idx, offset_idx=0.0, scale=1.0):
    """Sum of Gaussian blobs evaluated at index coordinates i*scale + offset
    (all lengths in units of the generating grid's points)."""
    xs = _coords(shape)
    out = np.zeros(shape)
    for c, a, s in zip(centres_idx, amps, sig_idx):
        r2 = np.zeros(shape)
        for j, x in enumerate(xs):
            r2 += (x * scale + offset_idx - c[j]) ** 2
        out += a * np.exp(-r2 / (2.0 * s * s))
    return out


def blob_medium(rng, shape, pml: int, *, c_amp=100.0, rho_amp=0.1, k=6, sig=(10.0, 30.0),
                c_clip=(1450.0, 1730.0), rho_clip=0.1, lossy=True, hetero_rho=True,
                levels=((1.0, 0.0),)):
    """Heterogeneous medium: c = 1500 + sum of k Gaussian blobs (+-c_amp m/s),
    rho = 1000*(1 + sum of k blobs (+-rho_amp)), clipped; alpha0 = 0.75.

    The blobs are continuous functions of position, drawn once; ``levels``
    lists ``(scale, offset)`` pairs mapping each requested grid's indices to
    generating-grid indices (a cell-centred coarse grid uses (2, 0.5)), so the
    same physical medium is sampled on every level.  Returns one tuple
    ``(c0, rho0, alpha0)`` per level (float32).
    """
    nd = len(shape)
    n_phys = list(reversed(shape))
    lo = [pml] * nd
    hi = [n_phys[j] - 1 - pml for j in range(nd)]
    cc, ca, cs = _blob_params(rng, k, nd, lo, hi, c_amp, *sig)
    rc, ra, rs = _blob_params(rng, k, nd, lo, hi, rho_amp, *sig)
    out = []
    for scale, offset in levels:
        lshape = tuple(int(round(s / scale)) for s in shape)
        c = 1500.0 + _blob_field(lshape, cc, ca, cs, offset, scale)
        c = np.clip(c, *c_clip)
        if hetero_rho:
            rho = 1000.0 * (1.0 + np.clip(_blob_field(lshape, rc, ra, rs, offset, scale),
                                          -rho_clip, rho_clip))
        else:
            rho = np.full(lshape, 1000.0)
        a0 = np.full(lshape, 0.75) if lossy else None
        out.append((_f32(c), _f32(rho), None if a0 is None else _f32(a0)))
    return out


# --------------------------------------------------------------------------
# phantoms (initial pressure)
# --------------------------------------------------------------------------

def disc_phantom(rng, shape, *, count=5, centre_radius=20.0, r_lo=2.0, r_hi=8.0):
    """Sum of `count` discs: centres uniform within `centre_radius` points of
    the grid centre, radii U[r_lo, r_hi] points, amplitudes U[0, 1]."""
    ny, nx = shape
    xs, ys = _coords(shape)
    out = np.zeros(shape)
    for _ in range(count):
        rr = centre_radius * np.sqrt(rng.uniform())
        th = rng.uniform(0, 2 * np.pi)
        cx, cy = nx / 2 + rr * np.cos(th), ny / 2 + rr * np.sin(th)
        rad = rng.uniform(r_lo, r_hi)
        amp = rng.uniform(0.0, 1.0)
        out += amp * ((xs - cx) ** 2 + (ys - cy) ** 2 <= rad * rad)
    return _f32(out)


def _segment_distance(xs, ys, p, q):
    d = q - p
    L2 = float(d @ d)
    if L2 == 0.0:
        return np.hypot(xs - p[0], ys - p[1])
    t = np.clip(((xs - p[0]) * d[0] + (ys - p[1]) * d[1]) / L2, 0.0, 1.0)
    return np.hypot(xs - (p[0] + t * d[0]), ys - (p[1] + t * d[1]))


def vessel_phantom(rng, shape, radius_pts: float, *, k=6, steps=(10.0, 30.0), width=(1.0, 3.0),
                   amp=(0.5, 1.0), levels=None):
    """`k` random-walk polylines (3-8 vertices, steps U[10,30] points, width
    U[1,3] points, amplitude U[0.5,1]) combined by maximum, kept inside
    0.8*radius_pts of the grid centre.  Edges get a one-point linear ramp.

    With ``levels`` (a list of ``(scale, offset)`` pairs, as in
    :func:`blob_medium`) the same polylines are sampled on each level's grid
    and a list of arrays is returned; otherwise one array."""
    ny, nx = shape
    centre = np.array([nx / 2, ny / 2])
    rmax = 0.8 * radius_pts
    lines = []
    for _ in range(k):
        nv = int(rng.integers(3, 9))
        rr = 0.6 * rmax * np.sqrt(rng.uniform())
        th = rng.uniform(0, 2 * np.pi)
        pts = [centre + rr * np.array([np.cos(th), np.sin(th)])]
        heading = rng.uniform(0, 2 * np.pi)
        for _v in range(nv - 1):
            heading += rng.uniform(-np.pi / 3, np.pi / 3)
            step = rng.uniform(*steps)
            nxt = pts[-1] + step * np.array([np.cos(heading), np.sin(heading)])
            off = nxt - centre
            dist = np.hypot(*off)
            if dist > rmax:
                nxt = centre + off * (rmax / dist)
                heading += np.pi / 2
            pts.append(nxt)
        lines.append((pts, rng.uniform(*width), rng.uniform(*amp)))
    outs = []
    for scale, offset in (levels or ((1.0, 0.0),)):
        lshape = tuple(int(round(s / scale)) for s in shape)
        xs, ys = _coords(lshape)
        xs = xs * scale + offset
        ys = ys * scale + offset
        out = np.zeros(lshape)
        for pts, w, a in lines:
            for p, q in zip(pts[:-1], pts[1:]):
                dseg = _segment_distance(xs, ys, p, q)
                out = np.maximum(out, a * np.clip(w / 2 + 0.5 - dseg, 0.0, 1.0))
        outs.append(_f32(out))
    return outs if levels is not None else outs[0]


def ellipsoid_phantom(rng, shape, pml: int, *, k=6, semi=(3.0, 12.0), amp=(0.5, 1.0)):
    """Sum of `k` randomly rotated ellipsoids (semi-axes U[3,12] points,
    amplitude U[0.5,1]) centred in the interior (3D)."""
    xs = _coords(shape)
    n_phys = list(reversed(shape))
    out = np.zeros(shape)
    for _ in range(k):
        c = np.array([rng.uniform(pml + 12, n_phys[j] - 1 - pml - 12) for j in range(3)])
        ax = rng.uniform(*semi, size=3)
        # random rotation from a QR of a Gaussian matrix
        qm, rm = np.linalg.qr(rng.standard_normal((3, 3)))
        qm = qm * np.sign(np.diag(rm))
        a = rng.uniform(*amp)
        rel = [xs[j] - c[j] for j in range(3)]
        acc = np.zeros(shape)
        for r in range(3):
            comp = qm[0, r] * rel[0] + qm[1, r] * rel[1] + qm[2, r] * rel[2]
            acc += (comp / ax[r]) ** 2
        out += a * (acc <= 1.0)
    return _f32(out)


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

def _desc2(n, dx, pml, nt, *, pml_on=True, dt=0.0, origin=(0.0, 0.0)):
    return GridDesc(ndim=2, n=(n, n), dx=(dx, dx), origin=tuple(origin), nt=nt, dt=dt, cfl=0.3,
                    pml_size=(pml, pml, 0), pml_alpha=2.0, alpha_power=1.5, pml=pml_on)


def config1(instance: int = 0) -> Instance:
    """64^2, dx 0.1 mm, homogeneous lossless (c 1500, rho 1000), 10-point PML,
    CFL 0.3, Nt 300, 64 sensors on a circle of radius 28 points, five discs."""
    rng = rng_for(1, instance)
    n, dx = 64, 1e-4
    shape = (n, n)
    c0 = _f32(np.full(shape, 1500.0))
    rho0 = _f32(np.full(shape, 1000.0))
    p0 = disc_phantom(rng, shape)
    sens = circle_sensors(n, dx, 0.0, 28.0, 64)
    return Instance(_desc2(n, dx, 10, 300), c0, rho0, None, sens, p0, name="cfg1")


def _hetero2d(config: int, instance: int, n: int, nt: int, *, ns=256, pml=20, dx=1e-4) -> Instance:
    rng = rng_for(config, instance)
    shape = (n, n)
    (c0, rho0, a0), = blob_medium(rng, shape, pml)
    radius = n / 2 - pml - 8
    p0 = vessel_phantom(rng, shape, radius)
    sens = half_circle_sensors(n, dx, 0.0, radius, ns)
    return Instance(_desc2(n, dx, pml, nt), c0, rho0, a0, sens, p0, name=f"cfg{config}.{instance}")


def config2(instance: int = 0) -> Instance:
    """256^2, dx 0.1 mm, Gaussian-blob c and rho, alpha0 0.75, y 1.5, 20-point
    PML, Nt 1200, 256 half-circle sensors (r = 100 points), vessel phantom."""
    return _hetero2d(2, instance, 256, 1200)


def _level_geometry(count: int):
    """(scale, offset) of each multi-grid level's indices in fine-grid
    indices: level l is cell-centred over 2^l blocks of fine points."""
    return tuple((float(2 ** l), (2 ** l - 1) / 2.0) for l in range(count))


def multi_level(cfg: int, instance: int, n: int, dx: float, pml: int, nt: int, ns: int,
                count: int) -> List[Instance]:
    """`count` multi-grid levels of one 2D problem: an n^2 fine level and
    its cell-centred coarse levels (level l: (n/2^l)^2, dx and dt times 2^l,
    PML points and N_t divided by 2^l).  Medium and phantom are continuous
    functions drawn once and sampled on every grid; the ns sensors (left
    half-circle of radius n/2 - pml - 8 points) share physical positions.
    The fine time step is CFL 0.3 of the fine grid's maximum sound speed."""
    rng = rng_for(cfg, instance)
    shape = (n, n)
    lv = _level_geometry(count)
    media = blob_medium(rng, shape, pml, levels=lv)
    radius = n / 2 - pml - 8
    p0s = vessel_phantom(rng, shape, radius, levels=lv)
    sens = half_circle_sensors(n, dx, 0.0, radius, ns)
    dt_f = 0.3 * dx / float(np.max(media[0][0]))
    out = [Instance(_desc2(n, dx, pml, nt, dt=dt_f), *media[0], sens, p0s[0], name=f"cfg{cfg}.fine")]
    for l in range(1, count):
        s, off = lv[l]
        nl = n >> l
        desc = GridDesc(ndim=2, n=(nl, nl), dx=(s * dx, s * dx), origin=(off * dx, off * dx),
                        nt=nt >> l, dt=s * dt_f, cfl=0.3, pml_size=(pml >> l, pml >> l, 0),
                        pml_alpha=2.0, alpha_power=1.5, pml=True)
        out.append(Instance(desc, *media[l], sens.copy(), p0s[l], name=f"cfg{cfg}.level{l}"))
    return out


def two_level(cfg: int, instance: int, n: int, dx: float, pml: int, nt: int, ns: int) -> Tuple[Instance, Instance]:
    """Two multi-grid levels of one 2D problem (``multi_level`` with two
    levels): an n^2 fine level and its (n/2)^2 cell-centred coarse level."""
    fine, coarse = multi_level(cfg, instance, n, dx, pml, nt, ns, 2)
    return fine, Instance(coarse.desc, coarse.c0, coarse.rho0, coarse.alpha0_db, coarse.sensors, coarse.p0,
                          name=f"cfg{cfg}.coarse")


def ellipsoids(rng, shape, pml: int, *, k=6, semi=(3.0, 12.0), amp=(0.5, 1.0), margin=12.0,
               levels=((1.0, 0.0),)):
    """The ellipsoid phantom of :func:`ellipsoid_phantom` (centres kept
    `margin` points clear of the PML) sampled on several levels
    (``(scale, offset)`` pairs as in :func:`blob_medium`); returns one array
    per level."""
    n_phys = list(reversed(shape))
    params = []
    for _ in range(k):
        c = np.array([rng.uniform(pml + margin, n_phys[j] - 1 - pml - margin) for j in range(3)])
        ax = rng.uniform(*semi, size=3)
        qm, rm = np.linalg.qr(rng.standard_normal((3, 3)))
        qm = qm * np.sign(np.diag(rm))
        params.append((c, ax, qm, rng.uniform(*amp)))
    outs = []
    for scale, offset in levels:
        lshape = tuple(int(round(s / scale)) for s in shape)
        xs = [x * scale + offset for x in _coords(lshape)]
        out = np.zeros(lshape)
        for c, ax, qm, a in params:
            rel = [xs[j] - c[j] for j in range(3)]
            acc = np.zeros(lshape)
            for r in range(3):
                comp = qm[0, r] * rel[0] + qm[1, r] * rel[1] + qm[2, r] * rel[2]
                acc += (comp / ax[r]) ** 2
            out += a * (acc <= 1.0)
        outs.append(_f32(out))
    return outs


def multi_level_3d(cfg: int, instance: int, n: int, dx: float, pml: int, nt: int, count: int) -> List[Instance]:
    """`count` multi-grid levels of one 3D problem (n^3 fine, cell-centred
    coarse levels as in :func:`multi_level`): medium as config 5 (c clipped
    to [1450, 1600], rho 1000, alpha0 0.75) with blobs of 4-12 points,
    ellipsoids of semi-axes 2-6 points centred 4 points clear of the PML,
    sensors on the interior nodes (x, y in [pml, n - 1 - pml]) of the fine
    plane z = pml at the same physical positions on every level."""
    rng = rng_for(cfg, instance)
    shape = (n, n, n)
    lv = _level_geometry(count)
    media = blob_medium(rng, shape, pml, c_clip=(1450.0, 1600.0), hetero_rho=False, sig=(4.0, 12.0), levels=lv)
    p0s = ellipsoids(rng, shape, pml, semi=(2.0, 6.0), margin=4.0, levels=lv)
    idx = np.arange(pml, n - pml, dtype=np.float64)
    gx, gy = np.meshgrid(idx, idx, indexing="xy")
    sens = np.stack([gx.ravel() * dx, gy.ravel() * dx, np.full(gx.size, pml * dx)], axis=1)
    dt_f = 0.3 * dx / 1600.0
    out = []
    for l in range(count):
        s, off = lv[l]
        nl = n >> l
        desc = GridDesc(ndim=3, n=(nl,) * 3, dx=(s * dx,) * 3, origin=(off * dx,) * 3, nt=nt >> l, dt=s * dt_f,
                        cfl=0.3, pml_size=(pml >> l,) * 3, pml_alpha=2.0, alpha_power=1.5, pml=True)
        out.append(Instance(desc, *media[l], sens.copy(), p0s[l], name=f"cfg{cfg}.level{l}"))
    return out


def config3(instance: int = 0) -> Tuple[Instance, Instance]:
    """Two multi-grid levels of one problem: 512^2 fine (dx 0.1 mm, 20-pt
    PML, Nt 2400) and its 256^2 cell-centred coarse level (dx 0.2 mm, 10-pt
    PML, Nt 1200, dt doubled), 256 sensors."""
    return two_level(3, instance, 512, 1e-4, 20, 2400, 256)


def config4(instance_count: int = 48) -> List[Instance]:
    """48 uneven 2D instances: 16 each of 128^2 (Nt 600), 256^2 (Nt 1200) and
    512^2 (Nt 2400), media and phantoms as config 2, seeds 4000..4047."""
    sizes = [(128, 600), (256, 1200), (512, 2400)]
    out = []
    for i in range(instance_count):
        n, nt = sizes[i // 16 % 3] if instance_count == 48 else sizes[i % 3]
        out.append(_hetero2d(4, i, n, nt))
    return out


def config5(instance: int = 0, n: int = 128, nt: int = 800) -> Instance:
    """128^3, dx 0.2 mm, c = 1500 + blobs clipped to [1450, 1600], rho 1000,
    alpha0 0.75, y 1.5, 16-point PML, Nt 800, sensors on every (x, y) node of
    the plane z = 16, six random ellipsoids."""
    rng = rng_for(5, instance)
    dx, pml = 2e-4, 16
    shape = (n, n, n)
    (c0, rho0, a0), = blob_medium(rng, shape, pml, c_clip=(1450.0, 1600.0), hetero_rho=False,
                                  sig=(10.0, 30.0))
    p0 = ellipsoid_phantom(rng, shape, pml)
    sens = plane_sensors(n, n, (dx,) * 3, (0.0,) * 3, pml)
    desc = GridDesc(ndim=3, n=(n, n, n), dx=(dx,) * 3, origin=(0.0,) * 3, nt=nt, dt=0.3 * dx / 1600.0,
                    cfl=0.3, pml_size=(pml,) * 3, pml_alpha=2.0, alpha_power=1.5, pml=True)
    return Instance(desc, c0, rho0, a0, sens, p0, name="cfg5")


def small_instance(seed: int, n=(16, 16), *, nt=20, ns=5, pml=3, lossy=True, hetero=True,
                   pml_on=True, dx=1e-4, ndim=None) -> Instance:
    """Tiny random problem for exhaustive tests (2D or 3D by len(n)).

    Medium: smooth random perturbations; p0: random smooth bump + noise;
    sensors: random positions strictly inside the grid."""
    rng = np.random.default_rng(seed)
    nd = len(n) if ndim is None else ndim
    shape = tuple(reversed(n))
    xs = _coords(shape)
    if hetero:
        c = 1500.0 + 60.0 * np.sin(2 * np.pi * xs[0] / n[0] + rng.uniform(0, 6)) * \
            np.cos(2 * np.pi * xs[1] / n[1] + rng.uniform(0, 6))
        rho = 1000.0 + 80.0 * np.cos(2 * np.pi * xs[-1] / n[-1] + rng.uniform(0, 6)) + \
            20.0 * rng.uniform(-1, 1, size=shape)
    else:
        c = np.full(shape, 1500.0)
        rho = np.full(shape, 1000.0)
    a0 = (0.75 + 0.25 * rng.uniform(-1, 1, size=shape)) if lossy else None
    p0 = rng.standard_normal(shape)
    sens = np.stack([rng.uniform(0.5, n[j] - 1.5, size=ns) * dx for j in range(nd)], axis=1)
    desc = GridDesc(ndim=nd, n=tuple(n), dx=(dx,) * nd, origin=(0.0,) * nd, nt=nt, dt=0.0, cfl=0.3,
                    pml_size=tuple([pml] * nd + [0] * (3 - nd)), pml_alpha=2.0, alpha_power=1.5,
                    pml=pml_on)
    return Instance(desc, _f32(c), _f32(rho), None if a0 is None else _f32(a0), sens, _f32(p0),
                    name=f"small{seed}")


def with_desc(inst: Instance, **kw) -> Instance:
    """Copy of an instance with descriptor fields replaced."""
    return Instance(replace(inst.desc, **kw), inst.c0, inst.rho0, inst.alpha0_db, inst.sensors,
                    inst.p0, inst.name, dict(inst.extra))
