"""Seeded synthetic inputs for the FWI gradient path.

This module is shared by the CPU oracle, the tests and the benchmark. It
holds no part of the method's arithmetic (no stencil, no adjoint, no codec):
only velocity models, source wavelets, acquisition geometry and analytic
test fields, each drawn from ``numpy.random.default_rng(seed)``.

Conventions
-----------
* Axes are (x, z) in 2D and (x, y, z) in 3D, depth z last and contiguous.
* ``shape`` is the physical grid; the computational grid adds ``nbl`` points
  on every side (40 in the paper's reference problem, Sec. 3 "Reference
  Problem").  Velocities are extended into that layer by edge replication.
* ``m = 1/c^2`` is the squared slowness of Eq. (1), in s^2/m^2.
* Source and receiver positions are physical-grid node indices.
* Time sample n of the wavelet is injected on the step n -> n+1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import ndimage

# Nyquist value of the 1D symbol of the order-SO central second-derivative
# stencil (largest eigenvalue of -h^2 d2/dx2).  These are configuration
# constants used to place dt at a fraction of the leapfrog stability limit
# dt_max = 2h / (vmax * sqrt(ndim * S)); they are input data, not solver code.
NYQUIST_SYMBOL = {4: 16.0 / 3.0, 8: 6.501587301587302, 16: 7.42692143835001}


def stable_dt(h: float, vmax: float, ndim: int, so: int, frac: float = 0.8) -> float:
    """dt at ``frac`` of the leapfrog stability limit for the given stencil."""
    return frac * 2.0 * h / (vmax * math.sqrt(ndim * NYQUIST_SYMBOL[so]))


def ricker(f0: float, dt: float, nt: int) -> np.ndarray:
    """Ricker wavelet of peak frequency ``f0`` sampled at n*dt, n = 0..nt-1.

    Delay t0 = 1.5/f0 and unit amplitude (the paper states only an 8 Hz
    Ricker source, Sec. 3 "Reference Problem"; delay and amplitude are our
    reading)."""
    t = np.arange(nt, dtype=np.float64) * dt - 1.5 / f0
    a = (math.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def extend(v: np.ndarray, nbl: int) -> np.ndarray:
    """Physical model -> computational grid by edge replication."""
    return np.pad(v, nbl, mode="edge") if nbl > 0 else v.copy()


def slowness2(v: np.ndarray) -> np.ndarray:
    """Squared slowness m = 1/c^2 (float64)."""
    return 1.0 / (np.asarray(v, dtype=np.float64) ** 2)


@dataclasses.dataclass
class Shot:
    """One shot: physical grid, discretisation and acquisition."""
    ndim: int
    shape: tuple            # physical dims
    h: float
    so: int
    nbl: int
    nt: int
    dt: float
    vmax: float
    f0: float
    src: tuple              # physical node
    rec: np.ndarray         # (nrec, ndim) int32 physical nodes

    @property
    def comp_shape(self) -> tuple:
        return tuple(n + 2 * self.nbl for n in self.shape)

    def wavelet(self) -> np.ndarray:
        return ricker(self.f0, self.dt, self.nt)


def _smooth_noise(rng, shape, sigma, amp):
    p = ndimage.gaussian_filter(rng.standard_normal(shape), sigma, mode="nearest")
    return p * (amp / np.max(np.abs(p)))


# ---------------------------------------------------------------- 2D layered
def layered_2d(shape=(101, 101), speeds=(1500.0, 2500.0, 3500.0), seed=12623,
               pert=0.05, sigma=5.0):
    """Equal-thickness horizontal layers in depth, plus a seeded Gaussian-
    smoothed perturbation scaled to max |p| = ``pert`` (the "true" model).

    Returns (v0, v_true) on the physical grid, float64 m/s."""
    nx, nz = shape
    v0 = np.empty(shape)
    edges = np.linspace(0, nz, len(speeds) + 1).round().astype(int)
    for i, s in enumerate(speeds):
        v0[:, edges[i]:edges[i + 1]] = s
    rng = np.random.default_rng(seed)
    p = _smooth_noise(rng, shape, sigma, pert)
    return v0, v0 * (1.0 + p)


def config1_shot(nt=500):
    """2D single shot: 101x101 at 10 m, SO4, 10 Hz, 101 receivers at 20 m."""
    vref = 3500.0
    dt = stable_dt(10.0, vref, 2, 4)
    rec = np.stack([np.arange(101), np.full(101, 2)], axis=1).astype(np.int32)
    return Shot(2, (101, 101), 10.0, 4, 40, nt, dt, vref * 1.05, 10.0, (50, 2), rec)


# ------------------------------------------------------- 3D layered (codec)
def layered_undulating_3d(shape, speeds=(1500.0, 2500.0, 3500.0, 4500.0),
                          seed=12624, amp_pts=10.0):
    """Layers in depth whose interfaces undulate sinusoidally (seeded phase
    and wavenumber), amplitude ``amp_pts`` grid points."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    x = np.arange(nx)[:, None]
    y = np.arange(ny)[None, :]
    v = np.full(shape, speeds[0])
    zz = np.arange(nz)[None, None, :]
    for i in range(1, len(speeds)):
        base = nz * i / len(speeds)
        kx, ky = rng.uniform(1.0, 3.0, 2) * 2 * math.pi / np.array([nx, ny])
        ph = rng.uniform(0, 2 * math.pi, 2)
        surf = base + amp_pts * np.sin(kx * x + ph[0]) * np.cos(ky * y + ph[1])
        v = np.where(zz >= surf[:, :, None], speeds[i], v)
    return v


def config2_shot(n=256, nt=300):
    """3D point source at the centre of a layered medium (codec snapshots)."""
    vref = 4500.0
    dt = stable_dt(10.0, vref, 3, 8)
    c = n // 2
    return Shot(3, (n, n, n), 10.0, 8, 40, nt, dt, vref, 15.0, (c, c, c),
                np.zeros((0, 3), np.int32))


def wavefield_like(shape, seed=12624, nshell=6, f_pts=8.0, noise=0.0):
    """Analytic stand-in for a propagated snapshot: a few expanding Ricker
    shells (spherical/circular wavefronts from seeded centres) with 1/r
    decay, optional white noise.  Values are O(1), like the fields the paper
    compresses (range about 1-2).  float32."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape],
                        indexing="ij")
    out = np.zeros(shape)
    for _ in range(nshell):
        c = [rng.uniform(0, s) for s in shape]
        r = np.sqrt(sum((g - ci) ** 2 for g, ci in zip(grids, c)))
        r0 = rng.uniform(0.2, 0.8) * max(shape)
        a = (math.pi * (r - r0) / f_pts) ** 2
        out += rng.uniform(0.3, 1.0) * (1 - 2 * a) * np.exp(-a) * (r0 / (r + r0))
    if noise:
        out += noise * rng.standard_normal(shape)
    return out.astype(np.float32)


# ------------------------------------------------- 3D thrust-faulted layers
def separable_field(shape, seed=12629, nterm=3):
    """Cheap large stand-in for a wavefield snapshot: a sum of ``nterm``
    separable products of seeded 1D wave packets (Gaussian-windowed cosines),
    values O(1).  float32; memory and time linear in the number of points."""
    rng = np.random.default_rng(seed)
    out = np.zeros(shape, np.float32)
    for _ in range(nterm):
        prod = None
        for n in shape:
            t = np.arange(n, dtype=np.float64)
            c, w = rng.uniform(0.2, 0.8) * n, rng.uniform(0.1, 0.3) * n
            k = rng.uniform(0.1, 0.6)
            prof = (np.cos(k * (t - c)) * np.exp(-((t - c) / w) ** 2)).astype(np.float32)
            prod = prof if prod is None else np.multiply.outer(prod, prof)
        out += np.float32(rng.uniform(0.3, 1.0)) * prod
    return out


def _thrust_params(shape, nlayer, seed, fold_pts, fault_pts):
    """Seeded fault planes and folded interface surfaces (2D arrays)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    x = np.arange(nx, dtype=np.float64)[:, None]
    y = np.arange(ny, dtype=np.float64)[None, :]
    # two thrust faults: planes x cos(a) + y sin(a) = d0 + z tan(dip); the
    # hanging wall is lifted by an offset
    faults = []
    for _ in range(2):
        a = rng.uniform(0, math.pi)
        d0 = rng.uniform(0.3, 0.7) * (nx * abs(math.cos(a)) + ny * abs(math.sin(a)))
        dip = math.tan(rng.uniform(math.radians(25), math.radians(45)))
        off = rng.uniform(0.5, 1.0) * fault_pts
        faults.append((math.cos(a), math.sin(a), d0, dip, off))
    surfs = []
    for i in range(1, nlayer):
        surf = np.full((nx, ny), nz * i / nlayer)
        for _ in range(2):
            k = rng.uniform(0.5, 2.5, 2) * 2 * math.pi / np.array([nx, ny])
            ph = rng.uniform(0, 2 * math.pi, 2)
            surf += 0.5 * fold_pts * np.sin(k[0] * x + ph[0]) * np.sin(k[1] * y + ph[1])
        surfs.append(surf)
    return faults, surfs


def thrust_3d(shape, nlayer=10, vmin=2200.0, vmax=6000.0, seed=12625,
              fold_pts=15.0, fault_pts=20.0):
    """Layered 3D model with folded interfaces and two dipping thrust faults
    (a synthetic stand-in for the SEG/EAGE Overthrust model, whose values are
    not used).  Velocity increases with layer index from vmin to vmax."""
    nx, ny, nz = shape
    faults, surfs = _thrust_params(shape, nlayer, seed, fold_pts, fault_pts)
    speeds = np.linspace(vmin, vmax, nlayer)
    x = np.arange(nx, dtype=np.float64)[:, None]
    y = np.arange(ny, dtype=np.float64)[None, :]
    zz = np.arange(nz, dtype=np.float64)[None, None, :]
    idx = np.zeros(shape, dtype=np.int16)
    for surf in surfs:
        zsurf = surf[:, :, None] + np.zeros_like(zz)
        for cx, sy, d0, dip, off in faults:
            hang = (cx * x + sy * y)[:, :, None] - dip * zz > d0
            zsurf = np.where(hang, zsurf - off, zsurf)
        idx += (zz >= zsurf).astype(np.int16)
    return speeds[idx]


def thrust_3d_torch(shape, device, nlayer=10, vmin=2200.0, vmax=6000.0, seed=12625,
                    fold_pts=15.0, fault_pts=20.0):
    """``thrust_3d`` assembled with torch on ``device`` (same draws)."""
    import torch
    nx, ny, nz = shape
    faults, surfs = _thrust_params(shape, nlayer, seed, fold_pts, fault_pts)
    f64 = dict(dtype=torch.float64, device=device)
    x = torch.arange(nx, **f64)[:, None, None]
    y = torch.arange(ny, **f64)[None, :, None]
    zz = torch.arange(nz, **f64)[None, None, :]
    idx = torch.zeros(shape, dtype=torch.int16, device=device)
    hangs = [((cx * x + sy * y) - dip * zz > d0, off) for cx, sy, d0, dip, off in faults]
    for surf in surfs:
        zsurf = torch.as_tensor(surf, **f64)[:, :, None].expand(nx, ny, nz)
        for hang, off in hangs:
            zsurf = torch.where(hang, zsurf - off, zsurf)
        idx += (zz >= zsurf).to(torch.int16)
    speeds = torch.as_tensor(np.linspace(vmin, vmax, nlayer), **f64)
    return speeds[idx.long()]


def gauss_smooth_torch(v, sigma, truncate=4.0):
    """Separable Gaussian smoothing with edge replication (torch): a weighted
    sum of shifted copies along each axis."""
    import torch
    r = int(truncate * sigma + 0.5)
    t = torch.arange(-r, r + 1, dtype=torch.float64)
    w = torch.exp(-0.5 * (t / sigma) ** 2)
    w = (w / w.sum()).tolist()
    out = v
    for ax in range(v.dim()):
        n = out.shape[ax]
        first = out.narrow(ax, 0, 1)
        last = out.narrow(ax, n - 1, 1)
        padded = torch.cat([first.expand(*[r if d == ax else -1 for d in range(v.dim())]),
                            out,
                            last.expand(*[r if d == ax else -1 for d in range(v.dim())])], dim=ax)
        acc = torch.zeros_like(out)
        for k in range(2 * r + 1):
            acc.add_(padded.narrow(ax, k, n), alpha=w[k])
        out = acc
    return out.contiguous()


def extend_torch(v, nbl):
    import torch.nn.functional as Fn
    if nbl <= 0:
        return v.clone()
    pad = (nbl,) * (2 * v.dim())
    return Fn.pad(v[None, None], pad, mode="replicate")[0, 0].contiguous()


def config3_shot(shape=(881, 881, 287), nt=2000, rec_step=4):
    """3D single shot at 25 m, SO8, 8 Hz; receivers every ``rec_step`` nodes
    on the surface at depth 2h."""
    vref = 6000.0
    h = 25.0
    dt = stable_dt(h, vref, 3, 8)
    nx, ny, _ = shape
    ix, iy = np.meshgrid(np.arange(0, nx, rec_step), np.arange(0, ny, rec_step),
                         indexing="ij")
    rec = np.stack([ix.ravel(), iy.ravel(), np.full(ix.size, 2)], axis=1).astype(np.int32)
    return Shot(3, shape, h, 8, 40, nt, dt, vref, 8.0, (nx // 2, ny // 2, 2), rec)


def config3_models(shape=(881, 881, 287), seed=12625):
    """(v_smooth, v_true): the gradient is taken at the smoothed model
    (Gaussian sigma = 3 points), observed data come from the sharp one."""
    v = thrust_3d(shape, seed=seed)
    vs = ndimage.gaussian_filter(v, 3.0, mode="nearest")
    return vs, v


# ------------------------------------------------------------ batched shots
def config4_shots(model_shape=(401, 401, 201), nshot=32, wmin=161, wmax=321,
                  seed=12626, nt=1500):
    """32 shots on uneven crops of one 3D model.  Each shot: crop origin
    (ox, oy), width W; source at the crop centre at depth 2h; receivers on
    every 2nd node of the crop surface at depth 2h.  Returns a list of
    (Shot, (ox, oy, W))."""
    rng = np.random.default_rng(seed)
    h = 20.0
    vref = 6000.0
    dt = stable_dt(h, vref, 3, 8)
    nx, ny, nz = model_shape
    out = []
    for _ in range(nshot):
        w = int(rng.integers(wmin, wmax + 1))
        ox = int(rng.integers(0, nx - w + 1))
        oy = int(rng.integers(0, ny - w + 1))
        ix, iy = np.meshgrid(np.arange(0, w, 2), np.arange(0, w, 2), indexing="ij")
        rec = np.stack([ix.ravel(), iy.ravel(), np.full(ix.size, 2)], axis=1).astype(np.int32)
        shot = Shot(3, (w, w, nz), h, 8, 40, nt, dt, vref, 8.0, (w // 2, w // 2, 2), rec)
        out.append((shot, (ox, oy, w)))
    return out


# ----------------------------------------------------------- 2D smooth (C5)
def smooth_2d(shape=(1001, 401), seed=12627, vtop=1500.0, vbot=4500.0,
              noise=0.05, sigma=20.0):
    """Linear increase with depth plus smoothed +-5% noise, clipped."""
    nx, nz = shape
    rng = np.random.default_rng(seed)
    z = np.arange(nz) / (nz - 1)
    v = vtop + (vbot - vtop) * z[None, :] + np.zeros(shape)
    v = v * (1 + _smooth_noise(rng, shape, sigma, noise))
    return np.clip(v, vtop, vbot)


def blobs_2d(v, seed=12628, nblob=3, amp=0.05, sigma=15.0):
    """True model: ``v`` with seeded +-5% Gaussian blobs."""
    rng = np.random.default_rng(seed)
    nx, nz = v.shape
    x = np.arange(nx)[:, None]
    z = np.arange(nz)[None, :]
    out = v.copy()
    for _ in range(nblob):
        cx, cz = rng.uniform(0.2, 0.8) * nx, rng.uniform(0.3, 0.8) * nz
        s = rng.choice([-1.0, 1.0]) * amp
        out *= 1 + s * np.exp(-((x - cx) ** 2 + (z - cz) ** 2) / (2 * sigma ** 2))
    return out


def config5_shots(shape=(1001, 401), nshot=16, nt=3000):
    vref = 4500.0
    h = 10.0
    dt = stable_dt(h, vref, 2, 16)
    nx, nz = shape
    rec = np.stack([np.arange(nx), np.full(nx, 2)], axis=1).astype(np.int32)
    xs = np.linspace(0, nx - 1, nshot + 2)[1:-1].round().astype(int)
    return [Shot(2, shape, h, 16, 40, nt, dt, vref * 1.05, 10.0, (int(x), 2), rec)
            for x in xs]


# ------------------------------------------------------------ tiny problems
def tiny_shot(ndim=2, n=24, so=4, nbl=6, nt=60, h=10.0, vmax=2500.0, f0=None,
              nrec=None, frac=0.8):
    """Small problem for oracle pins and parity tests.  f0 is chosen so the
    wavelet is resolved by about 8 points per wavelength at vmin=1500."""
    shape = (n,) * ndim
    dt = stable_dt(h, vmax, ndim, so, frac)
    if f0 is None:
        f0 = 1500.0 / (8 * h)
    c = n // 2
    src = (c,) * (ndim - 1) + (2,)
    if ndim == 2:
        xs = np.arange(n) if nrec is None else np.linspace(0, n - 1, nrec).round()
        rec = np.stack([xs, np.full(len(xs), 2)], 1)
    else:
        step = 2 if nrec is None else nrec
        ix, iy = np.meshgrid(np.arange(0, n, step), np.arange(0, n, step), indexing="ij")
        rec = np.stack([ix.ravel(), iy.ravel(), np.full(ix.size, 2)], 1)
    return Shot(ndim, shape, h, so, nbl, nt, dt, vmax, f0, src, rec.astype(np.int32))


def tiny_models(shape, seed=7, vmin=1500.0, vmax=2500.0):
    """(v0, v_true): smooth depth gradient and a perturbed version."""
    rng = np.random.default_rng(seed)
    nz = shape[-1]
    z = np.arange(nz) / max(nz - 1, 1)
    v0 = vmin + (vmax - vmin) * 0.6 * z.reshape((1,) * (len(shape) - 1) + (nz,))
    v0 = v0 + np.zeros(shape)
    p = _smooth_noise(rng, shape, 2.0, 0.05)
    return v0, v0 * (1 + p)
