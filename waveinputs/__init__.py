"""Seeded synthetic inputs for the acoustic-wave sweep and the explicit-
diffusion (Laplace-operator) sweep.

This module only *generates inputs*: velocity models, source wavelets,
source/receiver coordinates and the geometry of the standard workloads.  It
holds none of the method's arithmetic (no stencil, no time stepping, no
damping profile, no interpolation), so both the FP64 oracle and the HIP
library can be fed from it without sharing any of the computation.

Conventions
-----------
* Arrays are row-major with axis 0 the slowest ("depth", streamed on the GPU)
  and the last axis unit stride.
* Models are returned as float32 squared slowness m = 1/c^2 (s^2/m^2); the
  oracle promotes the same float32 values to float64, so both sides see the
  identical model.
* Coordinates are float64 metres measured from computational-grid node 0 (the
  outer face of the absorbing layer when there is one).
* The absorbing layer is added *outside* the physical shape; physical depths
  are offset by ``nbl`` points.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

C_MIN = 1500.0
C_MAX = 4500.0


def ricker(nt: int, dt: float, f0: float, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet sampled at t = n dt, n = 0..nt-1; t0 defaults to 1/f0."""
    if t0 is None:
        t0 = 1.0 / f0
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def sigma_max_estimate(c_max: float, nbl: int, h: float, reflection: float = 1e-3) -> float:
    """Damping-profile maximum (1/s) from the usual sponge estimate
    3 c_max ln(1/R) / (2 L), L = nbl h.  An input choice, not part of the sweep."""
    if nbl <= 0:
        return 0.0
    return 3.0 * c_max * math.log(1.0 / reflection) / (2.0 * nbl * h)


def pad_edges(c: np.ndarray, nbl: int) -> np.ndarray:
    """Extend a physical velocity model into the absorbing layer by edge replication."""
    if nbl <= 0:
        return c
    return np.pad(c, nbl, mode="edge")


def to_slowness2(c: np.ndarray) -> np.ndarray:
    return (1.0 / (c.astype(np.float64) ** 2)).astype(np.float32)


def constant_velocity(shape, c: float) -> np.ndarray:
    return np.full(tuple(shape), c, dtype=np.float64)


def layered_velocity(shape, nlayers: int, seed: int, cmin=C_MIN, cmax=C_MAX) -> np.ndarray:
    """nlayers equal-thickness horizontal layers along axis 0, velocities
    uniform-random in [cmin, cmax] (unsorted)."""
    rng = np.random.default_rng(seed)
    vel = rng.uniform(cmin, cmax, size=nlayers)
    n0 = shape[0]
    layer = np.minimum((np.arange(n0) * nlayers) // n0, nlayers - 1)
    prof = vel[layer]
    return np.broadcast_to(prof.reshape((n0,) + (1,) * (len(shape) - 1)), tuple(shape)).copy()


def smooth_random_velocity(shape, seed: int, sigma_cells: float = 8.0,
                           cmin=C_MIN, cmax=C_MAX, device=None) -> np.ndarray:
    """White noise N(0,1) -> Gaussian filter (sigma in cells, reflecting edges,
    truncated at 4 sigma) -> affine min-max map onto [cmin, cmax].

    device (a torch device) filters the same noise there (separable
    convolution with the same normalised taps and half-sample-symmetric
    edges), for grids whose CPU filtering takes a minute; the result equals
    the CPU one up to FP32 rounding of the filter sums."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(size=tuple(shape), dtype=np.float32)
    if device is not None:
        return _smooth_torch(noise, sigma_cells, cmin, cmax, device)
    from scipy.ndimage import gaussian_filter
    sm = gaussian_filter(noise, sigma=sigma_cells, mode="reflect", truncate=4.0, output=np.float32)
    lo, hi = float(sm.min()), float(sm.max())
    sm = (sm.astype(np.float64) - lo) / max(hi - lo, 1e-30)
    return cmin + (cmax - cmin) * sm


def _smooth_torch(noise: np.ndarray, sigma: float, cmin: float, cmax: float, device) -> np.ndarray:
    import torch
    import torch.nn.functional as F
    K = int(4.0 * sigma + 0.5)                       # truncate at 4 sigma, as scipy
    x = np.arange(-K, K + 1, dtype=np.float64)
    taps = np.exp(-0.5 * (x / sigma) ** 2)
    taps = torch.tensor(taps / taps.sum(), dtype=torch.float32, device=device)
    u = torch.from_numpy(noise).to(device)
    for ax in range(u.dim()):
        v = u.movedim(ax, -1)
        lead = v.shape[:-1]
        v = v.reshape(-1, 1, v.shape[-1])
        # half-sample-symmetric edges (d c b a | a b c d | d c b a)
        v = torch.cat([v[..., :K].flip(-1), v, v[..., -K:].flip(-1)], dim=-1)
        out = torch.empty((v.shape[0], 1, v.shape[-1] - 2 * K), dtype=torch.float32, device=device)
        step = max(1, (1 << 26) // v.shape[-1])
        for i in range(0, v.shape[0], step):
            out[i:i + step] = F.conv1d(v[i:i + step], taps.view(1, 1, -1))
        u = out.reshape(*lead, -1).movedim(-1, ax).contiguous()
        del v, out
    lo, hi = float(u.min()), float(u.max())
    sm = ((u.double() - lo) / max(hi - lo, 1e-30)).cpu().numpy()
    return cmin + (cmax - cmin) * sm


@dataclass
class Workload:
    """One synthetic problem: geometry, model, source and receivers."""
    name: str
    shape: tuple            # computational shape, absorbing layer included
    spacing: tuple
    dt: float
    so: int
    nt: int
    nbl: int
    sigma_max: float
    m: np.ndarray            # float32 [shape]
    src_xyz: np.ndarray      # float64 [nsrc, ndim]
    wavelet: np.ndarray      # float32 [nt, nsrc]
    rec_xyz: np.ndarray      # float64 [nrec, ndim]
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def npts(self):
        return int(np.prod(self.shape))


def _line(ndim, depth_idx, across_idx, n_last, h, nbl):
    """Receivers at physical depth index `depth_idx`, physical axis-1 index
    `across_idx` (3D), every node along the last axis of the physical domain."""
    k = np.arange(n_last, dtype=np.float64) + nbl
    if ndim == 3:
        xyz = np.stack([np.full_like(k, (depth_idx + nbl) * h[0]),
                        np.full_like(k, (across_idx + nbl) * h[1]),
                        k * h[2]], axis=1)
    else:
        xyz = np.stack([np.full_like(k, (depth_idx + nbl) * h[0]), k * h[1]], axis=1)
    return xyz


def make_workload(name: str, shape, h: float, so: int, nt: int, nbl: int, c_phys: np.ndarray,
                  f0: float, src_phys_idx, rec_depth_idx: Optional[int], cfl: float = 0.4,
                  c_max: float = None, extra=None) -> Workload:
    ndim = len(shape)
    spacing = (float(h),) * ndim
    if c_max is None:
        c_max = float(c_phys.max())
    dt = cfl * h / c_max
    c = pad_edges(c_phys, nbl)
    comp_shape = tuple(int(s) for s in c.shape)
    src = np.array([[(src_phys_idx[a] + nbl) * h for a in range(ndim)]], dtype=np.float64)
    wav = ricker(nt, dt, f0).reshape(nt, 1)
    if rec_depth_idx is None:
        rec = np.zeros((0, ndim))
    else:
        rec = _line(ndim, rec_depth_idx, shape[1] // 2 if ndim == 3 else 0, shape[-1], spacing, nbl)
    return Workload(name=name, shape=comp_shape, spacing=spacing, dt=dt, so=so, nt=nt, nbl=nbl,
                    sigma_max=sigma_max_estimate(c_max, nbl, h), m=to_slowness2(c), src_xyz=src,
                    wavelet=wav, rec_xyz=rec, extra=dict(extra or {}))


def point_source_64(nt: int = 100, n: int = 64) -> Workload:
    """64^3, h=10 m, so4, constant 1500 m/s, no damping, 15 Hz Ricker at the
    grid centre, 64 receivers at depth index 2 across the middle row."""
    shape = (n, n, n)
    w = make_workload("const_%dcube_so4" % n, shape, 10.0, 4, nt, 0, constant_velocity(shape, 1500.0), 15.0,
                      (n // 2, n // 2, n // 2), None)
    k = np.arange(n, dtype=np.float64)
    w.rec_xyz = np.stack([np.full_like(k, 2 * 10.0), np.full_like(k, (n // 2) * 10.0), k * 10.0], axis=1)
    return w


def layered_512(nt: int = 1000, n: int = 512, seed: int = 2, so: int = 8, nbl: int = 40) -> Workload:
    """512^3 (+40-point layer), h=10 m, so8, 8 random horizontal layers in
    1.5-4.5 km/s, 10 Hz Ricker at depth 20 in the middle, a receiver line at
    depth 2 (dt fixed by c_max = 4.5 km/s at CFL 0.4)."""
    shape = (n, n, n)
    c = layered_velocity(shape, 8, seed)
    return make_workload("layered_%dcube_so%d" % (n, so), shape, 10.0, so, nt, nbl, c, 10.0,
                         (min(20, n - 1), n // 2, n // 2), 2, c_max=C_MAX)


def smooth_768(so: int = 12, nt: int = 500, n: int = 768, seed: int = 3, nbl: int = 40, device=None) -> Workload:
    """768^3 (+40), h=12.5 m, smooth random velocity (sigma 8 cells), so12/16
    (device: filter the noise there, see smooth_random_velocity)."""
    shape = (n, n, n)
    c = smooth_random_velocity(shape, seed, device=device)
    return make_workload("smooth_%dcube_so%d" % (n, so), shape, 12.5, so, nt, nbl, c, 10.0,
                         (min(20, n - 1), n // 2, n // 2), 2, c_max=C_MAX)


def gradient_256(nt: int = 2000, n: int = 256, seed: int = 4, nbl: int = 40, ckpt_every: int = 50) -> dict:
    """Adjoint-gradient problem: smooth random true model, constant 2 km/s
    starting model, one Ricker shot at depth 20, 256 receivers at depth 2."""
    shape = (n, n, n)
    c_true = smooth_random_velocity(shape, seed)
    true = make_workload("smooth_%dcube_so8_true" % n, shape, 10.0, 8, nt, nbl, c_true, 10.0,
                         (min(20, n - 1), n // 2, n // 2), 2, c_max=C_MAX)
    init = make_workload("const2000_%dcube_so8_init" % n, shape, 10.0, 8, nt, nbl, constant_velocity(shape, 2000.0),
                         10.0, (min(20, n - 1), n // 2, n // 2), 2, c_max=C_MAX)
    return {"true": true, "init": init, "ckpt_every": ckpt_every}


def shot_batch(nshots: int = 32, nt: int = 800, seed: int = 5, sizes=None, workers: int = 1) -> list:
    """Batch of independent shots: per-axis sizes from {128, 144, ..., 320},
    space order alternating 4/8, per-shot smooth random model, random source
    (interior, depth >= 2 radius), receiver line at depth 2, no layer.  The
    models are generated on `workers` threads (same result for any count)."""
    rng = np.random.default_rng(seed)
    choices = np.arange(128, 321, 16)
    spec = []
    for i in range(nshots):
        shp = tuple(int(v) for v in (rng.choice(choices, size=3) if sizes is None else sizes[i]))
        so = 4 if i % 2 == 0 else 8
        r = so // 2
        src = (int(rng.integers(2 * r, shp[0] - 2 * r)), int(rng.integers(2 * r, shp[1] - 2 * r)),
               int(rng.integers(2 * r, shp[2] - 2 * r)))
        spec.append((shp, so, src))

    def one(i):
        shp, so, src = spec[i]
        c = smooth_random_velocity(shp, seed * 1000 + i)
        return make_workload("batch_shot%02d" % i, shp, 10.0, so, nt, 0, c, 10.0, src, 2, c_max=C_MAX)

    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            return list(ex.map(one, range(nshots)))
    return [one(i) for i in range(nshots)]


# --------------------------------------------------------------------------- Laplace-operator workload

@dataclass
class DiffWorkload:
    """Input of the explicit-diffusion sweep (the paper's Laplace-operator
    workload): grid, spacing, time step, diffusivity, order, steps and the
    initial field (float32)."""
    name: str
    shape: tuple
    spacing: tuple
    dt: float
    alpha: float
    so: int
    nt: int
    u0: np.ndarray

    @property
    def npts(self):
        return int(np.prod(self.shape))


def laplace_field(shape, seed: int) -> np.ndarray:
    """Deterministic initial field: a ramp from 1 to 2 over the points in
    row-major order (the paper's operator listing fills its grid the same
    way) plus seeded N(0, 0.1^2) noise, so that every point and every tile
    carries its own values.  float32."""
    n = int(np.prod(shape))
    ramp = np.linspace(1.0, 2.0, num=n).reshape(shape)
    rng = np.random.default_rng(seed)
    return (ramp + 0.1 * rng.standard_normal(shape)).astype(np.float32)


def laplace(n: int = 500, so: int = 8, nt: int = 32, seed: int = 6, shape=None) -> DiffWorkload:
    """The Laplace-operator workload of the evaluation chapter: an n^3 grid
    (500^3 x 32 steps and 600^3 x 16 steps there) at space order so, unit
    spacing and diffusivity.  The time step is 0.9 of 2 h^2 / (a d pi^2),
    below the stability limit of every order (the symbol of a centred second
    difference never exceeds pi^2 / h^2 in magnitude), so the field cannot
    diverge."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    nd = len(shape)
    h, a = 1.0, 1.0
    dt = 0.9 * 2.0 * h * h / (a * nd * math.pi ** 2)
    if len(set(shape)) == 1:
        name = "laplace_%dcube_so%d" % (shape[0], so)
    else:
        name = "laplace_%s_so%d" % ("x".join(map(str, shape)), so)
    return DiffWorkload(name, shape, (h,) * nd, dt, a, so, nt, laplace_field(shape, seed))
