"""Seeded synthetic inputs: velocity models, wavelets, acquisition geometry.

This module holds none of the wave-propagation arithmetic.  It only draws
inputs, so it may feed both the HIP library and the independent CPU oracle.
No public dataset is involved: every model is generated from a seed.

Workloads (shapes and value distributions of the paper's setting, a 3-D
acoustic medium sampled on a regular grid, Sections 3-4):

* ``anomaly_2d`` -- 2-D 128x128, dx 10 m, 2000 m/s plus a +300 m/s Gaussian anomaly
  (sigma 8 cells) at the centre, dt 1 ms, 500 steps, 20-cell sponge, 15 Hz
  Ricker at (z 4, x 64), 128 receivers on row 4.
* ``layered_3d`` -- 3-D 256^3, dx 10 m, layered (8-12 layers, 1500-4500 m/s, 5 %
  multiplicative noise), dt from CFL 0.4, 2000 steps, 24-cell sponge, 10 Hz
  Ricker at (4, 128, 128), 256x256 receivers on z 4.
* ``shots_2d`` -- 2-D 1024x320 (x by z), dx 12.5 m, smooth random truth in
  1500-4500 m/s and a smoothed (sigma 20) start model, 32 shots, 3000 steps,
  8 Hz Ricker, 1024 receivers, every-50 checkpoints.
* ``serve.make_stream`` -- a Poisson stream of mixed 2-D / 3-D forward and
  gradient requests.
* ``salt_3d`` -- 3-D 512x512x256 (x, y, z), dx 10 m, layers plus an ellipsoidal
  4500 m/s salt body, 3000 steps, revolve under a 40 GB wavefield budget,
  512x512 receivers; the oracle comparison runs on a 64^3 crop.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


# ---------------------------------------------------------------- wavelets
def ricker(f: float, nt: int, dt: float, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet samples w[n] = w(n dt), unit peak at t0 (default 1.5 / f)."""
    if t0 is None:
        t0 = 1.5 / f
    t = np.arange(nt) * dt - t0
    a = (np.pi * f * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float64)


# ---------------------------------------------------------- time step, sponge
def dt_from_cfl(vmax: float, dx: float, cfl: float = 0.4) -> float:
    return cfl * dx / vmax


def default_eta_max(vmax: float, nb: int, dx: float, reflection: float = 1e-3) -> float:
    """Peak sponge damping rate (1/s) for a quadratic profile of nb cells.

    The usual choice 3 vmax ln(1/R) / (2 nb dx) for a target reflection R.
    """
    if nb <= 0:
        return 0.0
    return 3.0 * vmax * math.log(1.0 / reflection) / (2.0 * nb * dx)


# ------------------------------------------------------------------ models
def gaussian_anomaly_2d(nz=128, nx=128, v0=2000.0, dv=300.0, sigma=8.0, centre=(64, 64)):
    z = np.arange(nz)[:, None] - centre[0]
    x = np.arange(nx)[None, :] - centre[1]
    return v0 + dv * np.exp(-(z * z + x * x) / (2.0 * sigma * sigma))


def layered(shape, rng, vmin=1500.0, vmax=4500.0, nlayers=None, noise=0.05):
    """Flat layers along axis 0 (depth): 8-12 interfaces at sorted uniform depths,
    velocities uniform in [vmin, vmax] sorted increasing with depth, times
    (1 + N(0, noise^2)) i.i.d. per cell."""
    nz = shape[0]
    if nlayers is None:
        nlayers = int(rng.integers(8, 13))
    depths = np.sort(rng.integers(1, nz, size=nlayers - 1))
    vel = np.sort(rng.uniform(vmin, vmax, size=nlayers))
    prof = np.empty(nz)
    layer = np.searchsorted(depths, np.arange(nz), side="right")
    prof[:] = vel[layer]
    v = np.broadcast_to(prof.reshape((nz,) + (1,) * (len(shape) - 1)), shape).copy()
    if noise:
        v *= 1.0 + noise * rng.standard_normal(shape)
    return v


def smooth_random_2d(nz, nx, rng, sigma=10.0, vmin=1500.0, vmax=4500.0):
    from scipy.ndimage import gaussian_filter
    a = gaussian_filter(rng.standard_normal((nz, nx)), sigma, mode="wrap")
    a = (a - a.min()) / (a.max() - a.min())
    return vmin + (vmax - vmin) * a


def smooth(v, sigma):
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(v, sigma, mode="nearest")


def salt_model(shape, rng, centre, semi_axes, v_salt=4500.0, vmin=1500.0, vmax=3500.0):
    v = layered(shape, rng, vmin, vmax, noise=0.0)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    r2 = sum(((g - c) / a) ** 2 for g, c, a in zip(grids, centre, semi_axes))
    v[r2 <= 1.0] = v_salt
    return v


# ---------------------------------------------------------------- geometry
def surface_receivers(model_shape, depth, stride=1):
    """Receivers on the plane (or row) z = depth, every `stride` cells."""
    if len(model_shape) == 2:
        x = np.arange(0, model_shape[1], stride)
        return np.stack([np.full_like(x, depth), x], axis=1).astype(np.int32)
    y, x = np.meshgrid(np.arange(0, model_shape[1], stride),
                       np.arange(0, model_shape[2], stride), indexing="ij")
    return np.stack([np.full(y.size, depth), y.ravel(), x.ravel()], axis=1).astype(np.int32)


# ---------------------------------------------------------------- problems
@dataclasses.dataclass
class Problem:
    """One synthetic workload: everything both sides need, as NumPy arrays."""
    name: str
    v: np.ndarray            # model velocity [nz][nx] or [nz][ny][nx], float64
    dx: float
    dt: float
    nt: int
    order: int
    nb: int
    eta_max: float
    wavelet: np.ndarray      # [S][nt] float64
    src_pos: np.ndarray      # [S][D] int32
    rec_pos: np.ndarray      # [S][R][D] int32
    v_start: Optional[np.ndarray] = None   # start model for gradient workloads
    ckpt: str = "all"

    @property
    def ndim(self):
        return self.v.ndim

    @property
    def nshots(self):
        return self.src_pos.shape[0]

    @property
    def nrec(self):
        return self.rec_pos.shape[1]

    @property
    def padded_cells(self):
        return int(np.prod([n + 2 * self.nb for n in self.v.shape]))

    @property
    def model_cells(self):
        return int(self.v.size)


def _pack(name, v, dx, dt, nt, order, nb, f, src_pos, rec_pos, eta_max=None, **kw):
    src_pos = np.asarray(src_pos, dtype=np.int32).reshape(-1, v.ndim)
    S = src_pos.shape[0]
    rec_pos = np.asarray(rec_pos, dtype=np.int32)
    if rec_pos.ndim == 2:
        rec_pos = np.broadcast_to(rec_pos, (S,) + rec_pos.shape).copy()
    w = np.broadcast_to(ricker(f, nt, dt), (S, nt)).copy()
    if eta_max is None:
        eta_max = default_eta_max(float(np.max(v)), nb, dx)
    return Problem(name, np.asarray(v, dtype=np.float64), float(dx), float(dt), int(nt),
                   int(order), int(nb), float(eta_max), w, src_pos, rec_pos, **kw)


def anomaly_2d(nt=500, order=8):
    v = gaussian_anomaly_2d()
    rec = surface_receivers(v.shape, 4)
    return _pack("anomaly-2d-128x128-nt%d" % nt, v, 10.0, 1e-3, nt, order, 20, 15.0,
                 [[4, 64]], rec)


def layered_3d(nt=2000, order=8, n=256, seed=2):
    rng = np.random.default_rng(seed)
    v = layered((n, n, n), rng)
    dt = dt_from_cfl(float(v.max()), 10.0, 0.4)
    rec = surface_receivers(v.shape, 4)
    return _pack("layered-3d-%d^3-nt%d" % (n, nt), v, 10.0, dt, nt, order, 24, 10.0,
                 [[4, n // 2, n // 2]], rec)


def slab_3d(nt=200, order=8, seed=6, shape=(128, 1024, 1024)):
    """One GPU's share of a 1024^3 layered model split into 8 slabs along z
    (128 x 1024 x 1024 cells).  No sponge: the zero frame stands in for the
    ghost planes a neighbouring slab would send.  Receivers every 4th cell at
    z = 4, source at the top centre."""
    rng = np.random.default_rng(seed)
    v = layered(shape, rng)
    dt = dt_from_cfl(float(v.max()), 10.0, 0.4)
    nz, ny, nx = shape
    rec = surface_receivers(shape, 4, stride=4)
    return _pack("slab-3d-%dx%dx%d-nt%d" % (nz, ny, nx, nt), v, 10.0, dt, nt, order, 0, 10.0,
                 [[4, ny // 2, nx // 2]], rec)


def shots_2d(nt=3000, order=8, nshots=32, seed=3, nz=320, nx=1024):
    rng = np.random.default_rng(seed)
    truth = smooth_random_2d(nz, nx, rng)
    start = smooth(truth, 20.0)
    spacing = nx // nshots
    src = [[4, spacing // 2 + spacing * i] for i in range(nshots)]
    rec = surface_receivers(truth.shape, 4)
    return _pack("shots-2d-%dx%d-%dshots-nt%d" % (nx, nz, nshots, nt), truth, 12.5, 1e-3,
                 nt, order, 20, 8.0, src, rec, v_start=start, ckpt="every:50")


def salt_3d(nt=3000, order=8, seed=5, shape=(256, 512, 512)):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    centre = (160 * nz // 256, ny // 2, nx // 2)
    semi = (48 * nz // 256, 96 * ny // 512, 96 * nx // 512)
    v = salt_model(shape, rng, centre, semi)
    dt = dt_from_cfl(4500.0, 10.0, 0.4)
    rec = surface_receivers(v.shape, 4)
    return _pack("salt-3d-%dx%dx%d-nt%d" % (nx, ny, nz, nt), v, 10.0, dt, nt, order, 24,
                 10.0, [[4, ny // 2, nx // 2]], rec, v_start=smooth(v, 8.0),
                 ckpt="revolve:40e9")


def salt_3d_crop(nt=3000, order=8, seed=5):
    """64^3 crop of the salt_3d model straddling the salt top (z 80-143,
    y/x 224-287), with its own sponge, centred source and 64x64 receivers."""
    full = salt_3d(nt=1, order=order, seed=seed)
    v = full.v[80:144, 224:288, 224:288].copy()
    rec = surface_receivers(v.shape, 4)
    dt = full.dt
    return _pack("saltcrop-3d-64^3-nt%d" % nt, v, 10.0, dt, nt, order, 24, 10.0,
                 [[4, 32, 32]], rec, eta_max=default_eta_max(4500.0, 24, 10.0),
                 v_start=smooth(v, 4.0), ckpt="revolve:0")


def small_2d(nz=37, nx=150, nt=120, order=8, nb=6, seed=11, nshots=1, nrec=23):
    """Ragged small 2-D case: several tiles in x with a tail, random velocity."""
    rng = np.random.default_rng(seed)
    v = 1800.0 + 900.0 * smooth(rng.random((nz, nx)), 2.0)
    dt = dt_from_cfl(float(v.max()), 10.0, 0.35)
    src = np.stack([rng.integers(0, nz, nshots), rng.integers(0, nx, nshots)], axis=1)
    rec = np.stack([rng.integers(0, nz, (nshots, nrec)), rng.integers(0, nx, (nshots, nrec))],
                   axis=2)
    return _pack("small2d-%dx%d" % (nx, nz), v, 10.0, dt, nt, order, nb, 25.0, src, rec)


def small_3d(shape=(21, 19, 70), nt=60, order=8, nb=5, seed=12, nshots=1, nrec=17):
    rng = np.random.default_rng(seed)
    v = 1800.0 + 900.0 * smooth(rng.random(shape), 1.5)
    dt = dt_from_cfl(float(v.max()), 10.0, 0.35)
    src = np.stack([rng.integers(0, n, nshots) for n in shape], axis=1)
    rec = np.stack([rng.integers(0, n, (nshots, nrec)) for n in shape], axis=2)
    return _pack("small3d-%dx%dx%d" % shape[::-1], v, 10.0, dt, nt, order, nb, 25.0,
                 src, rec)
