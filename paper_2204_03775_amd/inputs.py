"""Seeded synthetic inputs for the wave propagator.

This module only *generates inputs*: velocity models, source wavelets,
source/receiver positions and time steps.  It holds none of the propagator's
arithmetic and imports neither the HIP library nor the oracle, so both sides
of every parity check read exactly the same inputs from here.

The paper runs on synthetic grids whose velocity model it does not state
(Section V-B, Tables 2 and 3); the workloads here are synthetic too:

* ``small_parity``: 64^3, constant 1500 m/s, h = 10 m, dt = 1 ms, 100 steps,
  15 Hz Ricker at the centre, 16 seeded random receivers, zero ghost layer,
  no sponge.
* ``large_shot``: 512^3, h = 10 m, dt = 0.8 of the stability limit at
  4500 m/s, 1000 steps, five equal layers 1500..4500 m/s times
  (1 + 0.05 p) with p Gaussian-smoothed white noise scaled to max |p| = 1,
  20-cell sponge, 12 Hz Ricker near the top, 256 receivers on a line.
* ``batch_shots``: 32 shots (seed 2207) on uneven grids, nx, ny drawn from
  96..320 and nz from 96..256 (multiples of 16), each with 3..6 layers of
  sorted velocities drawn from 1500..4500 m/s, a 10..20 Hz Ricker at least
  25 cells from every face, 20-cell sponge, 128 receivers on the z = 22
  line; common dt (0.8 of the limit at 4500 m/s), 600 steps.
* ``crop_shot``: the 128^3 block z 0:128, y 192:320, x 192:320 of the
  large-shot model, its own 20-cell sponge, 500 steps, source at
  (25, 64, 64), 88 receivers at z = 22, y = 64, x = 20..107 (accuracy of
  the reduced-precision storage forms).
* ``gradient_shot``: 256^3, 800 steps, five equal layers 1500..4500 m/s
  (no noise) for the observed data; the evaluation model adds a Gaussian
  anomaly of +5 % (sigma 8 cells) centred at a point drawn (seed 2208) with
  depth in [n/5, 2n/5) and y, x in the middle third; 20-cell sponge, 12 Hz
  Ricker at
  (25, 128, 128), 128 receivers at z = 22, y = 128, x = 20..235;
  checkpoints every 50 steps (gradient of the least-squares misfit).
* ``paper_shape``: the paper's largest Table 2 shape, 755 x 994 x 1000
  (x, y, z), 1000 steps, constant 1500 m/s (its model is not stated), no
  sponge: a context run for the paper's cell-rate figures.
* ``gradient_crop``: the 48^3 block of both models centred on the anomaly,
  8-cell sponge (alpha 0.04), 300 steps, source at (12, 24, 24),
  28 receivers at z = 10, y = 24, x = 10..37 (checks of the gradient).

Random draws use ``numpy.random.default_rng(2204 + i)`` for workload i.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Maximum of the 8th-order second-derivative symbol |c_0 + 2 sum c_m cos(m pi)|
# (reached at the Nyquist wavenumber), used only to pick a stable dt.
SYMBOL_MAX = 2048.0 / 315.0


def stable_courant_limit(ndim: int = 3) -> float:
    """Largest v*dt/h for which leapfrog with this stencil stays stable on a
    cubic grid: k * ndim * SYMBOL_MAX / h^2 <= 4."""
    return 2.0 / math.sqrt(ndim * SYMBOL_MAX)


def cfl_dt(vmax: float, h: float, fraction: float = 0.8) -> float:
    return fraction * stable_courant_limit(3) * h / vmax


def ricker(freq: float, nt: int, dt: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet w(t_n), t_n = n dt, peak at t0 (default 1/freq)."""
    t0 = 1.0 / freq if t0 is None else t0
    tau = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * freq * tau) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def point_source_values(w: np.ndarray, v_src: float, dt: float, h) -> np.ndarray:
    """Values added to the source cell per step: dt^2 V^2 f with f a point
    source of time function w spread over one cell (1/(dx dy dz))."""
    dx, dy, dz = h
    return (v_src * dt) ** 2 * np.asarray(w, dtype=np.float64) / (dx * dy * dz)


def layered_velocity(nz: int, ny: int, nx: int, velocities, *, perturb: float = 0.0,
                     sigma: float = 4.0, seed: int = 0) -> np.ndarray:
    """Equal-thickness layers along z (top to bottom) times (1 + perturb * p),
    p = white noise smoothed by a separable Gaussian and scaled to max|p| = 1.
    Returned as float32 [nz][ny][nx] (large grids); values are exact to
    float32 rounding of the FP64 construction per layer."""
    vel = np.asarray(velocities, dtype=np.float64)
    nl = len(vel)
    layer = np.minimum((np.arange(nz) * nl) // nz, nl - 1)
    vz = vel[layer].astype(np.float32)
    v = np.empty((nz, ny, nx), dtype=np.float32)
    v[...] = vz[:, None, None]
    if perturb:
        p = smoothed_noise((nz, ny, nx), sigma, seed)
        v *= (1.0 + perturb * p).astype(np.float32)
    return v


def smoothed_noise(shape, sigma: float, seed: int) -> np.ndarray:
    from scipy.ndimage import gaussian_filter1d

    rng = np.random.default_rng(seed)
    p = rng.standard_normal(shape, dtype=np.float32)
    for ax in range(3):
        p = gaussian_filter1d(p, sigma, axis=ax, mode="nearest", truncate=4.0)
    p /= np.float32(np.max(np.abs(p)))
    return p


def random_receivers(shape, n: int, seed: int) -> np.ndarray:
    """n distinct interior points drawn without replacement; [n][3] (z, y, x)."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    flat = rng.choice(nz * ny * nx, size=n, replace=False)
    z, y, x = np.unravel_index(flat, (nz, ny, nx))
    return np.stack([z, y, x], axis=1).astype(np.int32)


def line_receivers(z: int, y: int, x0: int, x1: int, n: int) -> np.ndarray:
    xs = [x0 + int(round(r * (x1 - x0) / (n - 1))) for r in range(n)]
    return np.array([[z, y, x] for x in xs], dtype=np.int32)


@dataclass
class Problem:
    """One forward run: grid, physics, source, receivers and model."""

    name: str
    nx: int
    ny: int
    nz: int
    h: tuple
    dt: float
    nt: int
    sponge_width: int
    sponge_alpha: float
    src: tuple
    rec: np.ndarray
    s: np.ndarray            # [nt] FP64 value added to the source cell per step
    v: np.ndarray = field(repr=False)   # [nz][ny][nx] velocity (float32 or float64)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def points(self) -> int:
        return self.nx * self.ny * self.nz

    def k64(self) -> np.ndarray:
        """V^2 dt^2 per cell, FP64."""
        v = self.v.astype(np.float64)
        return (v * self.dt) ** 2

    def k32(self) -> np.ndarray:
        """V^2 dt^2 per cell rounded once to FP32."""
        return self.k64().astype(np.float32)


def small_parity() -> Problem:
    n = 64
    h = (10.0, 10.0, 10.0)
    dt, nt = 1e-3, 100
    v = np.full((n, n, n), 1500.0, dtype=np.float64)
    src = (n // 2, n // 2, n // 2)
    w = ricker(15.0, nt, dt)
    return Problem("small_parity", n, n, n, h, dt, nt, 0, 0.0, src,
                   random_receivers((n, n, n), 16, 2204),
                   point_source_values(w, 1500.0, dt, h), v)


def large_shot(n: int = 512, nt: int = 1000) -> Problem:
    h = (10.0, 10.0, 10.0)
    dt = cfl_dt(4500.0, 10.0, 0.8)
    v = large_model(n)
    src = (25, n // 2, n // 2)
    w = ricker(12.0, nt, dt)
    rec = line_receivers(22, n // 2, 20, n - 21, 256)
    return Problem("large_shot", n, n, n, h, dt, nt, 20, 0.015, src, rec,
                   point_source_values(w, float(v[src]), dt, h), v)


_LARGE_MODEL = {}


def large_model(n: int = 512) -> np.ndarray:
    """The large-shot velocity model (cached: generating 512^3 takes seconds)."""
    if n not in _LARGE_MODEL:
        _LARGE_MODEL[n] = layered_velocity(n, n, n, [1500.0, 2250.0, 3000.0, 3750.0, 4500.0],
                                           perturb=0.05, sigma=4.0, seed=2205)
    return _LARGE_MODEL[n]


def crop_shot(nt: int = 500) -> Problem:
    h = (10.0, 10.0, 10.0)
    dt = cfl_dt(4500.0, 10.0, 0.8)
    v = np.ascontiguousarray(large_model()[0:128, 192:320, 192:320])
    src = (25, 64, 64)
    w = ricker(12.0, nt, dt)
    rec = np.array([[22, 64, x] for x in range(20, 108)], dtype=np.int32)
    return Problem("crop_shot", 128, 128, 128, h, dt, nt, 20, 0.015, src, rec,
                   point_source_values(w, float(v[src]), dt, h), v)


def batch_shots(n: int = 32, nt: int = 600, seed: int = 2207) -> list:
    rng = np.random.default_rng(seed)
    h = (10.0, 10.0, 10.0)
    dt = cfl_dt(4500.0, 10.0, 0.8)
    W = 20
    shots = []
    for i in range(n):
        nx, ny = (int(16 * round(rng.integers(96, 321) / 16)) for _ in range(2))
        nz = int(16 * round(rng.integers(96, 257) / 16))
        nl = int(rng.integers(3, 7))
        vel = np.sort(rng.uniform(1500.0, 4500.0, size=nl))
        layer = np.minimum((np.arange(nz) * nl) // nz, nl - 1)
        v = np.empty((nz, ny, nx), dtype=np.float32)
        v[...] = vel[layer].astype(np.float32)[:, None, None]
        m = W + 5
        src = tuple(int(rng.integers(m, d - m)) for d in (nz, ny, nx))
        f = float(rng.uniform(10.0, 20.0))
        xs = np.linspace(m, nx - 1 - m, 128).round().astype(np.int32)
        rec = np.stack([np.full(128, 22), np.full(128, ny // 2), xs], axis=1).astype(np.int32)
        w = ricker(f, nt, dt)
        shots.append(Problem(f"shot{i}_{nx}x{ny}x{nz}", nx, ny, nz, h, dt, nt, W, 0.015, src, rec,
                             point_source_values(w, float(v[src]), dt, h), v))
    return shots


def random_problem(nx: int, ny: int, nz: int, nt: int, *, seed: int, h=(10.0, 12.0, 8.0),
                   sponge_width: int = 0, sponge_alpha: float = 0.015, nrec: int = 8,
                   vmin: float = 1500.0, vmax: float = 3500.0, freq: float = 25.0,
                   courant: float = 0.6) -> Problem:
    """Small heterogeneous problem for edge-case parity: anisotropic spacing,
    random smooth-free velocities, source and receivers anywhere inside."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(vmin, vmax, size=(nz, ny, nx))
    # stable for anisotropic spacing: k * SYMBOL_MAX * sum(1/h^2) <= 4
    lim = 2.0 / math.sqrt(SYMBOL_MAX * sum(1.0 / hh ** 2 for hh in h))
    dt = courant * lim / vmax
    src = tuple(int(rng.integers(0, d)) for d in (nz, ny, nx))
    npts = nx * ny * nz
    rec = random_receivers((nz, ny, nx), min(nrec, npts), seed + 1)
    w = ricker(freq, nt, dt, t0=1.2 / freq)
    return Problem(f"random_{nx}x{ny}x{nz}", nx, ny, nz, tuple(h), dt, nt, sponge_width,
                   sponge_alpha, src, rec, point_source_values(w, float(v[src]), dt, h), v)


@dataclass
class GradientProblem:
    """A shot in an evaluation model (``shot.v``) with data observed in
    another model (``v_obs``); the gradient is that of the least-squares
    misfit 0.5 || traces(v) - traces(v_obs) ||^2 with respect to k."""

    shot: Problem
    v_obs: np.ndarray = field(repr=False)
    every: int
    anomaly: tuple

    def observed(self) -> Problem:
        p = self.shot
        return Problem(p.name + "_obs", p.nx, p.ny, p.nz, p.h, p.dt, p.nt, p.sponge_width,
                       p.sponge_alpha, p.src, p.rec, p.s, self.v_obs)


_GRAD_MODELS = {}


def gradient_models(n: int = 256):
    """(layered model, model with the anomaly, anomaly centre), float32."""
    if n not in _GRAD_MODELS:
        base = layered_velocity(n, n, n, [1500.0, 2250.0, 3000.0, 3750.0, 4500.0])
        rng = np.random.default_rng(2208)
        # depth in [n/5, 2n/5): within reach of the surface receivers in 800
        # steps (drawn from the middle third, the anomaly's scattering reaches
        # them only in the record's last quarter, at 4e-7 of the trace
        # amplitude: below FP32 rounding); y and x in the middle third
        c = (int(rng.integers(n // 5, 2 * n // 5)),
             int(rng.integers(n // 3, 2 * n // 3)), int(rng.integers(n // 3, 2 * n // 3)))
        z, y, x = np.ogrid[:n, :n, :n]
        r2 = (z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2
        bump = np.exp(-r2 / (2.0 * 8.0 ** 2))
        ev = (base.astype(np.float64) * (1.0 + 0.05 * bump)).astype(np.float32)
        _GRAD_MODELS[n] = (base, ev, c)
    return _GRAD_MODELS[n]


def gradient_shot(n: int = 256, nt: int = 800, every: int = 50) -> GradientProblem:
    h = (10.0, 10.0, 10.0)
    dt = cfl_dt(4500.0, 10.0, 0.8)
    base, ev, c = gradient_models(n)
    src = (25, n // 2, n // 2)
    w = ricker(12.0, nt, dt)
    rec = line_receivers(22, n // 2, 20, n - 21, 128)
    shot = Problem("gradient_shot", n, n, n, h, dt, nt, 20, 0.015, src, rec,
                   point_source_values(w, float(ev[src]), dt, h), ev)
    return GradientProblem(shot, base, every, c)


def gradient_crop(nt: int = 300, m: int = 48) -> GradientProblem:
    h = (10.0, 10.0, 10.0)
    dt = cfl_dt(4500.0, 10.0, 0.8)
    base, ev, c = gradient_models()
    sl = tuple(slice(ci - m // 2, ci - m // 2 + m) for ci in c)
    vb = np.ascontiguousarray(base[sl])
    ve = np.ascontiguousarray(ev[sl])
    src = (12, m // 2, m // 2)
    w = ricker(12.0, nt, dt)
    rec = np.array([[10, m // 2, x] for x in range(10, m - 10)], dtype=np.int32)
    shot = Problem("gradient_crop", m, m, m, h, dt, nt, 8, 0.04, src, rec,
                   point_source_values(w, float(ve[src]), dt, h), ve)
    return GradientProblem(shot, vb, 50, tuple(m // 2 for _ in range(3)))


# Grid shapes of the paper's scaling experiments (x, y, z): Table 2 grows
# x and y at nz = 1000, Table 3 grows nz at 755 x 994.
PAPER_TABLE2_SHAPES = ((200, 200, 1000), (400, 400, 1000), (600, 600, 1000),
                       (755, 500, 1000), (755, 600, 1000), (755, 900, 1000),
                       (755, 990, 1000), (755, 994, 1000))
PAPER_TABLE3_SHAPES = tuple((755, 994, nz) for nz in (100, 200, 300, 400, 500, 700, 1000))


def paper_shape(nt: int = 1000, nx: int = 755, ny: int = 994, nz: int = 1000) -> Problem:
    """A grid shape of the paper's scaling experiments (default: the largest
    Table 2 shape, 755 x 994 x 1000) with nt steps, in a constant 1500 m/s
    medium (the paper does not state its model): h = 10 m, dt = 0.8 of the
    stability limit, zero ghost layer, no sponge, 15 Hz Ricker at the centre,
    up to 256 receivers on a line.  Context runs for a like-for-like cell
    rate against the paper's figures.  ``v`` is a read-only broadcast view
    (no dense copy)."""
    h = (10.0, 10.0, 10.0)
    dt = cfl_dt(1500.0, 10.0, 0.8)
    v = np.broadcast_to(np.float32(1500.0), (nz, ny, nx))
    src = (nz // 2, ny // 2, nx // 2)
    x0, x1 = 20, nx - 21
    rec = line_receivers(max(0, nz // 2 - 20), ny // 2, x0, x1, min(256, x1 - x0 + 1))
    w = ricker(15.0, nt, dt)
    return Problem("paper_shape", nx, ny, nz, h, dt, nt, 0, 0.0, src, rec,
                   point_source_values(w, 1500.0, dt, h), v)
