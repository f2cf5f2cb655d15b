"""Seeded synthetic inputs shared by the oracle-side and the GPU-side of every test and benchmark.

This module holds none of the method's arithmetic: it only draws random numbers and lays them out
as point clouds {x, y, z, a} (metres; x, y relative to the centre of global pixel (0, 0)) plus the
parameters of each workload.  The paper's 95,949-point object is not public, so every workload is a
synthetic stand-in with the sizes of the paper's experiment or of the measured configurations.

Point positions for the wavelet path are drawn on the 2^L pixel grid (the level-scaled shift of
Eq.(2) is an integer only there); depths and amplitudes are continuous.
"""
from __future__ import annotations

import numpy as np

PITCH = 1e-6          # hologram sampling pitch (Sec. 3: 1 um)
WAVELENGTH = 633e-9   # He-Ne line; the paper's reconstruction light is 632.8 nm (Sec. 3)


def uniform_points(seed: int, n: int, nx: int, ny: int, z_lo: float, z_hi: float,
                   pitch: float = PITCH) -> np.ndarray:
    """x, y uniform over the hologram area, z ~ U[z_lo, z_hi], a ~ U[0, 1) (continuous)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, nx * pitch, n)
    y = rng.uniform(0.0, ny * pitch, n)
    z = rng.uniform(z_lo, z_hi, n)
    a = rng.uniform(0.0, 1.0, n)
    return np.stack([x, y, z, a], axis=1)


def grid_points(seed: int, n: int, nx: int, ny: int, grid: int, z_lo: float, z_hi: float,
                pitch: float = PITCH, x0: int = 0, y0: int = 0) -> np.ndarray:
    """x, y uniform over the multiples of `grid` pixels inside [x0, x0+nx) x [y0, y0+ny)."""
    rng = np.random.default_rng(seed)
    gx = rng.integers(0, max(nx // grid, 1), n)
    gy = rng.integers(0, max(ny // grid, 1), n)
    z = rng.uniform(z_lo, z_hi, n)
    a = rng.uniform(0.0, 1.0, n)
    return np.stack([(x0 + gx * grid) * pitch, (y0 + gy * grid) * pitch, z, a], axis=1)


def height_field_points(seed: int, n: int, nw: int, grid: int, z_lo: float, z_hi: float,
                        pitch: float = PITCH, n_waves: int = 16) -> np.ndarray:
    """Points on a smooth random surface: z = H(x, y) with H a sum of 16 random plane waves
    (spatial frequency up to 4 cycles per aperture), min-max scaled to [z_lo, z_hi]."""
    rng = np.random.default_rng(seed)
    gx = rng.integers(0, nw // grid, n)
    gy = rng.integers(0, nw // grid, n)
    fx = rng.uniform(-4.0, 4.0, n_waves)
    fy = rng.uniform(-4.0, 4.0, n_waves)
    ph = rng.uniform(0.0, 2 * np.pi, n_waves)
    a = rng.uniform(0.0, 1.0, n)
    xs = (gx * grid).astype(np.float64)
    ys = (gy * grid).astype(np.float64)
    h = np.zeros(n)
    for k in range(n_waves):
        h += np.cos(2 * np.pi * (fx[k] * xs + fy[k] * ys) / nw + ph[k])
    h = (h - h.min()) / max(h.max() - h.min(), 1e-300)
    z = z_lo + h * (z_hi - z_lo)
    return np.stack([xs * pitch, ys * pitch, z, a], axis=1)


# Workload parameter records (sizes of the measured configurations).
DIRECT_512 = dict(name="direct-512x512-n1000", nx=512, ny=512, n=1000, z_lo=0.1e-3, z_hi=1.0e-3,
                  seed=0)
WASABI_2048 = dict(name="wasabi-2048x2048-n10000-L3-64planes", nx=2048, ny=2048, n=10_000,
                   z_lo=0.1e-3, z_hi=1.5e-3, n_depth=64, levels=3, gamma=0.05, max_window=1024,
                   seed=0)
WASABI_65536 = dict(name="wasabi-65536x65536-n1e6-L4-256planes", nx=65536, ny=65536,
                    n=1_000_000, z_lo=0.1e-3, z_hi=1.5e-3, n_depth=256, levels=4, gamma=0.02,
                    max_window=1024, seed=0)
WASABI_16384 = dict(name="wasabi-16384x16384-n2e5-L3-64planes", nx=16384, ny=16384, n=200_000,
                    z_lo=0.1e-3, z_hi=1.5e-3, n_depth=64, levels=3, gamma=0.05, max_window=1024,
                    seed=0)


def serve_specs(seed: int, n_jobs: int, sizes=(1024, 2048, 4096, 8192), median_n: float = 20_000,
                sigma: float = 1.0, n_lo: int = 1000, n_hi: int = 200_000):
    """Job mix of the serving workload: hologram side uniform over `sizes`, N log-normal with the
    given median and sigma, clipped to [n_lo, n_hi].  Returns (side, n, point_seed) per job."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_jobs):
        side = int(rng.choice(sizes))
        n = int(np.clip(np.exp(rng.normal(np.log(median_n), sigma)), n_lo, n_hi))
        out.append((side, n, seed * 1_000_003 + i + 1))
    return out


def serve_points(spec, grid: int = 8, z_lo: float = 0.1e-3, z_hi: float = 1.5e-3) -> np.ndarray:
    """Points of one serving job: on the 2^L grid inside the job's own hologram, z uniform."""
    side, n, pseed = spec
    return grid_points(pseed, n, side, side, grid, z_lo, z_hi)


def poisson_arrivals(seed: int, n_jobs: int, rate_per_s: float) -> np.ndarray:
    """Arrival times (s) of a Poisson stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n_jobs))
