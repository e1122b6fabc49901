"""Seeded synthetic workloads shaped like the paper's 2D benchmarks.

Velocity nodes (section 3.1, discrete velocity model): the box [-L, L]^d is
covered by N nodes per axis, v_i = -L + i * (2L/N), i = 0..N-1, so the grid is
periodic with period 2L (the reading used throughout this project).

Distribution functions are stored cell-major, f[cells][N]*d, with the last
velocity axis fastest.

Random draws per cell (vectorised over cells, in this order):
  rho  ~ U[0.5, 2]        shape (cells, 2)
  T    ~ U[0.5, 1.5]      shape (cells, 2)
  |u| = 0.5 * U^(1/d)     shape (cells, 2)
  direction of u: uniform on the circle (d=2, one angle) or sphere (d=3,
  normalised Gaussian triple), shape (cells, 2, ...)
f is the sum of the two Maxwellians of eq. (M), evaluated in float64 at the
nodes; callers cast to float32 for the GPU path.
"""

from __future__ import annotations

import math

import numpy as np

# Workloads (sizes follow the paper's velocity grids and cell counts).
CONFIGS = {
    "bkw16": dict(d=2, N=16, L=8.0, kernel="maxwell", M=16, cells=1, seed=1000),
    "hs2d_32": dict(d=2, N=32, L=8.0, kernel="hard_sphere", M=8, cells=4096, seed=1001),
    "maxwell2d_32": dict(d=2, N=32, L=8.0, kernel="maxwell", M=8, cells=4096, seed=1001),
    "hs2d_64_noisy": dict(d=2, N=64, L=10.0, kernel="hard_sphere", M=16, cells=20000,
                          seed=1002, noise=0.01),
    "hs3d_32": dict(d=3, N=32, L=8.0, kernel="hard_sphere", M=32, cells=8192, seed=1004),
    "hs3d_16": dict(d=3, N=16, L=8.0, kernel="hard_sphere", M=32, cells=8192, seed=1005),
}


def velocity_nodes(N: int, L: float) -> np.ndarray:
    """1-D node coordinates v_i = -L + i*2L/N (float64)."""
    return -L + np.arange(N, dtype=np.float64) * (2.0 * L / N)


def _grid(d: int, N: int, L: float):
    v = velocity_nodes(N, L)
    return np.meshgrid(*([v] * d), indexing="ij")


def maxwellian(d: int, N: int, L: float, rho, u, T) -> np.ndarray:
    """Maxwellian of eq. (M) with theta = T (gas constant 1) on the node grid.

    rho, T: arrays of shape (C,); u: shape (C, d). Returns (C, N, ..., N) float64.
    """
    rho = np.asarray(rho, dtype=np.float64).reshape(-1)
    T = np.asarray(T, dtype=np.float64).reshape(-1)
    u = np.asarray(u, dtype=np.float64).reshape(-1, d)
    g = _grid(d, N, L)
    shape = (-1,) + (1,) * d
    r2 = 0.0
    for a in range(d):
        r2 = r2 + (g[a][None] - u[:, a].reshape(shape)) ** 2
    norm = rho.reshape(shape) / (2.0 * math.pi * T.reshape(shape)) ** (d / 2.0)
    return norm * np.exp(-r2 / (2.0 * T.reshape(shape)))


def bkw_initial(N: int, L: float) -> np.ndarray:
    """BKW datum at t = 0 (S = 1/2): f0(v) = |v|^2 exp(-|v|^2) / pi, d = 2."""
    g = _grid(2, N, L)
    r2 = g[0] ** 2 + g[1] ** 2
    return (r2 * np.exp(-r2) / math.pi)[None]


def _ball(rng, cells: int, d: int) -> np.ndarray:
    r = 0.5 * rng.uniform(0.0, 1.0, size=(cells, 2)) ** (1.0 / d)
    if d == 2:
        phi = rng.uniform(0.0, 2.0 * math.pi, size=(cells, 2))
        dirs = np.stack([np.cos(phi), np.sin(phi)], axis=-1)
    else:
        z = rng.standard_normal(size=(cells, 2, 3))
        dirs = z / np.linalg.norm(z, axis=-1, keepdims=True)
    return r[..., None] * dirs


def mixture_cells(d: int, N: int, L: float, cells: int, seed: int) -> np.ndarray:
    """Two-Maxwellian mixture per cell, float64, shape (cells, N, ..., N)."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, size=(cells, 2))
    T = rng.uniform(0.5, 1.5, size=(cells, 2))
    u = _ball(rng, cells, d)
    out = np.empty((cells,) + (N,) * d, dtype=np.float64)
    chunk = max(1, (1 << 22) // (N ** d))
    for c0 in range(0, cells, chunk):
        c1 = min(cells, c0 + chunk)
        out[c0:c1] = (maxwellian(d, N, L, rho[c0:c1, 0], u[c0:c1, 0], T[c0:c1, 0])
                      + maxwellian(d, N, L, rho[c0:c1, 1], u[c0:c1, 1], T[c0:c1, 1]))
    return out


def noisy_mixture_cells(d: int, N: int, L: float, cells: int, seed: int,
                        level: float = 0.01) -> np.ndarray:
    """Mixture plus additive noise eta ~ U[-level, level] * max_j f per cell,
    clipped at zero (the precision-stress workload)."""
    f = mixture_cells(d, N, L, cells, seed)
    rng = np.random.default_rng(seed + 7919)
    axes = tuple(range(1, d + 1))
    fmax = f.max(axis=axes, keepdims=True)
    f = f + rng.uniform(-level, level, size=f.shape) * fmax
    return np.maximum(f, 0.0)


def config_inputs(name: str, cells: int | None = None) -> np.ndarray:
    """float64 input batch of a named workload (optionally a prefix of cells)."""
    c = CONFIGS[name]
    n = c["cells"] if cells is None else cells
    if name == "bkw16":
        return bkw_initial(c["N"], c["L"])
    if c.get("noise"):
        return noisy_mixture_cells(c["d"], c["N"], c["L"], n, c["seed"], c["noise"])
    return mixture_cells(c["d"], c["N"], c["L"], n, c["seed"])
