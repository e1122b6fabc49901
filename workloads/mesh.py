"""Seeded synthetic polygonal meshes for the transport workload (section 2.2).

The space grid follows the construction of section 2.2: generator points, their
Delaunay triangulation, and for every generator the polygon through the centres
of mass of the Delaunay triangles around it. The domain is the periodic unit
square [0, 1)^2 (3 x 3 periodic images of the generators go into the
triangulation, so every polygon of the central copy is complete).

Generators: an nx x ny lattice with every point moved by U[-jitter, jitter]
lattice spacings per axis (seeded), numbered in Morton (Z) order of the lattice
indices so that cells close in space are close in memory.

Mesh arrays (float64 coordinates, int64 indices), polygon-major:
  gen[n, 2]          generator of every cell
  cell_ptr[n + 1]    face/vertex slots of cell i: cell_ptr[i] .. cell_ptr[i+1]-1
  verts[m, 2]        polygon vertices, counter-clockwise, in the cell's own frame
  nbr[m]             the cell across face k (from vertex k to vertex k+1)
  shift[m, 2]        integer offset (as float64) that maps the neighbour's own
                     frame into this cell's frame (x_in_this = x_in_nbr + shift)
  twin[m]            the slot of the same face in the neighbour's list

This module holds the mesh and the initial data only, none of the
reconstruction or flux arithmetic.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .synth import maxwellian


@dataclasses.dataclass
class Mesh:
    gen: np.ndarray
    cell_ptr: np.ndarray
    verts: np.ndarray
    nbr: np.ndarray
    shift: np.ndarray
    twin: np.ndarray

    @property
    def n(self) -> int:
        return len(self.gen)

    def faces(self, i: int) -> range:
        return range(int(self.cell_ptr[i]), int(self.cell_ptr[i + 1]))


def _morton(ix: np.ndarray, iy: np.ndarray) -> np.ndarray:
    code = np.zeros(ix.shape, dtype=np.int64)
    for b in range(16):
        code |= ((ix >> b) & 1) << (2 * b)
        code |= ((iy >> b) & 1) << (2 * b + 1)
    return code


def periodic_dual_mesh(nx: int, ny: int | None = None, seed: int = 0, jitter: float = 0.35) -> Mesh:
    from scipy.spatial import Delaunay

    ny = nx if ny is None else ny
    if nx < 3 or ny < 3:
        raise ValueError("need at least 3 x 3 generators")
    rng = np.random.default_rng(seed)
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ix, iy = ix.reshape(-1), iy.reshape(-1)
    order = np.argsort(_morton(ix, iy), kind="stable")
    ix, iy = ix[order], iy[order]
    n = nx * ny
    jit = rng.uniform(-jitter, jitter, size=(n, 2))
    gen = np.stack([(ix + 0.5 + jit[:, 0]) / nx, (iy + 0.5 + jit[:, 1]) / ny], axis=1)

    shifts = np.array([(sx, sy) for sx in (-1, 0, 1) for sy in (-1, 0, 1)], dtype=np.float64)
    centre = 4                                          # image (0, 0)
    pts = np.concatenate([gen + s for s in shifts])
    tri = Delaunay(pts)
    simp = tri.simplices
    cen = pts[simp].mean(axis=1)

    incident: list[list[int]] = [[] for _ in range(n)]
    for t, row in enumerate(simp):
        for v in row:
            if v // n == centre:
                incident[v - centre * n].append(t)

    cell_ptr = np.zeros(n + 1, dtype=np.int64)
    verts, nbr, shift = [], [], []
    for i in range(n):
        ts = np.array(incident[i])
        gi = centre * n + i
        ang = np.arctan2(cen[ts, 1] - gen[i, 1], cen[ts, 0] - gen[i, 0])
        ts = ts[np.argsort(ang)]
        k = len(ts)
        for a in range(k):
            t0, t1 = simp[ts[a]], simp[ts[(a + 1) % k]]
            common = (set(t0.tolist()) & set(t1.tolist())) - {gi}
            if len(common) != 1:
                raise RuntimeError("triangle fan around a generator is not closed")
            v = common.pop()
            verts.append(cen[ts[a]])
            nbr.append(v % n)
            shift.append(shifts[v // n])
        cell_ptr[i + 1] = cell_ptr[i] + k

    verts = np.array(verts)
    nbr = np.array(nbr, dtype=np.int64)
    shift = np.array(shift)
    owner = np.repeat(np.arange(n), np.diff(cell_ptr))
    key = {(int(owner[s]), int(nbr[s]), int(shift[s, 0]), int(shift[s, 1])): s for s in range(len(nbr))}
    if len(key) != len(nbr):
        raise RuntimeError("two faces between the same pair of cells and images")
    twin = np.array([key[(int(nbr[s]), int(owner[s]), -int(shift[s, 0]), -int(shift[s, 1]))]
                     for s in range(len(nbr))], dtype=np.int64)
    return Mesh(gen=gen, cell_ptr=cell_ptr, verts=verts, nbr=nbr, shift=shift, twin=twin)


# Transport workloads: mesh size and velocity grid. "explosion_16k" follows the
# explosion problem of the numerical section (about 16,500 polygons, 32^2
# velocities) on the periodic unit square with the velocity box of the double
# Mach reflection and airfoil runs, [-10, 10]^2.
TRANSPORT_CONFIGS = {
    "explosion_small": dict(nx=12, N=16, L=10.0, seed=2001),
    "explosion_16k": dict(nx=128, N=32, L=10.0, seed=2002),
}


def explosion_inputs(mesh: Mesh, N: int, L: float, seed: int) -> np.ndarray:
    """Cell values f[n, N, N] (float64): the local Maxwellian of a circular
    explosion, density 1 and temperature 1 inside radius 0.25 around the centre,
    density 0.125 and temperature 0.8 outside, with a smooth seeded bulk
    velocity; evaluated at the generators."""
    rng = np.random.default_rng(seed)
    x, y = mesh.gen[:, 0], mesh.gen[:, 1]
    inside = (x - 0.5) ** 2 + (y - 0.5) ** 2 < 0.25 ** 2
    rho = np.where(inside, 1.0, 0.125)
    T = np.where(inside, 1.0, 0.8)
    a = rng.uniform(0.1, 0.3, size=2)
    ph = rng.uniform(0.0, 2 * np.pi, size=2)
    u = np.stack([a[0] * np.sin(2 * np.pi * y + ph[0]), a[1] * np.cos(2 * np.pi * x + ph[1])], axis=1)
    return maxwellian(2, N, L, rho, u, T)


def transport_case(name: str):
    c = TRANSPORT_CONFIGS[name]
    mesh = periodic_dual_mesh(c["nx"], seed=c["seed"])
    return mesh, explosion_inputs(mesh, c["N"], c["L"], c["seed"] + 1), c["N"], c["L"]
