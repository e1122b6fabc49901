"""Transport step on polygonal meshes: CWENO reconstruction and Rusanov fluxes
(section 2.2: eqs. (eqn.cellaverage), (CWENO:Popt), (CWENO:Popt1),
(CWENO:P0), (CWENO:Prec), (eqn.weights), (eqn.recpolydef),
(eq.Dubiner_phi_spatial), (finite_vol3), (finite_vol5)).

TEST INFRASTRUCTURE ONLY (see the package docstring). FP64, one cell at a time,
vectorised over the discrete velocities.

Notation: `deg` is the polynomial degree M of the reconstruction (the paper's M;
named deg here because M is the number of collision directions elsewhere),
K = (deg+1)(deg+2)/2 - 1 non-constant Taylor basis functions, n_e = 2 (K+1)
cells in the central stencil.

Readings (where the section leaves a choice open):
  * "closest neighbours" of the central stencil: the n_e - 1 cells (with their
    periodic image) whose generator points are nearest to the generator of P_i,
    among the cells within three face-neighbour rings; ties by cell index and
    image offset.
  * the one-sided P1 stencils: one per face L of P_i, {P_i, the neighbour
    across face L, the neighbour across face L+1} (cyclic, counter-clockwise).
  * linear weights: unnormalised 1e5 for the central polynomial and 1 for each
    one-sided one, normalised to sum 1.
  * oscillation indicator: sigma = sum over multi-indices 1 <= |b| <= deg of the
    cell mean of (d^b p / d xi^b)^2, xi = (x - x_b)/h_i (the scaled Taylor
    variables, so sigma is free of the cell size).
  * h_i ("radius of the circumcircle of P_i"): the largest distance from the
    barycentre to a vertex of P_i.
  * Rusanov: each discrete velocity is its own scalar linear law, so the
    dissipation speed on a face is |v_k . n|.
  * f at a face: the reconstruction of each side evaluated at G = deg + 1
    Gauss-Legendre points of the face; the cell integral of Q^w equals |P_i|
    times the cell value of Q (the Taylor basis has zero cell mean), so only
    the flux part is computed here.
Geometry integrals are exact: monomial moments of a polygon by the divergence
theorem, each edge integral by Gauss-Legendre of sufficient order.
"""

from __future__ import annotations

import dataclasses

import numpy as np

EPS_W = 1e-14    # epsilon of eq. (eqn.weights)
R_W = 4          # exponent r of eq. (eqn.weights)
LAMBDA_CENTRAL, LAMBDA_SIDED = 1e5, 1.0


def basis_exponents(deg: int) -> list[tuple[int, int]]:
    """(p, q) of the non-constant Taylor monomials, by total degree, p descending."""
    return [(t - q, q) for t in range(1, deg + 1) for q in range(t + 1)]


_GAUSS: dict[int, tuple[np.ndarray, np.ndarray]] = {}


def gauss01(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n-point Gauss-Legendre nodes and weights on [0, 1]."""
    if n not in _GAUSS:
        t, w = np.polynomial.legendre.leggauss(n)
        _GAUSS[n] = (0.5 * (t + 1.0), 0.5 * w)
    return _GAUSS[n]


def polygon_moment(P: np.ndarray, p: int, q: int) -> float:
    """Exact integral of x^p y^q over the polygon P (k x 2, counter-clockwise):
    by the divergence theorem it is the boundary integral of x^(p+1) y^q/(p+1) dy,
    and each edge integral (a polynomial of degree p+q+1 in the edge parameter)
    is taken by a Gauss-Legendre rule that is exact for it."""
    t, w = gauss01((p + q + 2) // 2 + 1)
    a, b = P, np.roll(P, -1, axis=0)
    x = a[:, None, 0] + t[None, :] * (b[:, None, 0] - a[:, None, 0])
    y = a[:, None, 1] + t[None, :] * (b[:, None, 1] - a[:, None, 1])
    dy = (b[:, 1] - a[:, 1])[:, None]
    return float(np.sum(w[None, :] * x ** (p + 1) * y ** q / (p + 1) * dy))


@dataclasses.dataclass
class CellGeom:
    area: float
    xb: np.ndarray          # barycentre (2,)
    h: float
    mean: np.ndarray        # cell mean of xi^p eta^q for the basis exponents (K,)
    moments: dict           # (p, q) -> cell mean of xi^p eta^q, total degree <= 2 deg


class Transport:
    """Per-mesh tables of the reconstruction (built lazily per cell)."""

    def __init__(self, mesh, deg: int):
        if deg not in (1, 2):
            raise ValueError("deg must be 1 or 2")
        self.mesh, self.deg = mesh, deg
        self.exps = basis_exponents(deg)
        self.K = len(self.exps)
        self.ne = 2 * (self.K + 1)
        lam = np.array([LAMBDA_CENTRAL] + [LAMBDA_SIDED] * 64)
        self._lam_raw = lam
        self._geom: dict[int, CellGeom] = {}
        self._cell: dict[int, dict] = {}

    # -- geometry ---------------------------------------------------------------
    def polygon(self, i: int, shift=(0.0, 0.0)) -> np.ndarray:
        s = self.mesh.faces(i)
        return self.mesh.verts[s.start:s.stop] + np.asarray(shift)

    def geom(self, i: int) -> CellGeom:
        g = self._geom.get(i)
        if g is not None:
            return g
        P = self.polygon(i)
        area = polygon_moment(P, 0, 0)
        xb = np.array([polygon_moment(P, 1, 0), polygon_moment(P, 0, 1)]) / area
        h = float(np.max(np.linalg.norm(P - xb, axis=1)))
        Pxi = (P - xb) / h
        a0 = polygon_moment(Pxi, 0, 0)
        moments = {(p, q): polygon_moment(Pxi, p, q) / a0
                   for t in range(2 * self.deg + 1) for q in range(t + 1) for p in [t - q]}
        mean = np.array([moments[e] for e in self.exps])
        g = CellGeom(area=area, xb=xb, h=h, mean=mean, moments=moments)
        self._geom[i] = g
        return g

    def basis_at(self, i: int, x: np.ndarray) -> np.ndarray:
        """phi^i_l(x) for points x (..., 2) in the frame of cell i: (..., K)."""
        g = self.geom(i)
        xi = (x - g.xb) / g.h
        return np.stack([xi[..., 0] ** p * xi[..., 1] ** q for p, q in self.exps], axis=-1) - g.mean

    def basis_avg_over(self, i: int, j: int, shift) -> np.ndarray:
        """Cell average over P_j (moved by shift into the frame of P_i) of phi^i: (K,)."""
        g = self.geom(i)
        Pxi = (self.polygon(j, shift) - g.xb) / g.h
        a0 = polygon_moment(Pxi, 0, 0)
        return np.array([polygon_moment(Pxi, p, q) / a0 for p, q in self.exps]) - g.mean

    # -- stencils ---------------------------------------------------------------
    def central_stencil(self, i: int) -> list[tuple[int, tuple[float, float]]]:
        """P_i's n_e - 1 nearest cells (by generator distance) within 3 rings."""
        m = self.mesh
        seen = {(i, 0.0, 0.0)}
        frontier = [(i, 0.0, 0.0)]
        for _ in range(3):
            nxt = []
            for (c, sx, sy) in frontier:
                for k in m.faces(c):
                    key = (int(m.nbr[k]), sx + m.shift[k, 0], sy + m.shift[k, 1])
                    if key not in seen:
                        seen.add(key)
                        nxt.append(key)
            frontier = nxt
        cand = []
        for (c, sx, sy) in seen:
            if (c, sx, sy) == (i, 0.0, 0.0):
                continue
            dx = m.gen[c, 0] + sx - m.gen[i, 0]
            dy = m.gen[c, 1] + sy - m.gen[i, 1]
            cand.append((dx * dx + dy * dy, c, sx, sy))
        cand.sort()
        if len(cand) < self.ne - 1:
            raise RuntimeError("mesh too small for the central stencil")
        return [(c, (sx, sy)) for _, c, sx, sy in cand[: self.ne - 1]]

    def cell_tables(self, i: int) -> dict:
        t = self._cell.get(i)
        if t is not None:
            return t
        m = self.mesh
        st = self.central_stencil(i)
        A = np.stack([self.basis_avg_over(i, j, s) for j, s in st])          # (n_e-1, K)
        faces = list(m.faces(i))
        nv = len(faces)
        lat = []
        for L in range(nv):
            k0, k1 = faces[L], faces[(L + 1) % nv]
            B = np.stack([self.basis_avg_over(i, int(m.nbr[k]), m.shift[k])[:2] for k in (k0, k1)])
            lat.append((int(m.nbr[k0]), int(m.nbr[k1]), B))
        lam = self._lam_raw[: nv + 1] / self._lam_raw[: nv + 1].sum()
        t = dict(stencil=st, A=A, lateral=lat, lam=lam)
        self._cell[i] = t
        return t

    # -- reconstruction ---------------------------------------------------------
    def sigma(self, i: int, c: np.ndarray) -> np.ndarray:
        """Oscillation indicator of sum_l c_l phi_l (c: (K, V)) on P_i."""
        mom = self.geom(i).moments
        out = np.zeros(c.shape[1:])
        for bt in range(1, self.deg + 1):
            for b2 in range(bt + 1):
                b1 = bt - b2
                # d^b of xi^p eta^q = p!/(p-b1)! q!/(q-b2)! xi^(p-b1) eta^(q-b2)
                terms = []
                for l, (p, q) in enumerate(self.exps):
                    if p >= b1 and q >= b2:
                        fac = float(np.prod(np.arange(p - b1 + 1, p + 1)) * np.prod(np.arange(q - b2 + 1, q + 1)))
                        terms.append((l, fac, p - b1, q - b2))
                for (l1, f1, p1, q1) in terms:
                    for (l2, f2, p2, q2) in terms:
                        out = out + f1 * f2 * mom[(p1 + p2, q1 + q2)] * c[l1] * c[l2]
        return out

    def reconstruct(self, i: int, fbar: np.ndarray, values=None, linear_weights: bool = False) -> np.ndarray:
        """Coefficients (K, V) of f^w on P_i (eq. (CWENO:Prec)); the constant part
        is fbar[i]. values(j, shift) -> (V,) cell average of the data over P_j
        moved by shift (default: fbar[j], the periodic data)."""
        t = self.cell_tables(i)
        get = (lambda j, s: fbar[j]) if values is None else values
        fi = get(i, (0.0, 0.0))
        d = np.stack([get(j, s) - fi for j, s in t["stencil"]])              # (n_e-1, V)
        c_opt = np.linalg.lstsq(t["A"], d, rcond=None)[0]                    # (K, V)
        m = self.mesh
        faces = list(m.faces(i))
        polys = []
        for L, (j0, j1, B) in enumerate(t["lateral"]):
            k0, k1 = faces[L], faces[(L + 1) % len(faces)]
            rhs = np.stack([get(j0, m.shift[k0]) - fi, get(j1, m.shift[k1]) - fi])
            cl = np.zeros_like(c_opt)
            cl[:2] = np.linalg.solve(B, rhs)
            polys.append(cl)
        lam = t["lam"]
        c0 = (c_opt - sum(lam[L + 1] * polys[L] for L in range(len(polys)))) / lam[0]
        polys = [c0] + polys
        if linear_weights:
            w = [np.full(fi.shape, l) for l in lam]
        else:
            wt = [lam[s] / (self.sigma(i, polys[s]) + EPS_W) ** R_W for s in range(len(polys))]
            tot = sum(wt)
            w = [x / tot for x in wt]
        return sum(w[s] * polys[s] for s in range(len(polys)))

    # -- fluxes -----------------------------------------------------------------
    def residual(self, fbar: np.ndarray, vel: np.ndarray, cells=None) -> np.ndarray:
        """R_i = -(1/|P_i|) sum over faces of the face integral of the Rusanov
        flux of the reconstructed states (eq. (finite_vol3)); fbar (n, V),
        vel (V, 2). Returns (len(cells), V)."""
        m = self.mesh
        cells = range(m.n) if cells is None else cells
        need = set()
        for i in cells:
            need.add(int(i))
            need.update(int(m.nbr[k]) for k in m.faces(int(i)))
        coef = {j: self.reconstruct(j, fbar) for j in sorted(need)}
        tg, wg = gauss01(self.deg + 1)
        out = []
        for i in cells:
            i = int(i)
            P = self.polygon(i)
            nv = len(P)
            acc = np.zeros(fbar.shape[1])
            for a, k in enumerate(m.faces(i)):
                p0, p1 = P[a], P[(a + 1) % nv]
                e = p1 - p0
                ln = float(np.hypot(e[0], e[1]))
                n = np.array([e[1], -e[0]]) / ln
                j, s = int(m.nbr[k]), m.shift[k]
                vn = vel @ n                                                  # (V,)
                for t, w in zip(tg, wg):
                    x = p0 + t * e
                    u_in = fbar[i] + self.basis_at(i, x) @ coef[i]
                    u_out = fbar[j] + self.basis_at(j, x - s) @ coef[j]
                    flux = 0.5 * vn * (u_in + u_out) - 0.5 * np.abs(vn) * (u_out - u_in)
                    acc = acc + w * ln * flux
            out.append(-acc / self.geom(i).area)
        return np.array(out)

    def step(self, fbar: np.ndarray, vel: np.ndarray, dt: float, cells=None) -> np.ndarray:
        """Explicit Euler transport step (eq. (finite_vol5) without the collision term)."""
        cells = range(self.mesh.n) if cells is None else cells
        return fbar[np.asarray(list(cells))] + dt * self.residual(fbar, vel, cells)


def velocity_pairs(N: int, L: float) -> np.ndarray:
    """(N*N, 2) velocities of the flattened grid f[i, a, b] -> (v_a, v_b), with the
    nodes of the collision grid, v_j = -L + j 2L/N, written as (2j - N) L/N (the
    same numbers, with the centre node exactly 0)."""
    v = (2.0 * np.arange(N) - N) * (L / N)
    a, b = np.meshgrid(v, v, indexing="ij")
    return np.stack([a.reshape(-1), b.reshape(-1)], axis=1)
