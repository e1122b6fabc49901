"""O3: the discrete operator Q_h by real-space quadrature of the Carleman form.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (defQBCarleman) writes Q = int int B~(x, y) delta(x.y) [f(v+y) f(v+x) -
f(v+x+y) f(v)] dx dy. Here that integral is evaluated directly, with no
Fourier multiplier formula at all: f is replaced by its trigonometric
interpolant on the node grid with the Nyquist modes removed (the function
whose Fourier coefficients the fast method uses, eq. (FU)), evaluated
off-grid by an explicit mode sum; the segment, square, disc and
segment-times-disc integrals are done by Gauss-Legendre (and trapezoid in the
polar angle); the directions and their weights are those of the discrete
operator. In exact arithmetic this equals O1 with the same directions, so the
comparison pins the filter closed forms, their arguments (kappa.e, e_perp,
the in-plane part), the constants B~ and W, and the index conventions.

For 2D hard spheres the radial weight sqrt(rho^2+rho'^2) is applied on the
model's Gauss-Legendre node pairs (nodes on [0, R] mirrored to [-R, 0])
directly, which equals O1 with the radial expansion kept at full rank
K_r = n_rho.
"""

from __future__ import annotations

import math

import numpy as np

from .spectral import Setup, active_mask, directions, forward_dft, mode_indices, vhs_weight


def _interpolant(f: np.ndarray, s: Setup):
    """Return a callable x -> f~(x) for points x of shape (P, d)."""
    d, N, L = s.d, s.N, s.L
    fh = forward_dft(np.asarray(f, dtype=np.float64), d) * active_mask(d, N)
    kap = (math.pi / L) * mode_indices(N).astype(np.float64)
    v0 = -L

    def ev(x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        out = np.empty(x.shape[0])
        step = 1 << 15
        for i0 in range(0, x.shape[0], step):
            xs = x[i0:i0 + step]
            E = [np.exp(1j * np.outer(xs[:, a] - v0, kap)) for a in range(d)]
            if d == 2:
                t = E[1] @ fh.T                      # t[p, k1] = sum_k2 fh[k1,k2] E2[p,k2]
                val = np.sum(E[0] * t, axis=1)
            else:
                t = E[2] @ fh.reshape(N * N, N).T    # (P, N*N): sum over k3
                t = t.reshape(-1, N, N)
                t = np.einsum("pk,pjk->pj", E[1], t)
                val = np.sum(E[0] * t, axis=1)
            out[i0:i0 + step] = val.real
        return out

    return ev


def _nodes(d: int, N: int, L: float, idx=None):
    v = -L + np.arange(N, dtype=np.float64) * (2.0 * L / N)
    g = np.meshgrid(*([v] * d), indexing="ij")
    pts = np.stack([gi.reshape(-1) for gi in g], axis=1)
    return pts if idx is None else pts[idx]


def q_brute(f: np.ndarray, s: Setup, n_line: int | None = None, n_r: int | None = None,
            n_psi: int | None = None, node_idx=None) -> np.ndarray:
    """Q_h at the nodes (flat index list node_idx, default all) of ONE cell f."""
    d, N, L = s.d, s.N, s.L
    R = s.radius
    b = s.coupling
    f = np.asarray(f, dtype=np.float64)
    ftil = _interpolant(f, s)
    pts = _nodes(d, N, L, node_idx)
    fj = f.reshape(-1) if node_idx is None else f.reshape(-1)[node_idx]
    dirs, dw = directions(s)
    gain = np.zeros(len(pts))
    loss = np.zeros(len(pts))
    if d == 2:
        if s.kernel == "maxwell":
            nl = n_line or (2 * N + 24)
            x, w = np.polynomial.legendre.leggauss(nl)
            rho, wr = R * x, R * w
            Bt = lambda r1, r2: 2.0 * b * np.ones_like(r1)      # noqa: E731
        else:
            # the radial rule of the model: n_rho Gauss-Legendre nodes on [0, R]
            # mirrored to [-R, 0] (the weight is even in each argument)
            x, w = np.polynomial.legendre.leggauss(s.n_rho)
            rho = np.concatenate([-0.5 * R * (x + 1.0), 0.5 * R * (x + 1.0)])
            wr = np.concatenate([0.5 * R * w, 0.5 * R * w])
            g = 1.0 if s.kernel == "hard_sphere" else s.gamma
            Bt = lambda r1, r2: 2.0 * b * vhs_weight(r1, r2, g)  # noqa: E731
        R1, R2 = np.meshgrid(rho, rho, indexing="ij")
        W2 = np.outer(wr, wr) * Bt(R1, R2)                  # (q, q)
        for p in range(len(dw)):
            e = dirs[p]
            ep = np.array([-e[1], e[0]])
            # 1/2 (measure) * 2 (half circle -> circle) * (pi/M)
            cw = dw[p]
            ga = ftil((pts[:, None, :] + rho[None, :, None] * e).reshape(-1, 2)).reshape(len(pts), -1)
            ha = ftil((pts[:, None, :] + rho[None, :, None] * ep).reshape(-1, 2)).reshape(len(pts), -1)
            gain += cw * np.einsum("ja,ab,jb->j", ga, W2, ha)
            sq = (pts[:, None, None, :] + R1[None, :, :, None] * e + R2[None, :, :, None] * ep)
            fs = ftil(sq.reshape(-1, 2)).reshape(len(pts), len(rho), len(rho))
            loss += cw * np.einsum("jab,ab->j", fs, W2)
    else:
        # 3D hard spheres, B~ = 4b: segment weighted by |rho|, disc in e_perp
        nl = n_line or (N + 12)
        x, w = np.polynomial.legendre.leggauss(nl)
        rho = np.concatenate([-R * 0.5 * (x + 1.0), R * 0.5 * (x + 1.0)])
        wr = np.concatenate([R * 0.5 * w, R * 0.5 * w]) * np.abs(rho)
        nr = n_r or (N + 12)
        xr, wrr = np.polynomial.legendre.leggauss(nr)
        rr = R * 0.5 * (xr + 1.0)
        npsi = n_psi or (2 * N + 16)
        psi = 2.0 * math.pi * np.arange(npsi) / npsi
        Bt = 4.0 * b
        for p in range(len(dw)):
            e = dirs[p]
            a = np.array([1.0, 0.0, 0.0]) if abs(e[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
            u1 = a - (a @ e) * e
            u1 /= np.linalg.norm(u1)
            u2 = np.cross(e, u1)
            disc = (rr[:, None, None] * (np.cos(psi)[None, :, None] * u1 + np.sin(psi)[None, :, None] * u2)).reshape(-1, 3)
            dwt = (wrr[:, None] * R * 0.5 * rr[:, None] * np.full((1, npsi), 2.0 * math.pi / npsi)).reshape(-1)
            cw = dw[p]
            ga = ftil((pts[:, None, :] + rho[None, :, None] * e).reshape(-1, 3)).reshape(len(pts), -1)
            hd = ftil((pts[:, None, :] + disc[None, :, :]).reshape(-1, 3)).reshape(len(pts), -1)
            gain += cw * Bt * (ga @ wr) * (hd @ dwt)
            for i in range(len(pts)):
                sq = pts[i][None, None, :] + rho[:, None, None] * e + disc[None, :, :]
                fs = ftil(sq.reshape(-1, 3)).reshape(len(rho), len(disc))
                loss[i] += cw * Bt * (wr @ fs @ dwt)
    return gain - fj * loss
