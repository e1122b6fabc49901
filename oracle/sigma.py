"""O4: modelling check, the sigma/omega form of eq. (Boltzmann).

TEST INFRASTRUCTURE ONLY (see the package docstring).

    Q(f)(v) = int_{R^d} int_{S^(d-1)} B(|q|) [f(v') f(v'_*) - f(v) f(v_*)] domega dv_*,
    v' = (v + v_* + |q| omega)/2,  v'_* = (v + v_* - |q| omega)/2,  q = v - v_*,
with B = b (Maxwell pseudo-molecules, section 2) or B = b |q| (hard spheres).
This is the physical operator, with no Carleman change of variables, no
truncation radius, no periodisation and no Fourier series. It is evaluated for
an analytic f (a Maxwellian mixture) by the trapezoid rule in v_* on a large
box and in the angle(s) of omega. Agreement with Q_h as N, L and the number
of directions grow pins the Carleman constants B~ (2b for 2D Maxwell,
2b|z| for 2D hard spheres, 4b for 3D hard spheres) and the weights W_p. It
is a modelling check, never a parity reference.
"""

from __future__ import annotations

import math

import numpy as np


def mixture(params):
    """Analytic f = sum_i Maxwellian(rho_i, u_i, T_i) of eq. (M); params is a
    list of (rho, u (d,), T). Returns a callable on points (P, d)."""
    def fun(x):
        x = np.asarray(x, dtype=np.float64)
        d = x.shape[-1]
        out = np.zeros(x.shape[:-1])
        for rho, u, T in params:
            r2 = np.sum((x - np.asarray(u)) ** 2, axis=-1)
            out += rho / (2.0 * math.pi * T) ** (d / 2.0) * np.exp(-r2 / (2.0 * T))
        return out
    return fun


def _sphere_rule(d: int, n: int):
    if d == 2:
        a = 2.0 * math.pi * np.arange(n) / n
        return np.stack([np.cos(a), np.sin(a)], axis=1), np.full(n, 2.0 * math.pi / n)
    x, w = np.polynomial.legendre.leggauss(n)
    nphi = 2 * n
    ph = 2.0 * math.pi * np.arange(nphi) / nphi
    st = np.sqrt(1.0 - x ** 2)
    om = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)),
                   np.outer(x, np.ones(nphi))], axis=-1).reshape(-1, 3)
    wt = np.outer(w, np.full(nphi, 2.0 * math.pi / nphi)).reshape(-1)
    return om, wt


def q_sigma(fun, targets: np.ndarray, kernel: str, b: float, box: float,
            n_star: int, n_omega: int, gamma: float = 1.0) -> np.ndarray:
    """Q(f) at the target velocities (T, d) by nested quadrature; kernel
    "maxwell" (B = b), "hard_sphere" (B = b|q|) or "vhs" (B = b|q|^gamma)."""
    targets = np.asarray(targets, dtype=np.float64)
    d = targets.shape[1]
    h = 2.0 * box / n_star
    ax = -box + h * (np.arange(n_star) + 0.5)
    vs = np.stack([g.reshape(-1) for g in np.meshgrid(*([ax] * d), indexing="ij")], axis=1)
    wv = h ** d
    om, wo = _sphere_rule(d, n_omega)
    fs = fun(vs)
    out = np.empty(len(targets))
    for i, v in enumerate(targets):
        q = v[None, :] - vs
        qn = np.linalg.norm(q, axis=1)
        if kernel == "maxwell":
            B = b * np.ones_like(qn)
        elif kernel == "hard_sphere":
            B = b * qn
        else:
            B = b * np.where(qn > 0, qn, 1.0) ** gamma * (qn > 0)
        c = 0.5 * (v[None, :] + vs)
        gain = 0.0
        for o, w in zip(om, wo):
            vp = c + 0.5 * qn[:, None] * o
            vps = c - 0.5 * qn[:, None] * o
            gain += w * np.sum(B * fun(vp) * fun(vps))
        loss = fun(v[None, :])[0] * np.sum(wo) * np.sum(B * fs)
        out[i] = (gain - loss) * wv
    return out
