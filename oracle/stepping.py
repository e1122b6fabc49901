"""Space-homogeneous time steps around Q_h (section 3.4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The homogeneous problem is d f/dt = Q(f)/eps. The paper's penalised IMEX
schemes (eqs. (Bref2), (GIMEXb), (GIMEX1b)) split Q = G_P + Q_BGK with
G_P = Q - Q_BGK explicit and Q_BGK = nu (M_f - f) implicit, nu = rho
(section 2). Both 1/eps factors are taken on the source terms, following
the continuous equation (Bref2).

In the homogeneous case the moments U are conserved, so the implicit
Maxwellian equals the explicit one and the first-order (IMEX Euler) stage
solves in closed form:
    f^{n+1} = f^n + (dt/eps) Q(f^n) / (1 + dt nu / eps),  nu = rho(f^n).
Pin (P12): this equals the literal penalised update with the Maxwellian terms
written out, and tends to explicit Euler as dt nu / eps -> 0.
"""

from __future__ import annotations

import numpy as np


def density(f: np.ndarray, d: int, L: float) -> np.ndarray:
    N = f.shape[-1]
    dv = (2.0 * L / N) ** d
    return f.reshape(f.shape[:-d] + (-1,)).sum(axis=-1) * dv


def explicit_euler(f, q, dt: float, eps: float = 1.0):
    return f + (dt / eps) * q


def imex_euler_penalized(f, q, dt: float, eps: float, d: int, L: float):
    nu = density(f, d, L).reshape(f.shape[:-d] + (1,) * d)
    return f + (dt / eps) * q / (1.0 + dt * nu / eps)


def imex_euler_penalized_literal(f, q, maxw, dt: float, eps: float, d: int, L: float):
    """Literal stage equation with an explicit Maxwellian array maxw:
    f1 = f + dt/eps [Q(f) - nu (M - f)] + dt/eps nu (M - f1), solved for f1."""
    nu = density(f, d, L).reshape(f.shape[:-d] + (1,) * d)
    rhs = f + (dt / eps) * (q - nu * (maxw - f)) + (dt / eps) * nu * maxw
    return rhs / (1.0 + dt * nu / eps)


# ------------------------------------------ multi-stage penalised IMEX RK

def _ars222():
    g = 1.0 - 1.0 / np.sqrt(2.0)
    dl = 1.0 - 1.0 / (2.0 * g)
    at = np.array([[0.0, 0.0, 0.0], [g, 0.0, 0.0], [dl, 1.0 - dl, 0.0]])
    a = np.array([[0.0, 0.0, 0.0], [0.0, g, 0.0], [0.0, 1.0 - g, g]])
    return at, a, at[-1].copy(), a[-1].copy()


def _bpr343():
    at = np.array([[0, 0, 0, 0, 0], [1, 0, 0, 0, 0], [4 / 9, 2 / 9, 0, 0, 0],
                   [1 / 4, 0, 3 / 4, 0, 0], [1 / 4, 0, 3 / 4, 0, 0]], dtype=np.float64)
    a = np.array([[0, 0, 0, 0, 0], [1 / 2, 1 / 2, 0, 0, 0], [5 / 18, -1 / 9, 1 / 2, 0, 0],
                  [1 / 2, 0, 0, 1 / 2, 0], [1 / 4, 0, 3 / 4, -1 / 2, 1 / 2]], dtype=np.float64)
    return at, a, at[-1].copy(), a[-1].copy()


# Butcher tableaux of section 3.4 (explicit A~, implicit A, weights w~, w):
# ARS(2,2,2) with gamma = 1 - 1/sqrt(2), delta = 1 - 1/(2 gamma), and BPR(3,4,3).
TABLEAUX = {"ars222": _ars222(), "bpr343": _bpr343()}


def discrete_moments(f: np.ndarray, d: int, L: float):
    """rho, u (d components) and T of f from grid sums (FP64): rho = sum f dv^d,
    rho u = sum v f dv^d, d rho T = sum |v - u|^2 f dv^d."""
    N = f.shape[-1]
    dv = (2.0 * L / N) ** d
    v = -L + np.arange(N) * (2.0 * L / N)
    grids = np.meshgrid(*([v] * d), indexing="ij")
    lead = f.shape[:-d]
    flat = f.reshape(lead + (-1,))
    rho = flat.sum(axis=-1) * dv
    u = np.stack([(flat * g.reshape(-1)).sum(axis=-1) * dv for g in grids], axis=-1) / rho[..., None]
    c2 = sum((g.reshape((1,) * len(lead) + (-1,)) - u[..., a, None]) ** 2 for a, g in enumerate(grids))
    T = (flat * c2).sum(axis=-1) * dv / (d * rho)
    return rho, u, T


def maxwellian_of(f: np.ndarray, d: int, L: float) -> np.ndarray:
    """Maxwellian of eq. (M) with the discrete moments of f, on the same grid."""
    rho, u, T = discrete_moments(f, d, L)
    N = f.shape[-1]
    v = -L + np.arange(N) * (2.0 * L / N)
    grids = np.meshgrid(*([v] * d), indexing="ij")
    lead = f.shape[:-d]
    shp = lead + (1,) * d
    r2 = sum((g[(None,) * len(lead)] - u[..., a].reshape(shp)) ** 2 for a, g in enumerate(grids))
    return rho.reshape(shp) / (2.0 * np.pi * T.reshape(shp)) ** (d / 2.0) * np.exp(-r2 / (2.0 * T.reshape(shp)))


def imex_rk_core(f, qfun, k: float, M, nu, scheme: str, return_stages: bool = False):
    """The stage recursion of the penalised IMEX RK scheme for given Maxwellian
    M and frequency nu (broadcastable to f), with k = dt/eps:
        F_l = [f + k (sum_{m<l} At_lm G_m + A_lm S_m) + A_ll k nu M] / (1 + A_ll k nu),
        G_m = Q(F_m) - S_m,  S_m = nu (M - F_m),
        f_new = f + k sum_m (wt_m G_m + w_m S_m)."""
    at, a, wt, w = TABLEAUX[scheme]
    F, G, S = [], [], []
    for l in range(len(wt)):
        rhs = f + a[l, l] * k * nu * M
        for m in range(l):
            rhs = rhs + k * (at[l, m] * G[m] + a[l, m] * S[m])
        Fl = rhs / (1.0 + a[l, l] * k * nu)
        Sl = nu * (M - Fl)
        need_q = (at[l + 1:, l] != 0.0).any() or wt[l] != 0.0
        Gl = (qfun(Fl) - Sl) if need_q else np.zeros_like(Fl)
        F.append(Fl)
        S.append(Sl)
        G.append(Gl)
    out = f + k * sum(wt[m] * G[m] + w[m] * S[m] for m in range(len(wt)))
    return (out, F) if return_stages else out


def imex_rk_penalized(f, qfun, dt: float, eps: float, d: int, L: float, scheme: str,
                      return_stages: bool = False):
    """One step of the penalised IMEX Runge-Kutta scheme (eqs. (GIMEXb),
    (GIMEX1b)) for the space-homogeneous problem d f/dt = Q(f)/eps.

    Q = G_P + Q_BGK with Q_BGK(F) = nu (M - F) taken implicitly (diagonal
    tableau entries) and G_P = Q - Q_BGK explicitly. Without transport the
    moment equation gives U^(l) = U^n, so every stage uses the Maxwellian M of
    the discrete moments of f^n and nu = rho(f^n) (see imex_rk_core).
    qfun maps a batch of fields to Q of the same shape.
    """
    f = np.asarray(f, dtype=np.float64)
    M = maxwellian_of(f, d, L)
    nu = density(f, d, L).reshape(f.shape[:-d] + (1,) * d)
    return imex_rk_core(f, qfun, dt / eps, M, nu, scheme, return_stages)
