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
