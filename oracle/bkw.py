"""BKW closed-form solution of the space-homogeneous 2D Maxwell-molecule
Boltzmann equation (section 4.1, the first convergence test) and the error
norms of eq. (error).

TEST INFRASTRUCTURE ONLY (see the package docstring).

    f(v, t) = exp(-|v|^2 / (2S)) / (2 pi S^2) [2S - 1 + (1-S)/(2S) |v|^2],
    S(t) = 1 - exp(-t/8)/2.

Pins: unit mass, energy 2 and fourth moment 8 - 2 exp(-t/4) by quadrature
(closed forms of the expression above); the analytic time derivative is
checked against a centred difference of f.
"""

from __future__ import annotations

import math

import numpy as np


def bkw_S(t: float) -> float:
    return 1.0 - 0.5 * math.exp(-t / 8.0)


def bkw_f(v2, t: float):
    """f at squared speeds v2 = |v|^2."""
    S = bkw_S(t)
    v2 = np.asarray(v2, dtype=np.float64)
    return np.exp(-v2 / (2.0 * S)) / (2.0 * math.pi * S * S) * (
        2.0 * S - 1.0 + (1.0 - S) / (2.0 * S) * v2)


def bkw_dfdt(v2, t: float):
    """Exact d f / d t = (d f / d S)(d S / d t), dS/dt = exp(-t/8)/16."""
    S = bkw_S(t)
    v2 = np.asarray(v2, dtype=np.float64)
    A = np.exp(-v2 / (2.0 * S)) / (2.0 * math.pi * S * S)
    Bp = 2.0 * S - 1.0 + (1.0 - S) / (2.0 * S) * v2
    dA = A * (v2 / (2.0 * S * S) - 2.0 / S)
    dB = 2.0 - v2 / (2.0 * S * S)
    return (dA * Bp + A * dB) * math.exp(-t / 8.0) / 16.0


def bkw_grid(N: int, L: float, t: float) -> np.ndarray:
    v = -L + np.arange(N, dtype=np.float64) * (2.0 * L / N)
    g1, g2 = np.meshgrid(v, v, indexing="ij")
    return bkw_f(g1 ** 2 + g2 ** 2, t)


def error_norms(f_num: np.ndarray, f_ref: np.ndarray):
    """Relative L1 and L2 errors of eq. (error) and the absolute max error."""
    e = np.abs(np.asarray(f_num) - np.asarray(f_ref)).reshape(-1)
    r = np.abs(np.asarray(f_ref)).reshape(-1)
    return (e.sum() / r.sum(), math.sqrt((e ** 2).sum() / (r ** 2).sum()), e.max())
