"""Classical spectral method: the direct double sum of eq. (CF1)/(ode) with
dense kernel modes (section 3.3, eqs. (VAR), (CF1), (KM), (ode), (FKM)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

  Q_hat_k = sum over l + m = k of beta(l, m) f_hat_l f_hat_m,
  beta(l, m) = B_F(l, m) - B_F(m, m),
in O(n^2) per cell (n = N^2 modes in 2D), the sum over l + m = k taken modulo N
as in the collocation of the fast method, so that the two differ only in the
kernel modes. The exact modes are the integrals of eq. (FKM) over the half
circle of directions and the two radial segments, evaluated here (reading) with
  * 8 N equispaced directions (the direction integrand is smooth and periodic,
    so the trapezoidal rule converges geometrically), and
  * for hard and variable hard spheres the radial weight expanded to full rank
    on 2 N + 16 Gauss-Legendre nodes of [0, R]; Maxwell molecules use the
    closed-form segment transform.
With `separable=True` the modes are the given Setup's own separable sum over
its M directions and K_r ranks (then Q equals the fast operator).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .spectral import Setup, filter_bank, forward_dft, inverse_dft


def exact_setup(s: Setup) -> Setup:
    """Setup whose separable sum is converged: the exact kernel modes."""
    if s.d != 2:
        raise ValueError("the classical method is implemented for d = 2")
    nr = 2 * s.N + 16
    return dataclasses.replace(s, M=8 * s.N, n_rho=nr, K_r=nr)


def kernel_modes(s: Setup) -> np.ndarray:
    """B[l, m] = sum_t W_t alpha_t(l) alpha'_t(m) over the flattened mode grid."""
    bank = filter_bank(s)
    n = s.N ** s.d
    A = np.stack([a.reshape(n) for _, a, _ in bank])
    Ap = np.stack([ap.reshape(n) for _, _, ap in bank])
    W = np.array([w for w, _, _ in bank])
    return (A.T * W) @ Ap


def beta_table(s: Setup, separable: bool = False) -> np.ndarray:
    """beta[l, m] = B(l, m) - B(m, m)."""
    B = kernel_modes(s if separable else exact_setup(s))
    return B - np.diag(B)[None, :]


def q_classical(f: np.ndarray, s: Setup, beta: np.ndarray | None = None) -> np.ndarray:
    """Q on the node grid for cells f (..., N, N) by the O(n^2) double sum."""
    f = np.asarray(f, dtype=np.float64)
    d, N = s.d, s.N
    n = N ** d
    if beta is None:
        beta = beta_table(s)
    lead = f.shape[:-d]
    fh = forward_dft(f, d).reshape(-1, n)
    # position of l = k - m (mod N) for every (k, m)
    k1, k2 = np.divmod(np.arange(n), N)
    l = ((k1[:, None] - k1[None, :]) % N) * N + (k2[:, None] - k2[None, :]) % N      # (k, m)
    bkm = beta[l, np.arange(n)[None, :]]                                              # beta(k - m, m)
    qh = np.einsum("km,ckm,cm->ck", bkm, fh[:, l], fh)
    return inverse_dft(qh.reshape(lead + (N,) * d), d).real
