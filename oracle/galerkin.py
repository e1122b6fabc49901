"""Dealiased (Galerkin) variant of Q_h (section 3.3, eqs. (VAR), (ode)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The projection of eq. (VAR) keeps the modes of f_N and takes the convolution
sum of eq. (ode) over l + m = k WITHOUT wrap-around (the collocation operator
of `spectral.q_fast` sums modulo N). Reading used here: f is first restricted
to the active modes of the N-grid (no component equal to -N/2, the same set on
which the filters live), the sum runs over active l, m, and the result keeps the
active k only.

Two views:
  * q_galerkin: the 3/2 rule. The spectrum is zero-padded to Nf = 3N/2 modes
    per axis; products of inverse transforms on the Nf grid are exact linear
    convolutions for the kept modes (|l + m| <= N - 2 never wraps onto
    |k| < N/2 modulo 3N/2); the fine-grid result is transformed back and
    truncated to the active N-grid modes.
  * q_direct_linear: the literal double sum of eq. (ode) with the separable
    direction approximation of B_F, no FFT and no padding (tiny grids only).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .spectral import (Setup, active_mask, filter_bank, forward_dft, inverse_dft, mode_indices, q_fast)


def fine_size(N: int) -> int:
    if N % 2:
        raise ValueError("the Galerkin variant needs an even N")
    return 3 * N // 2


def _embed(coarse: np.ndarray, d: int, N: int, Nf: int) -> np.ndarray:
    """Place an N-grid spectrum (FFT order, last d axes) at the same integer
    modes of an Nf-grid spectrum (zeros elsewhere)."""
    pos = mode_indices(N) % Nf
    out = np.zeros(coarse.shape[:-d] + (Nf,) * d, dtype=np.complex128)
    out[(Ellipsis,) + tuple(np.ix_(*([pos] * d)))] = coarse
    return out


def _extract(fine: np.ndarray, d: int, N: int, Nf: int) -> np.ndarray:
    """The N-grid modes of an Nf-grid spectrum (inverse of _embed)."""
    pos = mode_indices(N) % Nf
    return fine[(Ellipsis,) + tuple(np.ix_(*([pos] * d)))]


def galerkin_bank(s: Setup):
    """Filter bank of the Nf grid restricted to the active N-grid modes: the
    filters depend only on the wave vector (same period 2L, same R), so this is
    the N-grid bank embedded in the finer mode grid."""
    Nf = fine_size(s.N)
    sf = dataclasses.replace(s, N=Nf)
    mask = _embed(active_mask(s.d, s.N).astype(np.complex128), s.d, s.N, Nf).real > 0.5
    return sf, [(W, np.where(mask, a, 0.0), np.where(mask, ap, 0.0)) for W, a, ap in filter_bank(sf)]


def q_galerkin(f: np.ndarray, s: Setup, fine=None) -> np.ndarray:
    """Dealiased Q on the N-grid nodes (FP64). f: (..., N, .., N)."""
    f = np.asarray(f, dtype=np.float64)
    d, N = s.d, s.N
    Nf = fine_size(N)
    sf, bank = fine if fine is not None else galerkin_bank(s)
    act = active_mask(d, N)
    fh = forward_dft(f, d) * act
    f_fine = inverse_dft(_embed(fh, d, N, Nf), d).real
    q_fine = q_fast(f_fine, sf, bank)
    qh = _extract(forward_dft(q_fine, d), d, N, Nf) * act
    return inverse_dft(qh, d).real


def q_direct_linear(f: np.ndarray, s: Setup, bank=None) -> np.ndarray:
    """Literal eq. (ode) for ONE cell: Q_hat_k = sum_{l+m=k} beta(l,m) f_l f_m
    over active l, m, k with l + m taken in the integers (no wrap-around)."""
    f = np.asarray(f, dtype=np.float64)
    d, N = s.d, s.N
    if bank is None:
        bank = filter_bank(s)
    n = N ** d
    act = active_mask(d, N).reshape(n)
    fh = forward_dft(f, d).reshape(n) * act
    A = np.stack([a.reshape(n) for _, a, _ in bank])
    Ap = np.stack([ap.reshape(n) for _, _, ap in bank])
    W = np.array([w for w, _, _ in bank])
    BF = (A.T * W) @ Ap
    beta = BF - np.diag(BF)[None, :]
    modes = np.stack(np.meshgrid(*([mode_indices(N)] * d), indexing="ij")).reshape(d, n)
    ksum = modes[:, :, None] + modes[:, None, :]                       # integer sums (d, n, n)
    keep = np.all((ksum > -(N // 2)) & (ksum < N // 2), axis=0)
    keep &= act[:, None] & act[None, :]
    kpos = np.ravel_multi_index(tuple(ksum[i] % N for i in range(d)), (N,) * d)
    terms = fh[:, None] * fh[None, :] * beta
    qh = np.zeros(n, dtype=np.complex128)
    np.add.at(qh, kpos[keep], terms[keep])
    return inverse_dft(qh.reshape((N,) * d), d).real
