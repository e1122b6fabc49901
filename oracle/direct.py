"""O2: the discrete operator Q_h as the direct mode sum of eq. (ode).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.3 writes the fast spectral quadrature as
    Q_hat_k = sum_{l+m=k} beta_F(l, m) f_hat_l f_hat_m,
    beta_F(l, m) = B_F(l, m) - B_F(m, m),
with B_F(l, m) replaced by its separable direction sum
    B_F(l, m) ~ sum_p W_p alpha_p(l) alpha'_p(m).
Under the collocation reading the sum over l + m = k is taken modulo N (the
pointwise product on the N^d grid). This module evaluates that double sum
literally, in O(A n^2) operations, with no FFT convolution; it is compared
with O1 (which uses pointwise products of inverse FFTs) on tiny grids.
"""

from __future__ import annotations

import numpy as np

from .spectral import Setup, filter_bank, forward_dft, inverse_dft


def q_direct(f: np.ndarray, s: Setup, bank=None) -> np.ndarray:
    """Q_h(f) for ONE cell f of shape (N,)*d by the mode sum of eq. (ode)."""
    f = np.asarray(f, dtype=np.float64)
    d, N = s.d, s.N
    if bank is None:
        bank = filter_bank(s)
    n = N ** d
    fh = forward_dft(f, d).reshape(n)
    A = np.stack([a.reshape(n) for _, a, _ in bank])       # (P, n)
    Ap = np.stack([ap.reshape(n) for _, _, ap in bank])    # (P, n)
    W = np.array([w for w, _, _ in bank])
    BF = (A.T * W) @ Ap                                     # BF[l, m]
    beta = BF - np.diag(BF)[None, :]                        # BF(l,m) - BF(m,m)
    # array position of mode l + m (mod N), component-wise
    pos = np.indices((N,) * d).reshape(d, n)
    ksum = (pos[:, :, None] + pos[:, None, :]) % N          # (d, n, n)
    kflat = np.ravel_multi_index(tuple(ksum[i] for i in range(d)), (N,) * d)
    terms = fh[:, None] * fh[None, :] * beta
    qh = np.zeros(n, dtype=np.complex128)
    np.add.at(qh, kflat.reshape(-1), terms.reshape(-1))
    return inverse_dft(qh.reshape((N,) * d), d).real
