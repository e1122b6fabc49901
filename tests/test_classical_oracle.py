"""Pins of the classical spectral oracle (direct O(N^4) sum with exact kernel
modes, section 3.3) and of the variable-hard-sphere kernels, against facts
that do not come from the oracle itself: adaptive quadrature of the Maxwell
mode integral, an independent polar quadrature of the hard-sphere radial
integral, convergence under refinement, the fast operator (for the separable
modes), the BKW time derivative, mass conservation, and the physical
sigma-form of the collision integral for |q|^gamma kernels."""

import dataclasses
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as wl
from oracle import classical as cl
from oracle import spectral as sp
from oracle.bkw import bkw_dfdt, bkw_grid
from oracle.sigma import mixture, q_sigma


def _pair_vectors(N, L, l, m):
    kap = np.pi / L * sp.mode_indices(N)
    l1, l2 = divmod(int(l), N)
    m1, m2 = divmod(int(m), N)
    return np.array([kap[l1], kap[l2]]), np.array([kap[m1], kap[m2]])


def test_maxwell_exact_modes_match_adaptive_quadrature():
    """B(l, m) = 2b int_0^pi Phi(kl.e) Phi(km.e_perp) dtheta by scipy's quad."""
    N, L = 16, 8.0
    s = sp.Setup(d=2, N=N, L=L, kernel="maxwell", M=16)
    B = cl.kernel_modes(cl.exact_setup(s))
    R, b = s.radius, s.coupling
    idx = np.nonzero(sp.active_mask(2, N).reshape(-1))[0]
    rng = np.random.default_rng(0)
    for _ in range(5):
        l, m = rng.choice(idx, 2)
        kl, km = _pair_vectors(N, L, l, m)

        def fun(th):
            e = np.array([math.cos(th), math.sin(th)])
            ep = np.array([-e[1], e[0]])
            return (sp.phi_segment(np.array([kl @ e]), R)[0] * sp.phi_segment(np.array([km @ ep]), R)[0])
        v = integrate.quad(fun, 0.0, math.pi, limit=400, epsabs=0.0, epsrel=1e-12)[0]
        assert abs(B[l, m] - 2 * b * v) <= 1e-12 * np.abs(B).max()


def _hs_polar(sv, tv, R, nphi=48, nr=64):
    """4 int_0^R int_0^R sqrt(r1^2 + r2^2) cos(r1 s) cos(r2 t): polar coordinates
    about the cone point, the square cut along its diagonal, Gauss in r and phi."""
    x, w = np.polynomial.legendre.leggauss(nphi)
    xr, wr = np.polynomial.legendre.leggauss(nr)
    tot = 0.0
    for lo, hi, lim in ((0.0, math.pi / 4, np.cos), (math.pi / 4, math.pi / 2, np.sin)):
        ph = lo + (hi - lo) * 0.5 * (x + 1)
        wp = (hi - lo) * 0.5 * w
        rmax = R / lim(ph)
        r = rmax[:, None] * 0.5 * (xr[None, :] + 1)
        wrr = rmax[:, None] * 0.5 * wr[None, :]
        val = r * r * np.cos(r * np.cos(ph)[:, None] * sv) * np.cos(r * np.sin(ph)[:, None] * tv)
        tot += np.sum(wp[:, None] * wrr * val)
    return 4.0 * tot


def test_hard_sphere_exact_modes_match_polar_quadrature():
    N, L = 12, 6.0
    s = sp.Setup(d=2, N=N, L=L, kernel="hard_sphere", M=16)
    B = cl.kernel_modes(cl.exact_setup(s))
    R, b = s.radius, s.coupling
    idx = np.nonzero(sp.active_mask(2, N).reshape(-1))[0]
    rng = np.random.default_rng(1)
    nth = 8 * N
    th = math.pi * np.arange(nth) / nth
    for _ in range(2):
        l, m = rng.choice(idx, 2)
        kl, km = _pair_vectors(N, L, l, m)
        acc = sum(_hs_polar(kl @ [math.cos(t), math.sin(t)], km @ [-math.sin(t), math.cos(t)], R) for t in th)
        assert abs(B[l, m] - 2 * b * acc * math.pi / nth) <= 1e-9 * np.abs(B).max()


@pytest.mark.parametrize("kernel,tol", [("maxwell", 1e-13), ("hard_sphere", 1e-9)])
def test_exact_modes_are_converged(kernel, tol):
    s = sp.Setup(d=2, N=8, L=5.0, kernel=kernel, M=8)
    se = cl.exact_setup(s)
    B = cl.kernel_modes(se)
    B2 = cl.kernel_modes(dataclasses.replace(se, M=2 * se.M, n_rho=2 * se.n_rho, K_r=2 * se.n_rho))
    assert np.abs(B - B2).max() <= tol * np.abs(B).max()


@pytest.mark.parametrize("kernel", ["maxwell", "hard_sphere"])
def test_separable_modes_give_the_fast_operator(kernel):
    """The direct double sum with the fast method's own separable modes is the
    fast (FFT) operator: pins the mode arithmetic of the O(N^4) sum."""
    s = sp.Setup(d=2, N=12, L=5.0, kernel=kernel, M=8)
    f = wl.mixture_cells(2, 12, 5.0, 3, 17)
    q = cl.q_classical(f, s, cl.beta_table(s, separable=True))
    q0 = sp.q_fast(f, s)
    assert np.abs(q - q0).max() <= 1e-12 * np.abs(q0).max()


def test_classical_bkw_and_mass():
    """Q_classical(f_BKW) against the exact d f / dt (no direction quadrature
    error left: at least as close as the fast operator with 16 directions), and
    zero mass of Q."""
    N, L = 32, 8.0
    s = sp.Setup(d=2, N=N, L=L, kernel="maxwell", M=16)
    beta = cl.beta_table(s)
    v = -L + np.arange(N) * 2 * L / N
    g1, g2 = np.meshgrid(v, v, indexing="ij")
    for t in (0.0, 1.0):
        f = bkw_grid(N, L, t)
        ex = bkw_dfdt(g1 ** 2 + g2 ** 2, t)
        qc = cl.q_classical(f, s, beta)
        qf = sp.q_fast(f, s)
        ec, ef = np.abs(qc - ex).max(), np.abs(qf - ex).max()
        print(f"t={t}: classical {ec / np.abs(ex).max():.2e}, fast M=16 {ef / np.abs(ex).max():.2e}")
        assert ec <= 3e-4 * np.abs(ex).max() and ec <= 1.05 * ef
        assert abs(qc.sum()) <= 1e-13 * np.abs(qc).sum()


# ------------------------------------------------------- variable hard spheres

def test_vhs_endpoints_reduce_to_known_kernels():
    f = wl.mixture_cells(2, 16, 8.0, 2, 5)
    hs = sp.filter_bank(sp.Setup(d=2, N=16, L=8.0, kernel="hard_sphere", M=8))
    v1 = sp.filter_bank(sp.Setup(d=2, N=16, L=8.0, kernel="vhs", gamma=1.0, M=8))
    assert all(np.array_equal(a[1], b[1]) and a[0] == b[0] for a, b in zip(hs, v1))
    s0 = sp.Setup(d=2, N=16, L=8.0, kernel="vhs", gamma=0.0, M=8, K_r=1)
    qm = sp.q_fast(f, sp.Setup(d=2, N=16, L=8.0, kernel="maxwell", M=8))
    assert np.abs(sp.q_fast(f, s0) - qm).max() <= 1e-12 * np.abs(qm).max()


@pytest.mark.parametrize("gamma", [0.5, -0.5])
def test_vhs_matches_sigma_form(gamma):
    """Spectral VHS operator vs nested quadrature of the physical collision
    integral with B = b |q|^gamma at a few nodes."""
    params = [(1.2, np.array([0.3, -0.2]), 0.8), (0.7, np.array([-0.4, 0.1]), 1.3)]
    fun = mixture(params)
    L, N = 12.0, 64
    v = -L + np.arange(N) * 2 * L / N
    g = np.stack(np.meshgrid(v, v, indexing="ij"), -1).reshape(-1, 2)
    s = sp.Setup(d=2, N=N, L=L, kernel="vhs", gamma=gamma, M=32, K_r=16)
    q = sp.q_fast(fun(g).reshape(N, N), s).reshape(-1)
    idx = [32 * N + 32, 35 * N + 30, 27 * N + 36, 40 * N + 33]
    qs = q_sigma(fun, g[idx], "vhs", 1 / (2 * math.pi), 9.0, 96, 64, gamma=gamma)
    assert np.abs(q[idx] - qs).max() < 1e-6 * np.abs(q).max()
