"""O1: the fast spectral collision operator Q_h, FP64, written from section 3.3.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes (section 3.3, eqs. (FU), (FC), (defQBCarleman),
(Btilde), (ode), (FKM) and the separable sum over A directions that closes the
section): f is periodised on a box, expanded in a truncated Fourier series, the
collision operator is written in Carleman form with the kernel B~(x, y) and
the product x.y in a delta function, the kernel modes B_F(l, m) are integrals
over x, y in the ball B_0(R), and B_F is replaced by a sum of A separable
products alpha_p(l) alpha'_p(m), giving A convolutions computed by FFT.

Readings taken where the paper is silent or ambiguous (each is listed with its
reasoning in the project's design notes):
  * grid: v_i = -L + i*2L/N per axis, period 2L;
  * modes k in {-N/2 .. N/2-1}^d, kappa_k = (pi/L) k; every filter is zero on
    a mode with some component -N/2 (no Nyquist content in the fields);
  * Carleman truncation radius R = 2*lambda*L, lambda = 2/(3+sqrt 2)
    (R = lambda*L with r_literal=True);
  * collocation: the fields are multiplied pointwise on the N^d grid;
  * 2D: x = rho e, y = rho' e_perp with e on the half circle, M equispaced
    angles theta_p = pi p / M; delta(x.y) dx dy = 1/2 de drho drho';
  * 3D: x = rho e, y in the plane e_perp, e on the half sphere with an
    (n_theta Gauss-Legendre in cos theta) x (n_phi equispaced azimuth) rule,
    delta(x.y) dx dy = 1/2 |rho| de drho dy;
  * Carleman kernel B~ = 2^(d-1) |z|^(2-d) B(|z|) with |z|^2 = |x|^2+|y|^2:
      2D Maxwell (B = b):      B~ = 2 b            (separable)
      2D hard spheres (B=b|q|): B~ = 2 b sqrt(rho^2+rho'^2) (not separable:
        expanded in K_r products of even radial functions, see
        hs2d_radial_expansion)
      2D variable hard spheres (B = b|q|^gamma): B~ = 2 b (rho^2+rho'^2)^(gamma/2),
        the same expansion
      3D hard spheres:          B~ = 4 b           (separable)
  * default b = 1/|S^(d-1)| (1/(2 pi) in 2D, fixed by the BKW closed form);
  * the loss term uses the same direction quadrature as the gain.

Pins (tests/test_oracle_*.py): P1 DFT vs numpy.fft on single modes; P2 filter
closed forms vs adaptive quadrature; P3 O1 == O3 (real-space brute force);
P4 O1 == O2 (direct mode sum); P5 mass; P6 Q(M,M) -> 0 with N; P7 BKW
(Q_h(f_BKW) vs the exact d f_BKW / dt); P8 shift/rotation/reflection
equivariance and Q(cf) = c^2 Q(f); P10 sigma-form quadrature; P11 projection.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import special

LAMBDA = 2.0 / (3.0 + math.sqrt(2.0))


def default_radius(L: float, r_literal: bool = False) -> float:
    """Carleman truncation radius: 2*lambda*L by default, lambda*L if literal."""
    return (LAMBDA if r_literal else 2.0 * LAMBDA) * L


def default_coupling(d: int) -> float:
    """b = 1/|S^(d-1)|: 1/(2 pi) for d=2, 1/(4 pi) for d=3."""
    return 1.0 / (2.0 * math.pi) if d == 2 else 1.0 / (4.0 * math.pi)


@dataclass(frozen=True)
class Setup:
    """Discrete operator parameters (velocity dimension, grid, kernel, quadrature)."""
    d: int
    N: int
    L: float
    kernel: str = "maxwell"          # "maxwell" | "hard_sphere" | "vhs" (B = b |q|^gamma, 2D)
    M: int = 8                       # number of collision directions (the paper's A)
    b: float | None = None           # kernel constant b_0 or b_1
    K_r: int | None = None           # HS-2D radial rank; None -> smallest with ratio < tol
    R: float | None = None           # Carleman radius override
    r_literal: bool = False
    n_rho: int = 32                  # HS-2D: Gauss-Legendre nodes on [0, R]
    kr_tol: float = 1e-4             # HS-2D: eigenvalue ratio cut for the auto K_r
    gamma: float = 1.0               # VHS exponent (kernel "vhs"), -1 <= gamma <= 1

    @property
    def radius(self) -> float:
        return self.R if self.R is not None else default_radius(self.L, self.r_literal)

    @property
    def coupling(self) -> float:
        return self.b if self.b is not None else default_coupling(self.d)


# ---------------------------------------------------------------- modes / DFT

def mode_indices(N: int) -> np.ndarray:
    """Integer modes in FFT order: 0, 1, .., N/2-1, -N/2, .., -1 (eq. (FU))."""
    return np.fft.fftfreq(N, d=1.0 / N).round().astype(np.int64)


def wave_vectors(d: int, N: int, L: float) -> list[np.ndarray]:
    """kappa_k = (pi/L) k on the full mode grid, one array per component."""
    kap = (math.pi / L) * mode_indices(N).astype(np.float64)
    return np.meshgrid(*([kap] * d), indexing="ij")


def active_mask(d: int, N: int) -> np.ndarray:
    """True on modes with no component equal to -N/2 (Nyquist removed)."""
    ok = mode_indices(N) != -(N // 2)
    grids = np.meshgrid(*([ok] * d), indexing="ij")
    m = grids[0]
    for g in grids[1:]:
        m = m & g
    return m


def forward_dft(f: np.ndarray, d: int) -> np.ndarray:
    """f_hat_k = N^-d sum_j f_j exp(-2 pi i k.j / N), last d axes (eq. (FC) on nodes)."""
    N = f.shape[-1]
    return np.fft.fftn(f, axes=tuple(range(-d, 0))) / float(N) ** d


def inverse_dft(z: np.ndarray, d: int) -> np.ndarray:
    """g_j = sum_k z_k exp(+2 pi i k.j / N) (eq. (FU) evaluated at the nodes)."""
    N = z.shape[-1]
    return np.fft.ifftn(z, axes=tuple(range(-d, 0))) * float(N) ** d


# ------------------------------------------------------------ filter families

def phi_segment(s, R: float) -> np.ndarray:
    """Phi(s) = int_{-R}^{R} exp(i rho s) d rho = 2 sin(R s)/s, Phi(0) = 2R."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty_like(s)
    small = np.abs(s) < 1e-300
    out[~small] = 2.0 * np.sin(R * s[~small]) / s[~small]
    out[small] = 2.0 * R
    return out


def phi_weighted_segment(s, R: float) -> np.ndarray:
    """Phi3(s) = int_{-R}^{R} |rho| exp(i rho s) d rho
             = 2 [R sin(R s)/s - 2 sin^2(R s / 2)/s^2],  Phi3(0) = R^2."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty_like(s)
    x = R * np.abs(s)
    tiny = x < 1e-4
    sb = s[~tiny]
    out[~tiny] = 2.0 * (R * np.sin(R * sb) / sb - 2.0 * np.sin(0.5 * R * sb) ** 2 / sb ** 2)
    xt = x[tiny]
    # series 2 R^2 sum_n (-1)^n x^(2n) / ((2n)! (2n+2)), three terms suffice here
    out[tiny] = 2.0 * R * R * (0.5 - xt ** 2 / 8.0 + xt ** 4 / 144.0)
    return out


def psi_disc(t, R: float) -> np.ndarray:
    """Psi3(t) = int_{|y|<=R, y in a plane} exp(i m.y) dy = 2 pi R J1(R t)/t,
    with t the length of the in-plane part of m; Psi3(0) = pi R^2."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    small = np.abs(t) < 1e-300
    out[~small] = 2.0 * math.pi * R * special.j1(R * t[~small]) / t[~small]
    out[small] = math.pi * R * R
    return out


def vhs_weight(r1, r2, gamma: float):
    """(rho^2 + rho'^2)^(gamma/2): the radial part of the 2D Carleman kernel of
    B = b |q|^gamma (|z|^2 = rho^2 + rho'^2); the square root for gamma = 1."""
    r2s = r1 ** 2 + r2 ** 2
    if gamma == 1.0:
        return np.sqrt(r2s)
    if gamma == 0.0:
        return np.ones_like(r2s)
    return r2s ** (0.5 * gamma)


def hs2d_radial_expansion(R: float, n_rho: int = 32, K_r: int | None = None,
                          tol: float = 1e-4, gamma: float = 1.0):
    """Separable expansion of the 2D hard-sphere Carleman weight.

    The gain needs int int_{[-R,R]^2} sqrt(rho^2 + rho'^2) F(rho) G(rho'). The
    weight is even in each argument, so only the even parts of F and G enter and
    the integral is 4 int int_{[0,R]^2}. With n_rho Gauss-Legendre nodes rho_a
    and weights w_a on [0, R] (the endpoint clustering at 0 resolves the cone
    point of the weight), the symmetric matrix
        A_ab = 4 sqrt(w_a w_b) sqrt(rho_a^2 + rho_b^2)
    is diagonalised, A = sum_j lam_j V_j V_j^T, and for F = exp(i rho s),
    G = exp(i rho' t) the double sum becomes sum_j lam_j Phi_j(s) Phi_j(t) with
        Phi_j(s) = sum_a sqrt(w_a) V_aj cos(rho_a s).
    Pairs are sorted by |lam| descending; K_r = None keeps the smallest count
    with |lam_{K_r}| / |lam_0| < tol. The sign of V_j is fixed by Phi_j(0) >= 0.

    The same expansion serves the variable-hard-sphere kernels B = b |q|^gamma
    with the weight (rho^2 + rho'^2)^(gamma/2) (gamma = 1: hard spheres).

    Returns (lam[K], rho[n_rho], w[n_rho], V[n_rho, K]).
    """
    x, w = np.polynomial.legendre.leggauss(n_rho)
    rp = 0.5 * R * (x + 1.0)
    wp = 0.5 * R * w
    A = 4.0 * np.sqrt(np.outer(wp, wp)) * vhs_weight(rp[:, None], rp[None, :], gamma)
    lam, V = np.linalg.eigh(A)
    idx = np.argsort(-np.abs(lam))
    lam, V = lam[idx], V[:, idx]
    if K_r is None:
        ratio = np.abs(lam) / abs(lam[0])
        below = np.nonzero(ratio < tol)[0]
        K_r = int(below[0]) if below.size else len(lam)
    lam, V = lam[:K_r], V[:, :K_r].copy()
    phi0 = np.sqrt(wp) @ V
    for j in range(K_r):
        ref = phi0[j]
        if abs(ref) < 1e-12 * np.max(np.abs(np.sqrt(wp) * V[:, j])):
            ref = V[np.argmax(np.abs(V[:, j])), j]
        if ref < 0:
            V[:, j] = -V[:, j]
    return lam, rp, wp, V


def hs2d_phi(s, rho_pos, w_pos, Vj) -> np.ndarray:
    """Phi_j(s) = sum_a sqrt(w_a) V_aj cos(rho_a s)."""
    s = np.asarray(s, dtype=np.float64)
    coef = np.sqrt(w_pos) * Vj
    out = np.zeros_like(s)
    for a in range(len(rho_pos)):
        out += coef[a] * np.cos(rho_pos[a] * s)
    return out


def hemisphere_rule(M: int):
    """3D directions: n_theta Gauss-Legendre nodes in cos(theta) on (0, 1) times
    n_phi = 2 n_theta equispaced azimuths, M = 2 n_theta^2. Weights sum to 2 pi."""
    nt = int(round(math.sqrt(M / 2.0)))
    if 2 * nt * nt != M:
        raise ValueError("3D direction count must be 2*n_theta^2")
    nphi = 2 * nt
    x, w = np.polynomial.legendre.leggauss(nt)
    ct = 0.5 * (x + 1.0)
    wt = 0.5 * w
    dirs, wts = [], []
    for i in range(nt):
        st = math.sqrt(max(0.0, 1.0 - ct[i] ** 2))
        for j in range(nphi):
            ph = 2.0 * math.pi * j / nphi
            dirs.append((st * math.cos(ph), st * math.sin(ph), ct[i]))
            wts.append(wt[i] * 2.0 * math.pi / nphi)
    return np.array(dirs), np.array(wts)


def directions(s: Setup):
    """Unit vectors e_p and quadrature weights of the direction rule.

    2D: theta_p = pi p / M, e_p = (cos, sin), weight pi/M each (half circle).
    3D: hemisphere_rule(M), weights summing to 2 pi.
    """
    if s.d == 2:
        if s.M < 2 or s.M % 2:
            raise ValueError("2D needs an even number of directions")
        th = math.pi * np.arange(s.M) / s.M
        return np.stack([np.cos(th), np.sin(th)], axis=1), np.full(s.M, math.pi / s.M)
    return hemisphere_rule(s.M)


def filter_bank(s: Setup):
    """List of (W, alpha, alpha') over all directions (and radial ranks).

    alpha, alpha' are real arrays on the full mode grid (FFT order), zero on
    Nyquist modes; the gain is sum W * IDFT[alpha f_hat] * IDFT[alpha' f_hat].
    """
    R = s.radius
    b = s.coupling
    kv = wave_vectors(s.d, s.N, s.L)
    act = active_mask(s.d, s.N)
    dirs, dw = directions(s)
    bank = []
    if s.d == 2:
        if s.kernel == "maxwell":
            fams = [(1.0, lambda x: phi_segment(x, R))]
        elif s.kernel in ("hard_sphere", "vhs"):
            g = 1.0 if s.kernel == "hard_sphere" else s.gamma
            lam, rp, wp, V = hs2d_radial_expansion(R, s.n_rho, s.K_r, s.kr_tol, gamma=g)
            fams = [(lam[j], (lambda x, j=j: hs2d_phi(x, rp, wp, V[:, j])))
                    for j in range(len(lam))]
        else:
            raise ValueError(s.kernel)
        for p in range(s.M):
            e = dirs[p]
            ep = np.array([-e[1], e[0]])
            sp = kv[0] * e[0] + kv[1] * e[1]
            sq = kv[0] * ep[0] + kv[1] * ep[1]
            for lam_j, phi in fams:
                # B~ = 2b (Maxwell) or 2b * radial expansion (hard spheres);
                # the 1/2 of the Carleman measure and the factor 2 of folding
                # the circle onto its half cancel, leaving W = 2b * (pi/M) * lam_j.
                W = 2.0 * b * dw[p] * lam_j
                bank.append((W, np.where(act, phi(sp), 0.0), np.where(act, phi(sq), 0.0)))
    else:
        if s.kernel != "hard_sphere":
            raise ValueError("3D supports hard spheres only")
        for p in range(len(dw)):
            e = dirs[p]
            par = kv[0] * e[0] + kv[1] * e[1] + kv[2] * e[2]
            perp = np.sqrt(np.maximum(kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2 - par ** 2, 0.0))
            # B~ = 4b; 1/2 of the measure times 2 for the half sphere -> W = 4b w_p
            W = 4.0 * b * dw[p]
            bank.append((W, np.where(act, phi_weighted_segment(par, R), 0.0),
                         np.where(act, psi_disc(perp, R), 0.0)))
    return bank


def loss_multiplier(bank) -> np.ndarray:
    """l(k) = sum_p W_p alpha_p(k) alpha'_p(k): the loss kernel mode B_F(m, m)
    under the same direction quadrature as the gain."""
    out = 0.0
    for W, a, ap in bank:
        out = out + W * a * ap
    return out


def q_fast(f: np.ndarray, s: Setup, bank=None, return_parts: bool = False):
    """Q_h(f) on the node grid (FP64). f: (..., N, .., N) with d trailing axes.

    gain = sum_p W_p g_p h_p, g_p = IDFT[alpha_p f_hat], h_p = IDFT[alpha'_p f_hat];
    loss = f * IDFT[l f_hat]; Q_h = gain - loss.
    """
    f = np.asarray(f, dtype=np.float64)
    if bank is None:
        bank = filter_bank(s)
    fh = forward_dft(f, s.d)
    gain = np.zeros_like(f)
    for W, a, ap in bank:
        g = inverse_dft(a * fh, s.d).real
        h = inverse_dft(ap * fh, s.d).real
        gain += W * g * h
    loss = f * inverse_dft(loss_multiplier(bank) * fh, s.d).real
    if return_parts:
        return gain - loss, gain, loss
    return gain - loss


# ------------------------------------------------- moments and projection

def moment_matrix(d: int, N: int, L: float) -> np.ndarray:
    """C[r, j] = phi_r(v_j), phi = (1, v_1..v_d, |v|^2) (eq. (i5)); shape (d+2, N^d)."""
    v = -L + np.arange(N, dtype=np.float64) * (2.0 * L / N)
    g = np.meshgrid(*([v] * d), indexing="ij")
    rows = [np.ones(N ** d)] + [gi.reshape(-1) for gi in g]
    rows.append(sum(gi.reshape(-1) ** 2 for gi in g))
    return np.array(rows)


def moments(q: np.ndarray, d: int, L: float) -> np.ndarray:
    """Discrete moments sum_j phi(v_j) q_j dv^d, shape (..., d+2)."""
    N = q.shape[-1]
    C = moment_matrix(d, N, L)
    dv = (2.0 * L / N) ** d
    return q.reshape(q.shape[:-d] + (-1,)) @ C.T * dv


def project_conservative(q: np.ndarray, d: int, L: float) -> np.ndarray:
    """Minimal-l2 correction making all d+2 discrete moments vanish:
    Q <- Q - C^T (C C^T)^-1 C Q (not part of the paper, which accepts the
    truncation loss of section 3.1)."""
    N = q.shape[-1]
    C = moment_matrix(d, N, L)
    flat = q.reshape(q.shape[:-d] + (-1,))
    lam = np.linalg.solve(C @ C.T, C @ flat.reshape(-1, N ** d).T).T
    out = flat - (lam @ C).reshape(flat.shape)
    return out.reshape(q.shape)
