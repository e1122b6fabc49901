// Host-side plan of the fast spectral collision operator (FP64 tables).
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace qcoll {

// FP64 description of the discrete operator Q_h (section 3.3):
//   gain(v) = sum_t W_t g_t(v) h_t(v), g_t = IDFT[alpha_t f_hat], h_t = IDFT[alpha'_t f_hat]
//   loss(v) = f(v) IDFT[l f_hat](v),   l = sum_t W_t alpha_t alpha'_t
// t runs over directions (and radial ranks of the 2D hard-sphere expansion).
struct HostPlan {
  int d = 2, N = 0, M = 0, K_r = 1, kernel = 0;
  double L = 0, R = 0, b = 0;
  double gamma = 1.0;             // variable-hard-sphere exponent (kernel QCOLL_VHS)
  std::vector<double> dir;        // M x d unit vectors
  std::vector<double> dir_w;      // quadrature weight of each direction
  std::vector<double> lambda;     // radial eigenvalues (K_r), {1} when separable
  std::vector<double> W;          // per term t = p*K_r + j
  std::vector<std::vector<double>> alpha, alphap;  // per term, N^d values, FFT order
  std::vector<double> loss;       // N^d
  std::vector<double> gram_inv;   // (d+2)^2

  // Packed complex multipliers for the device (one inverse transform each):
  // 2D: term (p, j), p < M/2, pairs alpha_{p,j} with alpha_{p+M/2,j} (= alpha'_{p,j});
  // 3D: term p pairs alpha_p with alpha'_p. Scaled by sqrt|W| (sign on the real
  // part) and by N^-d (the forward DFT is computed unnormalised).
  std::vector<std::vector<std::complex<double>>> packed;  // P_gain x N^d
  std::vector<double> loss_scaled;                         // l / N^d
};

// kernel QCOLL_MAXWELL, QCOLL_HARD_SPHERE or QCOLL_VHS (2D, B = b |q|^gamma,
// -1 <= gamma <= 1); n_rho Gauss-Legendre nodes of the 2D radial expansion.
int build_host_plan(HostPlan& hp, int d, int N, double L, int kernel, double b, int M, int K_r,
                    unsigned flags, double gamma = 1.0, int n_rho = 32);

// Dealiased (Galerkin) variant: restrict a plan built on the fine grid
// Nf = 3 Nc / 2 to the active modes of the Nc grid (integer components strictly
// between -Nc/2 and Nc/2): filters, loss multiplier and packed multipliers are
// zeroed elsewhere, so that products on the fine grid are the non-wrapping
// convolutions of eq. (ode) for the kept modes.
void restrict_to_coarse_modes(HostPlan& hp, int Nc);

// Real trigonometric interpolation (Nf x Nc, row-major) from the Nc grid to the
// Nf grid through the active Nc modes, and the matching restriction (Nc x Nf):
// transform, keep the active Nc modes, transform back.
void galerkin_operators(int Nc, int Nf, std::vector<double>& interp, std::vector<double>& restrict_);

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on the Legendre recurrence).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Cyclic Jacobi eigen-decomposition of a symmetric matrix (row-major, n x n).
// On return evals[i] and column i of evecs (row-major n x n) are the pairs.
void jacobi_eigen(int n, std::vector<double> a, std::vector<double>& evals,
                  std::vector<double>& evecs);

}  // namespace qcoll
