// FP64 construction of the discrete collision operator's tables (section 3.3).
//
// Carleman form (eqs. defQBCarleman, Btilde): Q = int int B~(x,y) delta(x.y)
// [f(v+y) f(v+x) - f(v+x+y) f(v)] dx dy. With x = rho e and y orthogonal to e
// the delta function reduces the double integral to
//   2D: (1/2) int_{S^1} de int int B~ ... drho drho'      (y = rho' e_perp)
//   3D: (1/2) int_{S^2} de int |rho| drho int_{e_perp} ... dy
// Truncating x, y to the ball of radius R (eq. FKM) and integrating a Fourier
// mode exp(i kappa.v) along the segment / over the disc gives the filters
//   Phi(s)  = int_{-R}^{R} exp(i rho s) drho       = 2 sin(Rs)/s
//   Phi3(s) = int_{-R}^{R} |rho| exp(i rho s) drho = 2R sin(Rs)/s - 4 sin^2(Rs/2)/s^2
//   Psi3(t) = int_{|y|<=R} exp(i m.y) dy (plane)  = 2 pi R J1(Rt)/t
// and the direction integral becomes the sum over A = M directions that closes
// section 3.3. The Carleman weight is B~ = 2^(d-1) |z|^(2-d) B(|z|) with
// |z|^2 = |x|^2 + |y|^2, so B~ = 2b (2D Maxwell), 4b (3D hard spheres) and
// 2b sqrt(rho^2 + rho'^2) (2D hard spheres), the last one expanded here in K_r
// separable products of even radial functions.

#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

#include "qcoll.h"

namespace qcoll {

namespace {

constexpr double kPi = 3.14159265358979323846;

double filt_segment(double s, double R) {
  if (s == 0.0) return 2.0 * R;
  return 2.0 * std::sin(R * s) / s;
}

double filt_weighted_segment(double s, double R) {
  double x = R * std::fabs(s);
  if (x < 1e-4) {
    // 2 int_0^R rho cos(rho s) drho, Taylor in x = R s
    return 2.0 * R * R * (0.5 - x * x / 8.0 + x * x * x * x / 144.0);
  }
  double h = std::sin(0.5 * R * s);
  return 2.0 * R * std::sin(R * s) / s - 4.0 * h * h / (s * s);
}

double filt_disc(double t, double R) {
  if (t == 0.0) return kPi * R * R;
  return 2.0 * kPi * R * std::cyl_bessel_j(1.0, R * t) / t;
}

// Mode value of FFT position i (0, 1, .., N/2-1, -N/2, .., -1).
inline int mode_of(int i, int N) { return i < N / 2 ? i : i - N; }

}  // namespace

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = pk;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void jacobi_eigen(int n, std::vector<double> a, std::vector<double>& evals,
                  std::vector<double>& evecs) {
  evecs.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) evecs[i * n + i] = 1.0;
  auto A = [&](int i, int j) -> double& { return a[static_cast<size_t>(i) * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A(i, j) * A(i, j);
        if (i != j) off += A(i, j) * A(i, j);
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (A(q, q) - A(p, p)) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * akq;
          A(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * aqk;
          A(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = evecs[k * n + p], vkq = evecs[k * n + q];
          evecs[k * n + p] = c * vkp - s * vkq;
          evecs[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  evals.resize(n);
  for (int i = 0; i < n; ++i) evals[i] = A(i, i);
}

int build_host_plan(HostPlan& hp, int d, int N, double L, int kernel, double b, int M, int K_r,
                    unsigned flags, double gamma, int n_rho) {
  if (d != 2 && d != 3) return QCOLL_EINVAL;
  if (N < 4 || (N & 1) || N > 256) return QCOLL_EINVAL;
  if (!(L > 0.0) || !std::isfinite(L)) return QCOLL_EINVAL;
  if (kernel != QCOLL_MAXWELL && kernel != QCOLL_HARD_SPHERE && kernel != QCOLL_VHS) return QCOLL_EINVAL;
  if (kernel == QCOLL_VHS && (d != 2 || !(gamma >= -1.0 && gamma <= 1.0))) return QCOLL_EINVAL;
  if (n_rho < 4 || n_rho > 512) return QCOLL_EINVAL;
  if (kernel == QCOLL_HARD_SPHERE) gamma = 1.0;
  if (M < 1) return QCOLL_EINVAL;
  if (d == 2 && (M & 1)) return QCOLL_EINVAL;
  if (K_r < 0) return QCOLL_EINVAL;
  if (d == 3 && kernel == QCOLL_MAXWELL) return QCOLL_EUNSUPPORTED;
  int ntheta = 0;
  if (d == 3) {
    ntheta = static_cast<int>(std::lround(std::sqrt(M / 2.0)));
    if (2 * ntheta * ntheta != M) return QCOLL_EINVAL;
  }

  const double lam = 2.0 / (3.0 + std::sqrt(2.0));
  hp.d = d;
  hp.N = N;
  hp.L = L;
  hp.M = M;
  hp.kernel = kernel;
  hp.gamma = gamma;
  hp.R = ((flags & QCOLL_R_LITERAL) ? lam : 2.0 * lam) * L;
  hp.b = b > 0.0 ? b : (d == 2 ? 1.0 / (2.0 * kPi) : 1.0 / (4.0 * kPi));
  const double R = hp.R;

  // ---- directions
  hp.dir.clear();
  hp.dir_w.clear();
  if (d == 2) {
    for (int p = 0; p < M; ++p) {
      double th = kPi * p / M;
      hp.dir.push_back(std::cos(th));
      hp.dir.push_back(std::sin(th));
      hp.dir_w.push_back(kPi / M);
    }
  } else {
    std::vector<double> x, w;
    gauss_legendre(ntheta, x, w);
    int nphi = 2 * ntheta;
    for (int i = 0; i < ntheta; ++i) {
      double ct = 0.5 * (x[i] + 1.0), st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
      for (int j = 0; j < nphi; ++j) {
        double ph = 2.0 * kPi * j / nphi;
        hp.dir.push_back(st * std::cos(ph));
        hp.dir.push_back(st * std::sin(ph));
        hp.dir.push_back(ct);
        hp.dir_w.push_back(0.5 * w[i] * 2.0 * kPi / nphi);
      }
    }
  }

  // ---- radial families (2D)
  std::vector<double> rnode, rw, V;  // HS-2D: nodes on [0, R], weights, eigenvectors
  const int nr = n_rho;
  if (d == 2 && kernel != QCOLL_MAXWELL) {
    std::vector<double> x, w;
    gauss_legendre(nr, x, w);
    rnode.resize(nr);
    rw.resize(nr);
    for (int a = 0; a < nr; ++a) {
      rnode[a] = 0.5 * R * (x[a] + 1.0);
      rw[a] = 0.5 * R * w[a];
    }
    // even-part kernel matrix on [0,R]^2 (the weight (rho^2 + rho'^2)^(gamma/2)
    // is even in each argument; gamma = 1 for hard spheres)
    std::vector<double> A(static_cast<size_t>(nr) * nr);
    for (int a = 0; a < nr; ++a)
      for (int c = 0; c < nr; ++c) {
        const double r2 = rnode[a] * rnode[a] + rnode[c] * rnode[c];
        const double wgt = gamma == 1.0 ? std::sqrt(r2) : (gamma == 0.0 ? 1.0 : std::pow(r2, 0.5 * gamma));
        A[a * nr + c] = 4.0 * std::sqrt(rw[a] * rw[c]) * wgt;
      }
    std::vector<double> ev, vec;
    jacobi_eigen(nr, A, ev, vec);
    std::vector<int> ord(nr);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int i, int j) { return std::fabs(ev[i]) > std::fabs(ev[j]); });
    int keep = K_r;
    if (keep == 0) {
      keep = nr;
      for (int i = 0; i < nr; ++i)
        if (std::fabs(ev[ord[i]]) < 1e-4 * std::fabs(ev[ord[0]])) { keep = i; break; }
    }
    if (keep > nr) return QCOLL_EINVAL;
    hp.K_r = keep;
    hp.lambda.resize(keep);
    V.assign(static_cast<size_t>(nr) * keep, 0.0);
    for (int j = 0; j < keep; ++j) {
      hp.lambda[j] = ev[ord[j]];
      double phi0 = 0.0, big = 0.0;
      for (int a = 0; a < nr; ++a) {
        double v = vec[a * nr + ord[j]];
        phi0 += std::sqrt(rw[a]) * v;
        if (std::fabs(v) > std::fabs(big)) big = v;
      }
      double ref = std::fabs(phi0) > 1e-12 ? phi0 : big;
      double sgn = ref < 0 ? -1.0 : 1.0;
      for (int a = 0; a < nr; ++a) V[a * keep + j] = sgn * vec[a * nr + ord[j]];
    }
  } else {
    hp.K_r = 1;
    hp.lambda.assign(1, 1.0);
  }
  const int Kr = hp.K_r;

  auto radial = [&](int j, double s) -> double {
    if (d == 2 && kernel == QCOLL_MAXWELL) return filt_segment(s, R);
    double acc = 0.0;  // HS-2D eigen-filter Phi_j(s) = sum_a sqrt(w_a) V_aj cos(rho_a s)
    for (int a = 0; a < nr; ++a) acc += std::sqrt(rw[a]) * V[a * Kr + j] * std::cos(rnode[a] * s);
    return acc;
  };

  // ---- per-term filters on the full mode grid
  int64_t n = 1;
  for (int i = 0; i < d; ++i) n *= N;
  const double dk = kPi / L;
  std::vector<int> pos(d);
  auto kappa_of = [&](int64_t idx, double* kv) {
    int64_t r = idx;
    for (int a = d - 1; a >= 0; --a) {
      int ia = static_cast<int>(r % N);
      r /= N;
      kv[a] = dk * mode_of(ia, N);
      pos[a] = ia;
    }
  };
  auto nyquist = [&](void) {
    for (int a = 0; a < d; ++a)
      if (pos[a] == N / 2) return true;
    return false;
  };

  hp.W.clear();
  hp.alpha.clear();
  hp.alphap.clear();
  const int T = M * Kr;
  hp.alpha.assign(T, std::vector<double>(n, 0.0));
  hp.alphap.assign(T, std::vector<double>(n, 0.0));
  hp.W.assign(T, 0.0);
  double kv[3];
  for (int p = 0; p < M; ++p) {
    const double* e = &hp.dir[p * d];
    for (int j = 0; j < Kr; ++j) {
      int t = p * Kr + j;
      if (d == 2) {
        double Bt = 2.0 * hp.b * (kernel == QCOLL_MAXWELL ? 1.0 : hp.lambda[j]);
        hp.W[t] = Bt * hp.dir_w[p];
      } else {
        hp.W[t] = 4.0 * hp.b * hp.dir_w[p];
      }
      for (int64_t k = 0; k < n; ++k) {
        kappa_of(k, kv);
        if (nyquist()) continue;
        if (d == 2) {
          double s1 = kv[0] * e[0] + kv[1] * e[1];
          double s2 = -kv[0] * e[1] + kv[1] * e[0];
          hp.alpha[t][k] = radial(j, s1);
          hp.alphap[t][k] = radial(j, s2);
        } else {
          double par = kv[0] * e[0] + kv[1] * e[1] + kv[2] * e[2];
          double k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
          double perp = std::sqrt(std::max(0.0, k2 - par * par));
          hp.alpha[t][k] = filt_weighted_segment(par, R);
          hp.alphap[t][k] = filt_disc(perp, R);
        }
      }
    }
  }
  hp.loss.assign(n, 0.0);
  for (int t = 0; t < T; ++t)
    for (int64_t k = 0; k < n; ++k) hp.loss[k] += hp.W[t] * hp.alpha[t][k] * hp.alphap[t][k];

  // ---- packed multipliers for the device
  const double inv_n = 1.0 / static_cast<double>(n);
  hp.packed.clear();
  if (d == 2) {
    for (int p = 0; p < M / 2; ++p)
      for (int j = 0; j < Kr; ++j) {
        int t = p * Kr + j, tq = (p + M / 2) * Kr + j;
        // gain terms t and tq are equal (alpha'_t = alpha_tq): 2 W g_t g_tq
        double w2 = 2.0 * hp.W[t];
        double sw = std::sqrt(std::fabs(w2)) * inv_n, sg = w2 < 0 ? -1.0 : 1.0;
        std::vector<std::complex<double>> m(n);
        for (int64_t k = 0; k < n; ++k) m[k] = {sg * sw * hp.alpha[t][k], sw * hp.alpha[tq][k]};
        hp.packed.push_back(std::move(m));
      }
  } else {
    for (int t = 0; t < T; ++t) {
      double sw = std::sqrt(std::fabs(hp.W[t])) * inv_n, sg = hp.W[t] < 0 ? -1.0 : 1.0;
      std::vector<std::complex<double>> m(n);
      for (int64_t k = 0; k < n; ++k) m[k] = {sg * sw * hp.alpha[t][k], sw * hp.alphap[t][k]};
      hp.packed.push_back(std::move(m));
    }
  }
  hp.loss_scaled.resize(n);
  for (int64_t k = 0; k < n; ++k) hp.loss_scaled[k] = hp.loss[k] * inv_n;

  // ---- inverse Gram matrix of phi = (1, v, |v|^2) over the nodes
  const int m = d + 2;
  std::vector<double> G(m * m, 0.0);
  const double dv = 2.0 * L / N;
  std::vector<double> phi(m);
  for (int64_t k = 0; k < n; ++k) {
    int64_t r = k;
    double v2 = 0.0;
    phi[0] = 1.0;
    for (int a = d - 1; a >= 0; --a) {
      double va = -L + dv * static_cast<double>(r % N);
      r /= N;
      phi[1 + a] = va;
      v2 += va * va;
    }
    phi[m - 1] = v2;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) G[i * m + j] += phi[i] * phi[j];
  }
  // Gauss-Jordan inverse with partial pivoting
  std::vector<double> Ai(m * m, 0.0);
  for (int i = 0; i < m; ++i) Ai[i * m + i] = 1.0;
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(G[r * m + c]) > std::fabs(G[piv * m + c])) piv = r;
    if (G[piv * m + c] == 0.0) return QCOLL_EINVAL;
    for (int j = 0; j < m; ++j) {
      std::swap(G[c * m + j], G[piv * m + j]);
      std::swap(Ai[c * m + j], Ai[piv * m + j]);
    }
    double inv = 1.0 / G[c * m + c];
    for (int j = 0; j < m; ++j) {
      G[c * m + j] *= inv;
      Ai[c * m + j] *= inv;
    }
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      double fct = G[r * m + c];
      for (int j = 0; j < m; ++j) {
        G[r * m + j] -= fct * G[c * m + j];
        Ai[r * m + j] -= fct * Ai[c * m + j];
      }
    }
  }
  hp.gram_inv = Ai;
  return QCOLL_OK;
}

void restrict_to_coarse_modes(HostPlan& hp, int Nc) {
  const int d = hp.d, Nf = hp.N;
  int64_t n = 1;
  for (int a = 0; a < d; ++a) n *= Nf;
  for (int64_t k = 0; k < n; ++k) {
    int64_t rem = k;
    bool keep = true;
    for (int a = d - 1; a >= 0; --a) {
      const int m = mode_of(static_cast<int>(rem % Nf), Nf);
      rem /= Nf;
      if (!(m > -Nc / 2 && m < Nc / 2)) keep = false;
    }
    if (keep) continue;
    for (auto& v : hp.alpha) v[k] = 0.0;
    for (auto& v : hp.alphap) v[k] = 0.0;
    for (auto& v : hp.packed) v[k] = 0.0;
    hp.loss[k] = 0.0;
    hp.loss_scaled[k] = 0.0;
  }
}

void galerkin_operators(int Nc, int Nf, std::vector<double>& interp, std::vector<double>& restrict_) {
  const double two_pi = 6.283185307179586476925286766559;
  interp.assign(static_cast<size_t>(Nf) * Nc, 0.0);
  restrict_.assign(static_cast<size_t>(Nc) * Nf, 0.0);
  for (int a = 0; a < Nf; ++a)
    for (int j = 0; j < Nc; ++j) {
      // sum over the active modes k = -Nc/2+1 .. Nc/2-1 of exp(2 pi i k (a/Nf - j/Nc)): real
      const double x = static_cast<double>(a) / Nf - static_cast<double>(j) / Nc;
      double s = 1.0;
      for (int k = 1; k < Nc / 2; ++k) s += 2.0 * std::cos(two_pi * k * x);
      interp[static_cast<size_t>(a) * Nc + j] = s / Nc;
      restrict_[static_cast<size_t>(j) * Nf + a] = s / Nf;
    }
}

}  // namespace qcoll
