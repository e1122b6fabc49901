// Transport plan on polygonal meshes (section 2.2): cell geometry, the CWENO
// stencils and least-squares operators (eqs. (CWENO:Popt), (CWENO:Popt1),
// (CWENO:P0)), the Taylor basis of eq. (eq.Dubiner_phi_spatial), the
// oscillation forms of eq. (eqn.weights) and the face data of the fluxes
// (eqs. (finite_vol3), (finite_vol5)); FP64 on the host, FP32 tables on the
// device. Polygon integrals follow the section: the polygon is cut into
// triangles (here from its generator point, with signed areas) and each
// triangle is integrated by a Gauss rule exact for the polynomial degrees used
// (collapsed 3 x 3 Gauss-Legendre, exact to degree 4).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "transport_args.hpp"
#include "qcoll.h"

// Stencil ranking compares squared generator distances: no contraction into
// fused multiply-adds, so that the ranking depends only on the rounded inputs.
#pragma clang fp contract(off)

struct qcoll_transport_s {
  int64_t ncells = 0, nslots = 0;
  int deg = 2, K = 5, ne = 12, N = 0;
  double L = 0;
  std::vector<int64_t> cell_ptr, nbr, twin;
  std::vector<double> verts, shift, gen;
  // host tables
  std::vector<double> area, xb, yb, h;
  std::vector<int64_t> st_cell;        // [cells][ne-1]
  std::vector<int> st_sx, st_sy;
  std::vector<double> pinv;            // [cells][K][ne-1]
  std::vector<double> S;               // [cells][15]
  std::vector<double> face_phi;        // [slots][K]
  std::vector<double> binv;            // [slots][4]
  std::vector<double> fnx, fny, fcoef; // [slots]
  bool on_device = false;
  int device = 0;
  qcoll::TrCell* d_cells = nullptr;
  qcoll::TrFlux* d_flux = nullptr;
};

namespace {

using Poly = std::vector<std::pair<double, double>>;

// Collapsed Gauss rule on the reference triangle (0,0), (1,0), (0,1): weights sum to 1/2.
struct TriRule {
  double x[9], y[9], w[9];
  TriRule() {
    const double t[3] = {0.5 - 0.5 * std::sqrt(0.6), 0.5, 0.5 + 0.5 * std::sqrt(0.6)};
    const double wt[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    int k = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b, ++k) {
        x[k] = t[a] * (1.0 - t[b]);
        y[k] = t[b];
        w[k] = wt[a] * wt[b] * (1.0 - t[b]);
      }
  }
};
const TriRule kTri;

// Integral of g over the polygon (vertices P, any orientation-consistent
// counter-clockwise order) by signed triangles from the apex c.
template <class G>
double poly_integral(const Poly& P, double cx, double cy, G g) {
  double tot = 0.0;
  const size_t n = P.size();
  for (size_t a = 0; a < n; ++a) {
    const double ax = P[a].first - cx, ay = P[a].second - cy;
    const double bx = P[(a + 1) % n].first - cx, by = P[(a + 1) % n].second - cy;
    const double J = ax * by - bx * ay;
    double s = 0.0;
    for (int q = 0; q < 9; ++q) s += kTri.w[q] * g(cx + kTri.x[q] * ax + kTri.y[q] * bx, cy + kTri.x[q] * ay + kTri.y[q] * by);
    tot += J * s;
  }
  return tot;
}

Poly polygon(const qcoll_transport_s& t, int64_t c, double sx, double sy) {
  Poly P;
  for (int64_t k = t.cell_ptr[c]; k < t.cell_ptr[c + 1]; ++k) P.emplace_back(t.verts[2 * k] + sx, t.verts[2 * k + 1] + sy);
  return P;
}

int64_t owner_of(const qcoll_transport_s& t, int64_t slot) {
  return std::upper_bound(t.cell_ptr.begin(), t.cell_ptr.end(), slot) - t.cell_ptr.begin() - 1;
}

double ipow(double x, int p) {
  double r = 1.0;
  for (int i = 0; i < p; ++i) r *= x;
  return r;
}

// Exponents of the non-constant Taylor monomials by total degree, p descending.
void exponents(int deg, std::vector<int>& ep, std::vector<int>& eq) {
  ep.clear();
  eq.clear();
  for (int tdeg = 1; tdeg <= deg; ++tdeg)
    for (int q = 0; q <= tdeg; ++q) {
      ep.push_back(tdeg - q);
      eq.push_back(q);
    }
}

// Solve the symmetric positive definite system (Cholesky); false if singular.
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> Lm(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= Lm[j * n + k] * Lm[j * n + k];
    if (!(d > 1e-14 * std::fabs(A[j * n + j])) || !(d > 0)) return false;
    Lm[j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= Lm[i * n + k] * Lm[j * n + k];
      Lm[i * n + j] = s / Lm[j * n + j];
    }
  }
  // inverse = L^-T L^-1, column by column
  std::vector<double> inv(n * n, 0.0), col(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= Lm[i * n + k] * col[k];
      col[i] = s / Lm[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = col[i];
      for (int k = i + 1; k < n; ++k) s -= Lm[k * n + i] * inv[k * n + c];
      inv[i * n + c] = s / Lm[i * n + i];
    }
  }
  A = inv;
  return true;
}

int build_tables(qcoll_transport_s& t) {
  const int64_t n = t.ncells;
  std::vector<int> ep, eq;
  exponents(t.deg, ep, eq);
  const int K = t.K, ns = t.ne - 1;
  t.area.assign(n, 0);
  t.xb.assign(n, 0);
  t.yb.assign(n, 0);
  t.h.assign(n, 0);
  std::vector<double> mom(n * 25, 0.0);  // cell means of xi^p eta^q, p, q <= 4
  for (int64_t i = 0; i < n; ++i) {
    const Poly P = polygon(t, i, 0, 0);
    const double gx = t.gen[2 * i], gy = t.gen[2 * i + 1];
    const double A = poly_integral(P, gx, gy, [](double, double) { return 1.0; });
    if (!(A > 0)) return QCOLL_EINVAL;
    const double bx = poly_integral(P, gx, gy, [](double x, double) { return x; }) / A;
    const double by = poly_integral(P, gx, gy, [](double, double y) { return y; }) / A;
    double hh = 0;
    for (auto& v : P) hh = std::max(hh, std::hypot(v.first - bx, v.second - by));
    t.area[i] = A;
    t.xb[i] = bx;
    t.yb[i] = by;
    t.h[i] = hh;
    for (int p = 0; p <= 2 * t.deg; ++p)
      for (int q = 0; p + q <= 2 * t.deg; ++q)
        mom[i * 25 + p * 5 + q] =
            poly_integral(P, gx, gy, [&](double x, double y) { return ipow((x - bx) / hh, p) * ipow((y - by) / hh, q); }) / A;
  }
  // cell average over P_j moved by (sx, sy) of the Taylor basis of cell i
  auto basis_avg = [&](int64_t i, int64_t j, double sx, double sy, double* out) {
    const Poly P = polygon(t, j, sx, sy);
    const double gx = t.gen[2 * j] + sx, gy = t.gen[2 * j + 1] + sy;
    const double A = poly_integral(P, gx, gy, [](double, double) { return 1.0; });
    for (int l = 0; l < K; ++l) {
      const int p = ep[l], q = eq[l];
      const double v = poly_integral(P, gx, gy, [&](double x, double y) {
        return ipow((x - t.xb[i]) / t.h[i], p) * ipow((y - t.yb[i]) / t.h[i], q);
      });
      out[l] = v / A - mom[i * 25 + p * 5 + q];
    }
  };
  t.st_cell.assign(n * ns, 0);
  t.st_sx.assign(n * ns, 0);
  t.st_sy.assign(n * ns, 0);
  t.pinv.assign(n * K * ns, 0.0);
  t.S.assign(n * 15, 0.0);
  t.face_phi.assign(t.nslots * K, 0.0);
  t.binv.assign(t.nslots * 4, 0.0);
  t.fnx.assign(t.nslots, 0);
  t.fny.assign(t.nslots, 0);
  t.fcoef.assign(t.nslots, 0);
  // Gauss-Legendre on [0, 1] with deg + 1 points (exact for the face averages)
  const double g2t[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)}, g2w[2] = {0.5, 0.5};
  const double g3t[3] = {0.5 - 0.5 * std::sqrt(0.6), 0.5, 0.5 + 0.5 * std::sqrt(0.6)},
               g3w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  const int ng = t.deg + 1;
  const double* gt = t.deg == 1 ? g2t : g3t;
  const double* gw = t.deg == 1 ? g2w : g3w;

  for (int64_t i = 0; i < n; ++i) {
    // central stencil: nearest generators among the cells within three face rings
    std::map<std::tuple<int64_t, int, int>, int> seen;
    std::vector<std::tuple<int64_t, int, int>> frontier{{i, 0, 0}};
    seen[{i, 0, 0}] = 0;
    for (int ring = 0; ring < 3; ++ring) {
      std::vector<std::tuple<int64_t, int, int>> next;
      for (auto& [c, sx, sy] : frontier)
        for (int64_t k = t.cell_ptr[c]; k < t.cell_ptr[c + 1]; ++k) {
          std::tuple<int64_t, int, int> key{t.nbr[k], sx + static_cast<int>(std::lround(t.shift[2 * k])),
                                            sy + static_cast<int>(std::lround(t.shift[2 * k + 1]))};
          if (seen.emplace(key, ring + 1).second) next.push_back(key);
        }
      frontier.swap(next);
    }
    std::vector<std::tuple<double, int64_t, int, int>> cand;
    for (auto& kv : seen) {
      const auto& [c, sx, sy] = kv.first;
      if (c == i && sx == 0 && sy == 0) continue;
      const double dx = (t.gen[2 * c] + sx) - t.gen[2 * i];
      const double dy = (t.gen[2 * c + 1] + sy) - t.gen[2 * i + 1];
      const double dxx = dx * dx, dyy = dy * dy;
      cand.emplace_back(dxx + dyy, c, sx, sy);
    }
    if (static_cast<int>(cand.size()) < ns) return QCOLL_EINVAL;
    std::sort(cand.begin(), cand.end());
    std::vector<double> A(ns * K);
    for (int s = 0; s < ns; ++s) {
      const auto& [d2, c, sx, sy] = cand[s];
      (void)d2;
      t.st_cell[i * ns + s] = c;
      t.st_sx[i * ns + s] = sx;
      t.st_sy[i * ns + s] = sy;
      basis_avg(i, c, sx, sy, &A[s * K]);
    }
    // least squares: (A^T A)^-1 A^T
    std::vector<double> N(K * K, 0.0);
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b)
        for (int s = 0; s < ns; ++s) N[a * K + b] += A[s * K + a] * A[s * K + b];
    if (!spd_inverse(N, K)) return QCOLL_EINVAL;
    for (int a = 0; a < K; ++a)
      for (int s = 0; s < ns; ++s) {
        double v = 0;
        for (int b = 0; b < K; ++b) v += N[a * K + b] * A[s * K + b];
        t.pinv[(i * K + a) * ns + s] = v;
      }
    // oscillation form: sigma(c) = sum_a S_aa c_a^2 + sum_{a<b} S_ab c_a c_b (stored row by row)
    double* S = &t.S[i * 15];
    if (t.deg == 1) {
      S[0] = 1.0;   // (0,0)
      S[5] = 1.0;   // (1,1) in the 5x5 layout
    } else {
      const double* m = &mom[i * 25];
      const double m10 = m[5], m01 = m[1], m20 = m[10], m11 = m[6], m02 = m[2];
      // row 0: (0,0) (0,1) (0,2) (0,3) (0,4); row 1: (1,1) .. (1,4); row 2: (2,2) ..; row 3; row 4
      S[0] = 1.0;
      S[2] = 4.0 * m10;
      S[3] = 2.0 * m01;
      S[5] = 1.0;
      S[7] = 2.0 * m10;
      S[8] = 4.0 * m01;
      S[9] = 4.0 * m20 + 4.0;
      S[10] = 4.0 * m11;
      S[12] = m20 + m02 + 1.0;
      S[13] = 4.0 * m11;
      S[14] = 4.0 * m02 + 4.0;
    }
    // faces
    const int64_t s0 = t.cell_ptr[i], nf = t.cell_ptr[i + 1] - s0;
    for (int64_t L = 0; L < nf; ++L) {
      const int64_t k = s0 + L, k1 = s0 + (L + 1) % nf;
      const double p0x = t.verts[2 * k], p0y = t.verts[2 * k + 1];
      const double ex = t.verts[2 * k1] - p0x, ey = t.verts[2 * k1 + 1] - p0y;
      const double len = std::hypot(ex, ey);
      t.fnx[k] = ey / len;
      t.fny[k] = -ex / len;
      t.fcoef[k] = len / t.area[i];
      for (int l = 0; l < K; ++l) {
        double v = 0;
        for (int g = 0; g < ng; ++g) {
          const double x = (p0x + gt[g] * ex - t.xb[i]) / t.h[i], y = (p0y + gt[g] * ey - t.yb[i]) / t.h[i];
          v += gw[g] * ipow(x, ep[l]) * ipow(y, eq[l]);
        }
        t.face_phi[k * K + l] = v - mom[i * 25 + ep[l] * 5 + eq[l]];
      }
      // one-sided P1 stencil {i, across face L, across face L+1}
      double b0[qcoll::kTrMaxK], b1[qcoll::kTrMaxK];
      basis_avg(i, t.nbr[k], t.shift[2 * k], t.shift[2 * k + 1], b0);
      basis_avg(i, t.nbr[k1], t.shift[2 * k1], t.shift[2 * k1 + 1], b1);
      const double det = b0[0] * b1[1] - b0[1] * b1[0];
      const double sc = std::fabs(b0[0] * b1[1]) + std::fabs(b0[1] * b1[0]);
      if (!(std::fabs(det) > 1e-10 * sc)) return QCOLL_EINVAL;
      t.binv[k * 4 + 0] = b1[1] / det;
      t.binv[k * 4 + 1] = -b0[1] / det;
      t.binv[k * 4 + 2] = -b1[0] / det;
      t.binv[k * 4 + 3] = b0[0] / det;
    }
  }
  // the two sides of a face share its length and have exactly opposite normals
  // (the flux kernels decide in/outflow by the sign of v.n on each side)
  for (int64_t k = 0; k < t.nslots; ++k) {
    const int64_t tw = t.twin[k];
    if (tw <= k) continue;
    const int64_t j = t.nbr[k];
    const double len = t.fcoef[k] * t.area[owner_of(t, k)];
    t.fnx[tw] = -t.fnx[k];
    t.fny[tw] = -t.fny[k];
    t.fcoef[tw] = len / t.area[j];
  }
  return QCOLL_OK;
}

int upload_tables(qcoll_transport_s& t) {
  const int64_t n = t.ncells;
  const int K = t.K, ns = t.ne - 1;
  std::vector<qcoll::TrCell> cells(n);
  std::vector<qcoll::TrFlux> flux(n);
  for (int64_t i = 0; i < n; ++i) {
    qcoll::TrCell& c = cells[i];
    qcoll::TrFlux& x = flux[i];
    c.slot0 = x.slot0 = static_cast<int>(t.cell_ptr[i]);
    c.nf = x.nf = static_cast<int>(t.cell_ptr[i + 1] - t.cell_ptr[i]);
    for (int s = 0; s < ns; ++s) c.stencil[s] = static_cast<int>(t.st_cell[i * ns + s]);
    for (int a = 0; a < K; ++a)
      for (int s = 0; s < ns; ++s) c.pinv[a][s] = static_cast<float>(t.pinv[(i * K + a) * ns + s]);
    for (int e = 0; e < 15; ++e) c.S[e] = static_cast<float>(t.S[i * 15 + e]);
    for (int L = 0; L < c.nf; ++L) {
      const int64_t k = c.slot0 + L;
      c.nbr[L] = static_cast<int>(t.nbr[k]);
      for (int e = 0; e < 4; ++e) c.binv[L][e] = static_cast<float>(t.binv[k * 4 + e]);
      for (int l = 0; l < K; ++l) c.phi[L][l] = static_cast<float>(t.face_phi[k * K + l]);
      x.twin[L] = static_cast<int>(t.twin[k]);
      x.nx[L] = static_cast<float>(t.fnx[k]);
      x.ny[L] = static_cast<float>(t.fny[k]);
      x.coef[L] = static_cast<float>(t.fcoef[k]);
    }
  }
  if (hipMalloc(&t.d_cells, sizeof(qcoll::TrCell) * n) != hipSuccess) return QCOLL_ENOMEM;
  if (hipMalloc(&t.d_flux, sizeof(qcoll::TrFlux) * n) != hipSuccess) return QCOLL_ENOMEM;
  if (hipMemcpy(t.d_cells, cells.data(), sizeof(qcoll::TrCell) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.d_flux, flux.data(), sizeof(qcoll::TrFlux) * n, hipMemcpyHostToDevice) != hipSuccess)
    return QCOLL_EDEVICE;
  return QCOLL_OK;
}

void release(qcoll_transport_s* t) {
  if (t->on_device) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(t->device);
    (void)hipFree(t->d_cells);
    (void)hipFree(t->d_flux);
    (void)hipSetDevice(cur);
  }
  delete t;
}

}  // namespace

extern "C" {

static int transport_plan_create(qcoll_transport_t* out, int64_t cells, const int64_t* cell_ptr,
                                 const double* verts, const int64_t* nbr, const double* shift, const int64_t* twin,
                                 const double* gen, int degree, int n_per_dim, double L, unsigned flags);

// No exception crosses the C ABI: a failed host allocation is QCOLL_ENOMEM.
int qcoll_transport_plan(qcoll_transport_t* out, int64_t cells, const int64_t* cell_ptr, const double* verts,
                         const int64_t* nbr, const double* shift, const int64_t* twin, const double* gen,
                         int degree, int n_per_dim, double L, unsigned flags) {
  try {
    return transport_plan_create(out, cells, cell_ptr, verts, nbr, shift, twin, gen, degree, n_per_dim, L, flags);
  } catch (const std::bad_alloc&) {
    if (out) *out = nullptr;
    return QCOLL_ENOMEM;
  }
}

static int transport_plan_create(qcoll_transport_t* out, int64_t cells, const int64_t* cell_ptr,
                                 const double* verts, const int64_t* nbr, const double* shift, const int64_t* twin,
                                 const double* gen, int degree, int n_per_dim, double L, unsigned flags) {
  if (!out) return QCOLL_EINVAL;
  *out = nullptr;
  if (cells < 1 || cells > (int64_t(1) << 30) || !cell_ptr || !verts || !nbr || !shift || !twin || !gen)
    return QCOLL_EINVAL;
  if ((degree != 1 && degree != 2) || n_per_dim < 2 || n_per_dim > 64 || !(L > 0) || !std::isfinite(L))
    return QCOLL_EINVAL;
  if (flags & ~QCOLL_HOST_ONLY) return QCOLL_EINVAL;
  if (cell_ptr[0] != 0) return QCOLL_EINVAL;
  for (int64_t i = 0; i < cells; ++i) {
    const int64_t nf = cell_ptr[i + 1] - cell_ptr[i];
    if (nf < 3 || nf > qcoll::kTrMaxFaces) return QCOLL_EINVAL;
  }
  const int64_t m = cell_ptr[cells];
  if (m > (int64_t(1) << 31) - 1) return QCOLL_EINVAL;
  for (int64_t i = 0; i < cells; ++i)
    for (int64_t k = cell_ptr[i]; k < cell_ptr[i + 1]; ++k) {
      if (nbr[k] < 0 || nbr[k] >= cells || twin[k] < 0 || twin[k] >= m) return QCOLL_EINVAL;
      const int64_t tw = twin[k];
      if (twin[tw] != k || nbr[tw] != i || shift[2 * tw] != -shift[2 * k] || shift[2 * tw + 1] != -shift[2 * k + 1])
        return QCOLL_EINVAL;
      if (!std::isfinite(verts[2 * k]) || !std::isfinite(verts[2 * k + 1]) ||
          std::fabs(shift[2 * k]) > 1e6 || std::fabs(shift[2 * k + 1]) > 1e6 ||
          shift[2 * k] != std::round(shift[2 * k]) || shift[2 * k + 1] != std::round(shift[2 * k + 1]))
        return QCOLL_EINVAL;
    }
  qcoll_transport_s* t = new (std::nothrow) qcoll_transport_s;
  if (!t) return QCOLL_ENOMEM;
  t->ncells = cells;
  t->nslots = m;
  t->deg = degree;
  t->K = degree == 2 ? 5 : 2;
  t->ne = 2 * (t->K + 1);
  t->N = n_per_dim;
  t->L = L;
  t->cell_ptr.assign(cell_ptr, cell_ptr + cells + 1);
  t->nbr.assign(nbr, nbr + m);
  t->twin.assign(twin, twin + m);
  t->verts.assign(verts, verts + 2 * m);
  t->shift.assign(shift, shift + 2 * m);
  t->gen.assign(gen, gen + 2 * cells);
  int rc = build_tables(*t);
  if (rc) {
    delete t;
    return rc;
  }
  if (!(flags & QCOLL_HOST_ONLY)) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1 || hipGetDevice(&t->device) != hipSuccess) {
      delete t;
      return QCOLL_EDEVICE;
    }
    t->on_device = true;
    rc = upload_tables(*t);
    if (rc) {
      release(t);
      return rc;
    }
  }
  *out = t;
  return QCOLL_OK;
}

int64_t qcoll_transport_work_bytes(qcoll_transport_t t) {
  if (!t) return -1;
  return t->nslots * static_cast<int64_t>(t->N) * t->N * static_cast<int64_t>(sizeof(float));
}

static int transport_call(qcoll_transport_t t, const float* f, float* out, int step, double dt, void* work,
                          int64_t work_bytes, hipStream_t stream) {
  if (!t) return QCOLL_EINVAL;
  if (!t->on_device) return QCOLL_EUNSUPPORTED;
  if (!f || !out || !work || work_bytes < qcoll_transport_work_bytes(t) || f == out || !std::isfinite(dt))
    return QCOLL_EINVAL;
  qcoll::TransportArgs a;
  a.cells = t->d_cells;
  a.flux = t->d_flux;
  a.f = f;
  a.fv = static_cast<float*>(work);
  a.out = out;
  a.ncells = t->ncells;
  a.N = t->N;
  a.V = t->N * t->N;
  a.vh = static_cast<float>(t->L / t->N);
  a.degree = t->deg;
  a.step = step;
  a.dt = static_cast<float>(dt);
  return qcoll::launch_transport(a, stream) ? QCOLL_EDEVICE : QCOLL_OK;
}

int qcoll_transport_rhs(qcoll_transport_t t, const float* f, float* R, void* work, int64_t work_bytes,
                        hipStream_t stream) {
  return transport_call(t, f, R, 0, 0.0, work, work_bytes, stream);
}

int qcoll_transport_step(qcoll_transport_t t, const float* f, float* out, double dt, void* work, int64_t work_bytes,
                         hipStream_t stream) {
  return transport_call(t, f, out, 1, dt, work, work_bytes, stream);
}

int qcoll_transport_table(qcoll_transport_t t, int which, int64_t i, double* out, int64_t n) {
  if (!t || !out || n < 0 || i < 0 || i >= t->ncells) return QCOLL_EINVAL;
  const int ns = t->ne - 1, K = t->K;
  std::vector<double> v;
  switch (which) {
    case 0:
      for (int s = 0; s < ns; ++s) v.push_back(static_cast<double>(t->st_cell[i * ns + s]));
      for (int s = 0; s < ns; ++s) v.push_back(t->st_sx[i * ns + s]);
      for (int s = 0; s < ns; ++s) v.push_back(t->st_sy[i * ns + s]);
      break;
    case 1: v = {t->area[i], t->xb[i], t->yb[i], t->h[i]}; break;
    case 2: v.assign(t->pinv.begin() + i * K * ns, t->pinv.begin() + (i + 1) * K * ns); break;
    case 3:
      v.assign(t->face_phi.begin() + t->cell_ptr[i] * K, t->face_phi.begin() + t->cell_ptr[i + 1] * K);
      break;
    case 4:
      for (int64_t k = t->cell_ptr[i]; k < t->cell_ptr[i + 1]; ++k) {
        v.push_back(t->fnx[k]);
        v.push_back(t->fny[k]);
        v.push_back(t->fcoef[k]);
        for (int e = 0; e < 4; ++e) v.push_back(t->binv[k * 4 + e]);
      }
      break;
    case 5: v.assign(t->S.begin() + i * 15, t->S.begin() + (i + 1) * 15); break;
    default: return QCOLL_EINVAL;
  }
  if (static_cast<int64_t>(v.size()) > n) return QCOLL_EINVAL;
  std::memcpy(out, v.data(), v.size() * sizeof(double));
  return static_cast<int>(v.size());
}

void qcoll_transport_destroy(qcoll_transport_t t) {
  if (t) release(t);
}

}  // extern "C"
