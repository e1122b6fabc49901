// Device helpers shared by the 2D collision kernels (included by each .hip file).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace qcoll {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));



typedef float f32x4 __attribute__((ext_vector_type(4)));

// Wavefront-wide max of non-negative values with DPP moves only (no LDS):
// rotations within each row of 16 lanes, then the row broadcasts of lanes 15
// and 31; lane 63 ends with the maximum, which is read back as a uniform value.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_max(float x) {
  int y = __builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), CTRL, ROWS, 0xf, false);
  return fmaxf(x, __int_as_float(y));
}

__device__ __forceinline__ float wave_max(float x) {
  x = dpp_max<0x121, 0xf>(x);  // row_ror:1
  x = dpp_max<0x122, 0xf>(x);  // row_ror:2
  x = dpp_max<0x124, 0xf>(x);  // row_ror:4
  x = dpp_max<0x128, 0xf>(x);  // row_ror:8
  x = dpp_max<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x = dpp_max<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Exponent e with x < 2^e for x > 0 (0 for x == 0 or non-finite input).
__device__ __forceinline__ int exp_above(float x) {
  if (!(x > 0.0f) || !(x <= 3.0e38f)) return 0;
  int e;
  frexpf(x, &e);
  return e;
}

// Exponent e with x < 2^e for a double x > 0 (0 for x == 0 or non-finite input).
__device__ __forceinline__ int exp_above_d(double x) {
  if (!(x > 0.0) || !(x <= 1.7e308)) return 0;
  int e;
  frexp(x, &e);
  return e;
}

// Wavefront-wide max of non-negative doubles (butterfly of lane exchanges).
__device__ __forceinline__ double wave_max_d(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
  return x;
}

// Register layouts of one cell's N x N field across a wavefront: register v
// of lane `lane` holds element (row(v, lane), col(lane)).
struct Lay32 {  // 32x32 MFMA result tile
  static constexpr int N = 32, V = 16;
  __device__ static int row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }
  __device__ static int col(int lane) { return lane & 31; }
};
struct Lay16 {  // 16x16 MFMA result tile
  static constexpr int N = 16, V = 4;
  __device__ static int row(int v, int lane) { return 4 * (lane >> 4) + v; }
  __device__ static int col(int lane) { return lane & 15; }
};

// ------------------------------------------------------------- epilogue

// Butcher tableaux of the multi-stage IMEX steps (section 3.4): explicit At
// and implicit A, rows = stages. [0] ARS(2,2,2) with gamma = 1 - 1/sqrt 2 and
// delta = 1 - 1/(2 gamma); [1] BPR(3,4,3). Both are stiffly accurate, so the
// step's result is the last stage.
constexpr double kRsqrt2 = 0.70710678118654752440084436210485;
constexpr double kGam = 1.0 - kRsqrt2;
constexpr double kDel = 1.0 - 1.0 / (2.0 * kGam);
__constant__ double kRkAt[2][5][5] = {
    {{0, 0, 0, 0, 0}, {kGam, 0, 0, 0, 0}, {kDel, 1.0 - kDel, 0, 0, 0}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}},
    {{0, 0, 0, 0, 0}, {1, 0, 0, 0, 0}, {4.0 / 9, 2.0 / 9, 0, 0, 0}, {0.25, 0, 0.75, 0, 0}, {0.25, 0, 0.75, 0, 0}}};
__constant__ double kRkA[2][5][5] = {
    {{0, 0, 0, 0, 0}, {0, kGam, 0, 0, 0}, {0, 1.0 - kGam, kGam, 0, 0}, {0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}},
    {{0, 0, 0, 0, 0}, {0.5, 0.5, 0, 0, 0}, {5.0 / 18, -1.0 / 9, 0.5, 0, 0}, {0.5, 0, 0, 0.5, 0},
     {0.25, 0, 0.75, -0.5, 0.5}}};
// A - At, entry by entry (the weight of nu (M - F_m) in the stage update).
__constant__ double kRkD[2][5][5] = {
    {{0, 0, 0, 0, 0}, {0 - kGam, kGam, 0, 0, 0}, {0 - kDel, (1.0 - kGam) - (1.0 - kDel), kGam, 0, 0}, {0, 0, 0, 0, 0},
     {0, 0, 0, 0, 0}},
    {{0, 0, 0, 0, 0}, {0.5 - 1, 0.5, 0, 0, 0}, {5.0 / 18 - 4.0 / 9, -1.0 / 9 - 2.0 / 9, 0.5, 0, 0},
     {0.5 - 0.25, 0, 0 - 0.75, 0.5, 0}, {0.25 - 0.25, 0, 0.75 - 0.75, -0.5, 0.5}}};

// exp(x) for x <= 0 in FP64 (the Maxwellian of the stage updates): x = k ln 2
// + r with k = rint(x / ln 2) and |r| <= ln(2) / 2 (ln 2 in two parts, so that r
// is exact to a few units of 2^-60), exp(r) from its Taylor series to degree 13
// (truncation error below 2^-60 on that interval) in Horner form, times 2^k.
// NaN stays NaN; results below the subnormal range are 0. The constants come
// from the table c (kExpConst): read in the epilogue of each cell, they do not
// occupy registers through the transform loops, as immediate constants
// hoisted out of the cell loop would.
#define QCOLL_EXP_CONSTANTS                                                                                    \
  {1.4426950408889634074, 6.93147180369123816490e-01, 1.90821492927058770002e-10, 1.0, 1.0, 0.5, 1.0 / 6.0, \
   1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0, 1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0,      \
   1.0 / 39916800.0, 1.0 / 479001600.0, 1.0 / 6227020800.0}
__constant__ double kExpConst[17] = QCOLL_EXP_CONSTANTS;

__host__ __device__ __forceinline__ double exp_nonpos(double x, const double* c) {
  if (!(x > -745.2)) return x != x ? x : 0.0;
  const double k = __builtin_rint(x * c[0]);
  double r = __builtin_fma(-k, c[1], x);   // ln 2, high part
  r = __builtin_fma(-k, c[2], r);          // ln 2, low part
  double p = c[16];                         // 1/13!
#pragma unroll
  for (int i = 15; i >= 3; --i) p = __builtin_fma(p, r, c[i]);
  return __builtin_ldexp(p, static_cast<int>(k));
}

// p[idx] where `in`, else 0, without a branch: lanes outside the grid read
// element 0 of the same cell (always present) and drop it. A conditional load
// becomes an exec-masked block of its own, and the compiler then waits for each
// load before the next block; unconditional loads of a row issue back to back.
__device__ __forceinline__ float load_or_zero(const float* p, bool in, int idx) {
  const float x = p[in ? idx : 0];
  return in ? x : 0.0f;
}

// The table of exp_nonpos behind an opaque pointer, taken once per cell.
__device__ __forceinline__ const double* exp_consts() {
  const double* c = kExpConst;
  asm volatile("" : "+s"(c));
  return c;
}

// Store Q, or apply the conservation projection (FP64 moments, wave
// reductions) and store Q as double, or apply the stage update to f.
// RG: rows per group of the stage update's loads (register budget of the caller).
template <int OUT, class LY, int RG = 4>
__device__ void finish_cell(const KernelArgs& a, int64_t cell, const float* fv, double* q, int lane) {
  if constexpr (OUT < 0) {  // epilogue chosen at run time (batched launches: eval, projection, step)
    if (a.out_kind == 0) finish_cell<0, LY>(a, cell, fv, q, lane);
    else if (a.out_kind == 1) finish_cell<1, LY>(a, cell, fv, q, lane);
    else finish_cell<2, LY>(a, cell, fv, q, lane);
    return;
  }
  // The velocities and addresses below are the same for every cell; an opaque
  // lane index, which depends on the cell's result, keeps the compiler from
  // hoisting them (and the epilogue's loads) out of the cell loop or ahead of
  // the transform loop, where they would occupy registers through it.
  asm volatile("" : "+v"(lane) : "v"(q[0]));
  constexpr int kV = LY::V;
  const int n = a.n;
  const int c = LY::col(lane);
  const int64_t base = cell * static_cast<int64_t>(n) * n;
  if (OUT == 0) {
    float* Qc = reinterpret_cast<float*>(a.q) + base;
#pragma unroll
    for (int v = 0; v < kV; ++v) {
      const int r = LY::row(v, lane);
      if (r < n && c < n) Qc[r * n + c] = static_cast<float>(q[v]);
    }
    return;
  }
  if (OUT == 4) {  // Q as double, no projection (the fine-grid stage of the Galerkin variant)
    double* Qc = reinterpret_cast<double*>(a.q) + base;
#pragma unroll
    for (int v = 0; v < kV; ++v) {
      const int r = LY::row(v, lane);
      if (r < n && c < n) Qc[r * n + c] = q[v];
    }
    return;
  }
  if (OUT == 1) {
    // moments sum_j phi(v_j) Q_j with phi = (1, v1, v2, |v|^2) (Q is zero
    // outside the n x n grid); lambda = G^-1 m; Q <- Q - lambda . phi
    const double v2c = -a.L + a.dv * c;
    double m0 = 0, m1 = 0, m2 = 0, m3 = 0;
#pragma unroll
    for (int v = 0; v < kV; ++v) {
      const double v1 = -a.L + a.dv * LY::row(v, lane);
      m0 += q[v];
      m1 += v1 * q[v];
      m2 += v2c * q[v];
      m3 += (v1 * v1 + v2c * v2c) * q[v];
    }
    m0 = wave_sum(m0);
    m1 = wave_sum(m1);
    m2 = wave_sum(m2);
    m3 = wave_sum(m3);
    double lam[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      lam[i] = a.gram_inv[i * 4 + 0] * m0 + a.gram_inv[i * 4 + 1] * m1 + a.gram_inv[i * 4 + 2] * m2 +
               a.gram_inv[i * 4 + 3] * m3;
    double* Qc = reinterpret_cast<double*>(a.q) + base;
#pragma unroll
    for (int v = 0; v < kV; ++v) {
      const int r = LY::row(v, lane);
      const double v1 = -a.L + a.dv * r;
      double corr = lam[0] + lam[1] * v1 + lam[2] * v2c + lam[3] * (v1 * v1 + v2c * v2c);
      if (r < n && c < n) Qc[r * n + c] = q[v] - corr;
    }
    return;
  }
  if (OUT == 3) {
    // Stage l of the penalised IMEX RK step (eqs. (GIMEXb), (GIMEX1b), space
    // homogeneous): with M the Maxwellian of the discrete moments of f^n and
    // nu = rho(f^n), S_m = nu (M - F_m), G_m = Q(F_m) - S_m,
    //   F_l = [f^n + k sum_{m<l} (At_lm G_m + A_lm S_m) + A_ll k nu M] / (1 + A_ll k nu).
    // q holds Q(F_{l-1}) of this launch (FP64), fv the input F_{l-1}.
    // opaque stage indices: the tableau coefficients are loaded here, per cell,
    // not hoisted into scalar registers held through the transform loops
    int sch = a.rk_scheme - 1, l = a.rk_stage;
    asm volatile("" : "+s"(sch), "+s"(l));
    const int S = sch == 0 ? 3 : 5;
    const double* At = kRkAt[sch][l - 1];
    const double* Ai = kRkA[sch][l - 1];
    const double* Dd = kRkD[sch][l - 1];
    float* fnp = a.rk_fn + base;
    // The moments of f^n are the same in every stage of the step: stage 2,
    // whose input F_1 is f^n (fv, zero outside the grid), sums them and keeps
    // them for the later stages, which read them back (32 bytes per cell in
    // place of a pass over f^n and four wavefront reductions). The address
    // depends on the opaque lane (lane / 64 is 0), so that the read stays here.
    const double v2c = -a.L + a.dv * c;
    double* mp = a.rk_mom + cell * 4 + (lane >> 6);
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    if (l == 2) {
#pragma unroll
      for (int v = 0; v < kV; ++v) {
        const double fnv = static_cast<double>(fv[v]);
        const double v1 = -a.L + a.dv * LY::row(v, lane);
        s0 += fnv;
        s1 += v1 * fnv;
        s2 += v2c * fnv;
        s3 += (v1 * v1 + v2c * v2c) * fnv;
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      s3 = wave_sum(s3);
      if (lane == 0) {
        mp[0] = s0;
        mp[1] = s1;
        mp[2] = s2;
        mp[3] = s3;
      }
    } else {
      s0 = mp[0];
      s1 = mp[1];
      s2 = mp[2];
      s3 = mp[3];
    }
    // the update loads of each group are unconditional (out-of-grid lanes read
    // element 0 and drop it), so that they issue together: f^n (a cache hit
    // after the first group; not held in registers) and the earlier stages'
    // values and Q
    const double rho = s0 * a.dv * a.dv, u1 = s1 / s0, u2 = s2 / s0;
    const double T = 0.5 * (s3 / s0 - u1 * u1 - u2 * u2);
    const double nu = rho, k = a.dt_eps;
    const double cM = rho / (2.0 * 3.14159265358979323846 * T);
    // F_l = rhs / den with rhs = f^n + k (nu (A_ll M + sum_m D_lm (M - F_m)) +
    // sum_m At_lm Q(F_m)), D = A - At: the scheme's sums regrouped so that the
    // weights are the tableau's own (scalar registers), and one reciprocal of
    // den per cell instead of a division per point.
    const double rden = 1.0 / (1.0 + Ai[l - 1] * k * nu);
    bool useq[4];   // Q(F_m) enters the update (At_lm != 0); per cell, not per point
#pragma unroll
    for (int m = 1; m <= 4; ++m) useq[m - 1] = At[m - 1] != 0.0;
    const double* ec = exp_consts();
    // the Maxwellian factors by velocity axis, M = cM e1(v1) e2(v2): this lane's
    // column factor, and the row factor of row (lane mod N), which the rows'
    // updates fetch from that lane (two exponentials per lane instead of one
    // per point)
    const double e2 = exp_nonpos(-(v2c - u2) * (v2c - u2) / (2.0 * T), ec);
    const double vr = -a.L + a.dv * (lane % LY::N);
    const double e1 = exp_nonpos(-(vr - u1) * (vr - u1) / (2.0 * T), ec);
    int bad = 0;
    // four rows at a time: the slot loads of the earlier stages for these rows
    // issue together (up to 2 stage values and 3 Q values per row), then the
    // update of each row in the order of the scheme's sums
    constexpr int kC = kV < RG ? kV : RG;
    double chain = q[0];   // the loads of a group wait for the previous group's update
#pragma unroll
    for (int v0 = 0; v0 < kV; v0 += kC) {
      float Fs[4][kC], Qs[4][kC];   // [m - 1][row]: F_m (m >= 2) and Q_m of stages m < l - 1
      float fn[kC];
      int cc = c;
      asm volatile("" : "+v"(cc) : "v"(chain));   // else all groups' loads are hoisted together
#pragma unroll
      for (int j = 0; j < kC; ++j) {
        const int r = LY::row(v0 + j, lane);
        fn[j] = load_or_zero(fnp, r < n && cc < n, r * n + cc);
      }
#pragma unroll
      for (int m = 1; m <= 4; ++m) {
        if (m >= l - 1) break;       // wave-uniform
        const float* Fp = a.rk_work + (m - 2) * a.rk_stride + base;
        const float* Qp = a.rk_work + (S - 3 + m) * a.rk_stride + base;
#pragma unroll
        for (int j = 0; j < kC; ++j) {
          const int r = LY::row(v0 + j, lane);
          const bool in = r < n && cc < n;
          if (m >= 2) Fs[m - 1][j] = load_or_zero(Fp, in, r * n + cc);
          Qs[m - 1][j] = load_or_zero(Qp, in, r * n + cc);
        }
      }
#pragma unroll
      for (int j = 0; j < kC; ++j) {
        const int v = v0 + j;
        const int r = LY::row(v, lane);
        const double fnv = static_cast<double>(fn[j]);
        const double M = cM * __shfl(e1, r) * e2;
        double t1 = Ai[l - 1] * M, t2 = 0.0;
#pragma unroll
        for (int m = 1; m <= 4; ++m) {
          if (m >= l) break;
          const double Fm = m == 1 ? fnv : (m == l - 1 ? static_cast<double>(fv[v]) : static_cast<double>(Fs[m - 1][j]));
          t1 += Dd[m - 1] * (M - Fm);
          if (useq[m - 1]) {
            const double Qm = m == l - 1 ? q[v] : static_cast<double>(Qs[m - 1][j]);
            t2 += At[m - 1] * Qm;
          }
        }
        const double rhs = fnv + k * (nu * t1 + t2);
        chain = rhs;
        if (!(r < n && c < n)) continue;
        const int o = r * n + c;
        const float Fl = static_cast<float>(rhs * rden);
        if (l == S) {
          bad |= !(fabsf(Fl) <= 3.0e38f);
          fnp[o] = Fl;
        } else {
          a.rk_work[(l - 2) * a.rk_stride + base + o] = Fl;
          a.rk_work[(S - 3 + (l - 1)) * a.rk_stride + base + o] = static_cast<float>(q[v]);
        }
      }
    }
    if (l == S && a.status) {
      bad = __any(bad) ? 1 : 0;
      if ((threadIdx.x & 63) == 0) a.status[cell] = bad;
    }
    return;
  }
  // OUT == 2: stage update in place
  double rho = 0.0;
#pragma unroll
  for (int v = 0; v < kV; ++v) rho += static_cast<double>(fv[v]);
  rho = wave_sum(rho) * a.dv * a.dv;
  const double k = a.scheme == 1 ? a.dt_eps / (1.0 + a.dt_eps * rho) : a.dt_eps;
  float* fcell = const_cast<float*>(a.f) + base;
  int bad = 0;
#pragma unroll
  for (int v = 0; v < kV; ++v) {
    const int r = LY::row(v, lane);
    float nv = static_cast<float>(static_cast<double>(fv[v]) + k * q[v]);
    if (r < n && c < n) {
      bad |= !(fabsf(nv) <= 3.0e38f);
      fcell[r * n + c] = nv;
    }
  }
  if (a.status) {
    bad = __any(bad) ? 1 : 0;
    if ((threadIdx.x & 63) == 0) a.status[cell] = bad;
  }
}

// Load one cell's n x n field into a register layout, zero outside the grid.
// `after`: a value computed just before the reload (a loads issued after the
// transform loops must not move ahead of them, where f would be held live).
template <class LY>
__device__ __forceinline__ void load_cell(const KernelArgs& a, int64_t cell, int lane, float* fv,
                                          float after = 0.0f) {
  asm volatile("" : "+v"(lane) : "v"(after));  // per-cell addresses, not hoisted (as in finish_cell)
  const int n = a.n, c = LY::col(lane);
  const float* fc = a.f + cell * static_cast<int64_t>(n) * n;
#pragma unroll
  for (int v = 0; v < LY::V; ++v) {
    const int r = LY::row(v, lane);
    fv[v] = load_or_zero(fc, r < n && c < n, r * n + c);
  }
}

// ------------------------------------------------------------ FX16 splits

struct Split3 {
  half8 l, h, o;  // fixed-point lead, FP16 hi and lo of the remainder
};

typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// Pairwise split into lead / hi / lo FP16 parts. The conversions go through
// v_cvt_pkrtz_f16_f32 (round toward zero): the lead is an exact small integer,
// and whatever hi loses to rounding is carried by lo, so the rounding mode of
// the conversion does not change the accuracy of the three-part sum.
struct P3 {
  half2v l, h, o;
};

typedef __fp16 fp16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ half2v pk(float a, float b) {
  fp16x2 r = __builtin_amdgcn_cvt_pkrtz(a, b);
  return __builtin_bit_cast(half2v, r);
}

// -1.0f that the compiler cannot fold: r + (-1) * hi with hi an FP16 value is
// then one v_fma_mix_f32 (FP16 operand converted inside the FMA) instead of a
// conversion plus a subtraction.
__device__ __forceinline__ float opaque_neg_one() {
  float m = -1.0f;
  asm("" : "+s"(m));
  return m;
}

__device__ __forceinline__ P3 finish_pair(float na, float nb, float ra, float rb) {
  const float m1 = opaque_neg_one();
  P3 s;
  s.l = pk(na, nb);
  s.h = pk(ra, rb);
  s.o = pk(fmaf(m1, static_cast<float>(s.h.x), ra), fmaf(m1, static_cast<float>(s.h.y), rb));
  return s;
}

// ya, yb already scaled so that |y| < 512.5 (FP64 inputs).
__device__ __forceinline__ P3 split2_f64(double ya, double yb) {
  double na = __builtin_rint(ya), nb = __builtin_rint(yb);
  return finish_pair(static_cast<float>(na), static_cast<float>(nb), static_cast<float>(ya - na),
                     static_cast<float>(yb - nb));
}

// From accumulator pairs (a0 exact, a1 small) scaled by the power of two c.
__device__ __forceinline__ P3 split2_acc(float a0, float a1, float b0, float b1, float c) {
  float ya = a0 * c, yb = b0 * c;
  float na = __builtin_rintf(ya), nb = __builtin_rintf(yb);
  return finish_pair(na, nb, fmaf(a1, c, ya - na), fmaf(b1, c, yb - nb));
}

__device__ __forceinline__ void put2(Split3& A, int t, const P3& s) {
  A.l[t] = s.l.x;
  A.l[t + 1] = s.l.y;
  A.h[t] = s.h.x;
  A.h[t + 1] = s.h.y;
  A.o[t] = s.o.x;
  A.o[t + 1] = s.o.y;
}

}  // namespace
}  // namespace qcoll
