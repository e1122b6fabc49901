// Per-cell bodies of the 2D kernels on 16x16 MFMA tiles (grids of up to 16
// points per axis, zero-padded), shared by the single-plan and the batched
// multi-plan kernels.
#pragma once

#include "kernels_common.hpp"

namespace qcoll {
namespace {

constexpr int kN16 = 16;

__device__ __forceinline__ f32x4 mfma1632(half8 a, half8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void mma6_16(const Split3& a, const Split3& b, f32x4& acc0, f32x4& acc1) {
  acc0 = mfma1632(a.l, b.l, acc0);
  acc1 = mfma1632(a.l, b.h, acc1);
  acc1 = mfma1632(a.h, b.l, acc1);
  acc1 = mfma1632(a.l, b.o, acc1);
  acc1 = mfma1632(a.h, b.h, acc1);
  acc1 = mfma1632(a.o, b.l, acc1);
}

enum { kFwdRe = 0, kFwdIm = 1, kInvRe = 2, kInvIm = 3 };

__device__ __forceinline__ float tile_absmax16(const f32x4& r0, const f32x4& r1, const f32x4& i0,
                                               const f32x4& i1) {
  // max (|acc0| + |acc1|): bounds |acc0| (the next lead) and |acc0 + acc1|
  float m = 0.0f;
#pragma unroll
  for (int v = 0; v < 4; ++v) m = fmaxf(m, fmaxf(fabsf(r0[v]) + fabsf(r1[v]), fabsf(i0[v]) + fabsf(i1[v])));
  return wave_max(m);
}

// Left operand [re rows | im rows] from a complex result tile.
__device__ __forceinline__ void slice16(const f32x4& r0, const f32x4& r1, const f32x4& i0, const f32x4& i1,
                                        float c, Split3& A) {
  put2(A, 0, split2_acc(r0[0], r1[0], r0[1], r1[1], c));
  put2(A, 2, split2_acc(r0[2], r1[2], r0[3], r1[3], c));
  put2(A, 4, split2_acc(i0[0], i1[0], i0[1], i1[1], c));
  put2(A, 6, split2_acc(i0[2], i1[2], i0[3], i1[3], c));
}

// Z = m * f_hat (FP64, |Z| < 2^9) split into the left operand.
__device__ __forceinline__ void spectrum16(const double* m, const double* fr, const double* fi, Split3& A) {
  double yr[4], yi[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    yr[v] = m[2 * v] * fr[v] - m[2 * v + 1] * fi[v];
    yi[v] = m[2 * v] * fi[v] + m[2 * v + 1] * fr[v];
  }
  put2(A, 0, split2_f64(yr[0], yr[1]));
  put2(A, 2, split2_f64(yr[2], yr[3]));
  put2(A, 4, split2_f64(yi[0], yi[1]));
  put2(A, 6, split2_f64(yi[2], yi[3]));
}

__device__ __forceinline__ void cpass16(const Split3& A, const Split3& Bre, const Split3& Bim, f32x4& r0,
                                        f32x4& r1, f32x4& i0, f32x4& i1) {
  r0 = r1 = i0 = i1 = f32x4{};
  mma6_16(A, Bre, r0, r1);
  mma6_16(A, Bim, i0, i1);
}

template <int OUT>  // OUT: 0 eval float, 1 eval double (projection), 2 step, -1 from a.out_kind
__device__ __forceinline__ void fx16_t16_body(const KernelArgs& a, int64_t first, int64_t stride) {
  const int lane = threadIdx.x & 63;
  Split3 E[4];
  {
    const half8* src = reinterpret_cast<const half8*>(a.econst) + lane * 12;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      E[m].l = src[m * 3 + 0];
      E[m].h = src[m * 3 + 1];
      E[m].o = src[m * 3 + 2];
    }
  }
  for (int64_t cell = first; cell < a.cells; cell += stride) {
    float fv[4];
    load_cell<Lay16>(a, cell, lane, fv);
    float fm = fmaxf(fmaxf(fabsf(fv[0]), fabsf(fv[1])), fmaxf(fabsf(fv[2]), fabsf(fv[3])));
    fm = wave_max(fm);
    const int a0 = 9 - exp_above(fm);
    const double cf = ldexp(1.0, a0);  // FP64: 2^a0 exceeds the FP32 range for max|f| < 2^-118
    Split3 A;
    put2(A, 0, split2_f64(static_cast<double>(fv[0]) * cf, static_cast<double>(fv[1]) * cf));
    put2(A, 2, split2_f64(static_cast<double>(fv[2]) * cf, static_cast<double>(fv[3]) * cf));
#pragma unroll
    for (int t = 4; t < 8; ++t) A.l[t] = A.h[t] = A.o[t] = static_cast<_Float16>(0.0f);
    f32x4 r0, r1, i0, i1;
    cpass16(A, E[kFwdRe], E[kFwdIm], r0, r1, i0, i1);
    int sc = -(a0 + 9);
    int a1 = 9 - exp_above(tile_absmax16(r0, r1, i0, i1));
    slice16(r0, r1, i0, i1, ldexpf(1.0f, a1), A);
    cpass16(A, E[kFwdRe], E[kFwdIm], r0, r1, i0, i1);
    sc = sc - a1 - 9;
    double fr[4], fi[4];
    float fhm = 0.0f;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      fr[v] = static_cast<double>(r0[v]) + static_cast<double>(r1[v]);
      fi[v] = static_cast<double>(i0[v]) + static_cast<double>(i1[v]);
      fhm = fmaxf(fhm, fmaxf(fabsf(static_cast<float>(fr[v])), fabsf(static_cast<float>(fi[v]))));
    }
    fhm = wave_max(fhm * 1.0000002f);
    const int bsh = 9 - (exp_above(fhm) + 1);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      fr[v] = ldexp(fr[v], bsh);
      fi[v] = ldexp(fi[v], bsh);
    }
    const int s_fh = sc - bsh;
    double gain[4] = {0.0, 0.0, 0.0, 0.0};
    int sd_last = 0;
    for (int q = 0; q <= a.P; ++q) {
      const double* mq = a.filt + (static_cast<int64_t>(q) * 64 + lane) * 8;
      double m[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) m[i] = mq[i];
      spectrum16(m, fr, fi, A);
      cpass16(A, E[kInvRe], E[kInvIm], r0, r1, i0, i1);
      int sd = a.filt_exp[q] + s_fh - 9;
      const int a2 = 9 - exp_above(tile_absmax16(r0, r1, i0, i1));
      slice16(r0, r1, i0, i1, ldexpf(1.0f, a2), A);
      cpass16(A, E[kInvRe], E[kInvIm], r0, r1, i0, i1);
      sd = sd - a2 - 9;
      sd_last = sd;
      const double w = q < a.P ? ldexp(1.0, 2 * sd) : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double re = static_cast<double>(r0[v]) + static_cast<double>(r1[v]);
        double im = static_cast<double>(i0[v]) + static_cast<double>(i1[v]);
        gain[v] = fma(re * w, im, gain[v]);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
      gain[v] -= static_cast<double>(fv[v]) *
                 ldexp(static_cast<double>(r0[v]) + static_cast<double>(r1[v]), sd_last);
    finish_cell<OUT, Lay16>(a, cell, fv, gain, lane);
  }
}

// ------------------------------------------------------------ FP32 (N = 16)

__device__ __forceinline__ f32x4 mfma164(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Complex pass with 16x16x4 FP32 MFMA: step (part, v) takes register v of the
// real (part 0) or imaginary (part 1) input tile; B[set][part*4 + v] is the
// matching DFT-matrix value Mat[4 g + v][n].
__device__ __forceinline__ void cpass16_f32(const float* xr, const float* xi, const float* Bre,
                                            const float* Bim, f32x4& re, f32x4& im) {
  re = im = f32x4{};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    re = mfma164(xr[v], Bre[v], re);
    re = mfma164(xi[v], Bre[4 + v], re);
    im = mfma164(xr[v], Bim[v], im);
    im = mfma164(xi[v], Bim[4 + v], im);
  }
}

template <int OUT>  // OUT: 0 eval float, 1 eval double (projection), 2 step, -1 from a.out_kind
__device__ __forceinline__ void fp32_t16_body(const KernelArgs& a, int64_t first, int64_t stride) {
  const int lane = threadIdx.x & 63;
  float B[4][8];
  {
    const float* src = reinterpret_cast<const float*>(a.econst) + lane * 32;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int t = 0; t < 8; ++t) B[m][t] = src[m * 8 + t];
  }
  const float zero[4] = {0.f, 0.f, 0.f, 0.f};
  for (int64_t cell = first; cell < a.cells; cell += stride) {
    float fv[4];
    load_cell<Lay16>(a, cell, lane, fv);
    f32x4 re, im;
    cpass16_f32(fv, zero, B[kFwdRe], B[kFwdIm], re, im);
    float ur[4], ui[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      ur[v] = re[v];
      ui[v] = im[v];
    }
    cpass16_f32(ur, ui, B[kFwdRe], B[kFwdIm], re, im);
    float fr[4], fi[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      fr[v] = re[v];
      fi[v] = im[v];
    }
    double gain[4] = {0.0, 0.0, 0.0, 0.0};
    float lf[4];
    for (int q = 0; q <= a.P; ++q) {
      const float* mq = q < a.P ? a.filt32 + (static_cast<int64_t>(q) * 64 + lane) * 8 : nullptr;
      float zr[4], zi[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (q < a.P) {
          zr[v] = mq[2 * v] * fr[v] - mq[2 * v + 1] * fi[v];
          zi[v] = mq[2 * v] * fi[v] + mq[2 * v + 1] * fr[v];
        } else {
          float l = a.loss32[lane * 4 + v];
          zr[v] = l * fr[v];
          zi[v] = l * fi[v];
        }
      }
      cpass16_f32(zr, zi, B[kInvRe], B[kInvIm], re, im);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        zr[v] = re[v];
        zi[v] = im[v];
      }
      cpass16_f32(zr, zi, B[kInvRe], B[kInvIm], re, im);
      if (q < a.P) {
#pragma unroll
        for (int v = 0; v < 4; ++v) gain[v] += static_cast<double>(re[v] * im[v]);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) lf[v] = re[v];
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) gain[v] -= static_cast<double>(fv[v]) * static_cast<double>(lf[v]);
    finish_cell<OUT, Lay16>(a, cell, fv, gain, lane);
  }
}

}  // namespace
}  // namespace qcoll
