// Per-cell bodies of the 2D kernels on 32x32 MFMA tiles (grids of 18..32
// points per axis, zero-padded), shared by the single-plan and the batched
// multi-plan kernels.
#pragma once

#include "kernels_common.hpp"

namespace qcoll {
namespace {

constexpr int kN = 32;

__device__ __forceinline__ int rrow(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }


// ------------------------------------------------------------ FX16 (N = 32)

__device__ __forceinline__ f32x16 mfma16(half8 a, half8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// acc0 += a.l*b.l (exact); acc1 += the five remaining products down to 2^-20.
__device__ __forceinline__ void mma6(const Split3& a, const Split3& b, f32x16& acc0, f32x16& acc1) {
  acc0 = mfma16(a.l, b.l, acc0);
  acc1 = mfma16(a.l, b.h, acc1);
  acc1 = mfma16(a.h, b.l, acc1);
  acc1 = mfma16(a.l, b.o, acc1);
  acc1 = mfma16(a.h, b.h, acc1);
  acc1 = mfma16(a.o, b.l, acc1);
}

// Left operand (K = 64: real part rows, then imaginary part rows) from a
// complex result tile held as accumulator pairs.
__device__ __forceinline__ void slice_tiles(const f32x16& r0, const f32x16& r1, const f32x16& i0,
                                            const f32x16& i1, float c, Split3 A[4]) {
#pragma unroll
  for (int v = 0; v < 16; v += 2) {
    put2(A[v >> 3], v & 7, split2_acc(r0[v], r1[v], r0[v + 1], r1[v + 1], c));
    put2(A[2 + (v >> 3)], v & 7, split2_acc(i0[v], i1[v], i0[v + 1], i1[v + 1], c));
  }
}

__device__ __forceinline__ void load_filter(const double* mq, double* m) {
  const double2* src = reinterpret_cast<const double2*>(mq);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    double2 t = src[v];
    m[2 * v] = t.x;
    m[2 * v + 1] = t.y;
  }
}

// Z = m * f_hat for modes v, v+1 of one packed filter (FP64 complex product,
// |Z| < 2^9 by the scaling of m and f_hat), split into the left operand of the
// first inverse pass.
__device__ __forceinline__ void split_spectrum_pair(const double* m, const double* fr, const double* fi,
                                                    Split3 A[4], int v) {
  double yr[2], yi[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    double mr = m[2 * (v + u)], mi = m[2 * (v + u) + 1];
    yr[u] = mr * fr[v + u] - mi * fi[v + u];
    yi[u] = mr * fi[v + u] + mi * fr[v + u];
  }
  put2(A[v >> 3], v & 7, split2_f64(yr[0], yr[1]));
  put2(A[2 + (v >> 3)], v & 7, split2_f64(yi[0], yi[1]));
}

__device__ __forceinline__ void split_spectrum(const double* m, const double* fr, const double* fi,
                                               Split3 A[4]) {
#pragma unroll
  for (int v = 0; v < 16; v += 2) split_spectrum_pair(m, fr, fi, A, v);
}

__device__ __forceinline__ float tile_absmax(const f32x16& r0, const f32x16& r1, const f32x16& i0,
                                             const f32x16& i1) {
  float m = 0.0f;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    m = fmaxf(m, fabsf(r0[v] + r1[v]));
    m = fmaxf(m, fabsf(i0[v] + i1[v]));
  }
  return wave_max(m);
}

// One complex DFT pass (K = 64) with DFT-matrix operands:
//   real out = A_re * B[re_a] + A_im * B[re_b],  imag out = A_re * B[im_a] + A_im * B[im_b]
// where the B index selects Er, Ei or -Ei (0, 1, 2).
__device__ __forceinline__ void pass64(const Split3 A[4], const Split3 E[3][2], int re_a, int re_b,
                                       int im_a, int im_b, bool want_im, f32x16& r0, f32x16& r1,
                                       f32x16& i0, f32x16& i1) {
  r0 = r1 = i0 = i1 = f32x16{};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    mma6(A[s], E[re_a][s], r0, r1);
    mma6(A[2 + s], E[re_b][s], r0, r1);
    if (want_im) {
      mma6(A[s], E[im_a][s], i0, i1);
      mma6(A[2 + s], E[im_b][s], i0, i1);
    }
  }
}

enum { kEr = 0, kEi = 1, kNEi = 2 };

template <int OUT>  // OUT: 0 eval float, 1 eval double (projection), 2 step, -1 from a.out_kind
__device__ __forceinline__ void fx16_t32_body(const KernelArgs& a, int64_t first, int64_t stride) {
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5, c = lane & 31;

  // DFT-matrix operands (Er, Ei, -Ei; two K-slices; lead/hi/lo), per lane.
  Split3 E[3][2];
  {
    const half8* src = reinterpret_cast<const half8*>(a.econst) + lane * 18;
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        E[m][s].l = src[(m * 2 + s) * 3 + 0];
        E[m][s].h = src[(m * 2 + s) * 3 + 1];
        E[m][s].o = src[(m * 2 + s) * 3 + 2];
      }
  }

  for (int64_t cell = first; cell < a.cells; cell += stride) {
    float fv[16];
    load_cell<Lay32>(a, cell, lane, fv);

    // ---- forward pass 1 (real input, contraction over the first axis)
    float fm = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) fm = fmaxf(fm, fabsf(fv[v]));
    fm = wave_max(fm);
    const int a0 = 9 - exp_above(fm);
    const float cf = ldexpf(1.0f, a0);
    Split3 A[4];
#pragma unroll
    for (int v = 0; v < 16; v += 2)
      put2(A[v >> 3], v & 7, split2_f64(static_cast<double>(fv[v] * cf), static_cast<double>(fv[v + 1] * cf)));
    f32x16 r0{}, r1{}, i0{}, i1{};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      mma6(A[s], E[kEr][s], r0, r1);
      mma6(A[s], E[kNEi][s], i0, i1);
    }
    int sc = -(a0 + 9);  // true value = accumulator * 2^sc

    // ---- forward pass 2 (complex, contraction over the second axis)
    int a1 = 9 - exp_above(tile_absmax(r0, r1, i0, i1));
    slice_tiles(r0, r1, i0, i1, ldexpf(1.0f, a1), A);
    pass64(A, E, kEr, kEi, kNEi, kEr, true, r0, r1, i0, i1);
    sc = sc - a1 - 9;

    // unnormalised spectrum in FP64, rescaled so that |f_hat| < 2^9
    double fr[16], fi[16];
    float fhm = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      fr[v] = static_cast<double>(r0[v]) + static_cast<double>(r1[v]);
      fi[v] = static_cast<double>(i0[v]) + static_cast<double>(i1[v]);
      fhm = fmaxf(fhm, fmaxf(fabsf(static_cast<float>(fr[v])), fabsf(static_cast<float>(fi[v]))));
    }
    fhm = wave_max(fhm * 1.0000002f);
    const int bsh = 9 - (exp_above(fhm) + 1);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      fr[v] = ldexp(fr[v], bsh);
      fi[v] = ldexp(fi[v], bsh);
    }
    const int s_fh = sc - bsh;  // true f_hat = fr * 2^s_fh

    double gain[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) gain[v] = 0.0;

    // Packed transforms q = 0..P-1 contribute Re * Im of their inverse DFT to the
    // gain; entry P of the table is the real loss multiplier, whose inverse DFT
    // (real part) is the loss field. Software pipeline: the spectrum of
    // transform q+1 is formed and split while the MFMAs of pass B of transform q
    // run.
    double mbuf[32];
    load_filter(a.filt + static_cast<int64_t>(lane) * 32, mbuf);
    split_spectrum(mbuf, fr, fi, A);
    int sd_last = 0;
    for (int q = 0; q <= a.P; ++q) {
      // prefetch the next filter; its loads complete under pass A
      const int qn = q < a.P ? q + 1 : q;
      load_filter(a.filt + (static_cast<int64_t>(qn) * 64 + lane) * 32, mbuf);
      // inverse pass A (contraction over the first axis)
      pass64(A, E, kEr, kNEi, kEi, kEr, true, r0, r1, i0, i1);
      int sd = a.filt_exp[q] + s_fh - 9;
      const int a2 = 9 - exp_above(tile_absmax(r0, r1, i0, i1));
      Split3 B[4];
      slice_tiles(r0, r1, i0, i1, ldexpf(1.0f, a2), B);
      // inverse pass B (second axis) in 8 chunks of 6 MFMAs, each followed by
      // the split of two modes of the next spectrum (independent VALU work that
      // executes while the matrix cores run)
      r0 = r1 = i0 = i1 = f32x16{};
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        const int s = ch >> 2, part = (ch >> 1) & 1, im = ch & 1;
        const Split3& Aop = B[part ? 2 + s : s];
        const Split3& Bop = E[im ? (part ? kEr : kEi) : (part ? kNEi : kEr)][s];
        if (im) mma6(Aop, Bop, i0, i1);
        else mma6(Aop, Bop, r0, r1);
        split_spectrum_pair(mbuf, fr, fi, A, 2 * ch);
        __builtin_amdgcn_sched_barrier(0);
      }
      sd = sd - a2 - 9;
      sd_last = sd;
      const double w = q < a.P ? ldexp(1.0, 2 * sd) : 0.0;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        double re = static_cast<double>(r0[v]) + static_cast<double>(r1[v]);
        double im = static_cast<double>(i0[v]) + static_cast<double>(i1[v]);
        gain[v] = fma(re * w, im, gain[v]);
      }
    }
    // the last transform is the loss field: Q = gain - f * loss
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      double lf = ldexp(static_cast<double>(r0[v]) + static_cast<double>(r1[v]), sd_last);
      gain[v] = gain[v] - static_cast<double>(fv[v]) * lf;
    }
    finish_cell<OUT, Lay32>(a, cell, fv, gain, lane);
  }
}

// ------------------------------------------------------------ FP32 variant

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

template <int OUT>  // OUT: 0 eval float, 1 eval double (projection), 2 step, -1 from a.out_kind
__device__ __forceinline__ void fp32_t32_body(const KernelArgs& a, int64_t first, int64_t stride) {
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5, c = lane & 31;
  float Er[16], Ei[16], Ne[16];
  {
    const float* src = reinterpret_cast<const float*>(a.econst) + lane * 48;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      Er[v] = src[v];
      Ei[v] = src[16 + v];
      Ne[v] = src[32 + v];
    }
  }
  for (int64_t cell = first; cell < a.cells; cell += stride) {
    float fv[16];
    load_cell<Lay32>(a, cell, lane, fv);
    f32x16 re{}, im{};
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      re = mfma32(fv[v], Er[v], re);
      im = mfma32(fv[v], Ne[v], im);
    }
    f32x16 fre{}, fim{};
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      fre = mfma32(re[v], Er[v], fre);
      fre = mfma32(im[v], Ei[v], fre);
      fim = mfma32(re[v], Ne[v], fim);
      fim = mfma32(im[v], Er[v], fim);
    }
    double gain[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) gain[v] = 0.0;
    for (int q = 0; q <= a.P; ++q) {
      const bool loss = (q == a.P);
      float zr[16], zi[16];
      if (!loss) {
        const float* mq = a.filt32 + (static_cast<int64_t>(q) * 64 + lane) * 32;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          float mr = mq[2 * v], mi = mq[2 * v + 1];
          zr[v] = mr * fre[v] - mi * fim[v];
          zi[v] = mr * fim[v] + mi * fre[v];
        }
      } else {
        const float* lq = a.loss32 + lane * 16;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          zr[v] = lq[v] * fre[v];
          zi[v] = lq[v] * fim[v];
        }
      }
      f32x16 dr{}, di{};
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        dr = mfma32(zr[v], Er[v], dr);
        dr = mfma32(zi[v], Ne[v], dr);
        di = mfma32(zr[v], Ei[v], di);
        di = mfma32(zi[v], Er[v], di);
      }
      f32x16 yr{}, yi{};
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        yr = mfma32(dr[v], Er[v], yr);
        yr = mfma32(di[v], Ne[v], yr);
        if (!loss) {
          yi = mfma32(dr[v], Ei[v], yi);
          yi = mfma32(di[v], Er[v], yi);
        }
      }
      if (!loss) {
#pragma unroll
        for (int v = 0; v < 16; ++v) gain[v] += static_cast<double>(yr[v] * yi[v]);
      } else {
#pragma unroll
        for (int v = 0; v < 16; ++v)
          gain[v] = gain[v] - static_cast<double>(fv[v]) * static_cast<double>(yr[v]);
      }
    }
    finish_cell<OUT, Lay32>(a, cell, fv, gain, lane);
  }
}

}  // namespace
}  // namespace qcoll
