// Per-cell bodies of the 2D kernels on 32x32 MFMA tiles (grids of 18..32
// points per axis, zero-padded), shared by the single-plan and the batched
// multi-plan kernels.
#pragma once

#include <type_traits>

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

// Bound on the magnitudes of a complex result tile held as accumulator pairs:
// max (|acc0| + |acc1|) bounds both |acc0| (the part that becomes the lead of
// the next split) and |acc0 + acc1|. (The sums are canonical floats, so the
// maxima need no NaN quieting and fold into v_max3.)
__device__ __forceinline__ float tile_absmax(const f32x16& r0, const f32x16& r1, const f32x16& i0,
                                             const f32x16& i1) {
  float m = 0.0f;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    m = fmaxf(m, fabsf(r0[v]) + fabsf(r1[v]));
    m = fmaxf(m, fabsf(i0[v]) + fabsf(i1[v]));
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

// DFT-matrix operands with the hi and lo parts in LDS: the leads stay in
// registers (24 VGPRs), the hi and lo parts are read from a block-shared LDS
// table right before their products: lo at [mat][K-slice][lane], hi
// kEoHiOffset entries further.
struct Lead {
  half8 l;
};

constexpr int kEoHiOffset = 6 * 64;

__device__ __forceinline__ void mma6_lo_lds(const Split3& a, const Lead& b, const half8* bo, f32x16& acc0,
                                            f32x16& acc1) {
  const half8 b_o = bo[0];
  const half8 b_h = bo[kEoHiOffset];
  acc0 = mfma16(a.l, b.l, acc0);
  acc1 = mfma16(a.h, b.l, acc1);
  acc1 = mfma16(a.o, b.l, acc1);
  acc1 = mfma16(a.l, b_h, acc1);
  acc1 = mfma16(a.h, b_h, acc1);
  acc1 = mfma16(a.l, b_o, acc1);
}

// pass64 with Lead operands; eo is the LDS table of hi and lo parts. An opaque lane
// index keeps the table reads inside the caller's loops.
__device__ __forceinline__ void pass64_lo_lds(const Split3 A[4], const Lead E[3][2], const half8* eo, int re_a,
                                              int re_b, int im_a, int im_b, bool want_im, f32x16& r0, f32x16& r1,
                                              f32x16& i0, f32x16& i1) {
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  r0 = r1 = i0 = i1 = f32x16{};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    mma6_lo_lds(A[s], E[re_a][s], eo + (re_a * 2 + s) * 64 + lane, r0, r1);
    mma6_lo_lds(A[2 + s], E[re_b][s], eo + (re_b * 2 + s) * 64 + lane, r0, r1);
    if (want_im) {
      mma6_lo_lds(A[s], E[im_a][s], eo + (im_a * 2 + s) * 64 + lane, i0, i1);
      mma6_lo_lds(A[2 + s], E[im_b][s], eo + (im_b * 2 + s) * 64 + lane, i0, i1);
    }
  }
}

// Fill the block-shared LDS table of DFT-matrix lo parts (all threads of the
// workgroup take part; ends with a workgroup barrier).
__device__ __forceinline__ void load_eo_table(const KernelArgs& a, half8* eo) {
  const half8* src = reinterpret_cast<const half8*>(a.econst);
  for (int i = threadIdx.x; i < 2 * kEoHiOffset; i += blockDim.x) {
    const int part = i < kEoHiOffset ? 2 : 1;   // lo, then hi
    const int j = i < kEoHiOffset ? i : i - kEoHiOffset;
    const int ms = j >> 6, ln = j & 63;
    eo[i] = src[ln * 18 + ms * 3 + part];
  }
  __syncthreads();
}

// Byte offset of this lane's entry in a [register][lane] table of 16-byte
// values, kept opaque so that per-register addresses are formed where they are
// used (a uniform base plus a 32-bit lane offset) instead of being hoisted into
// sixteen 64-bit VGPR pairs.
__device__ __forceinline__ unsigned opaque_lane16(int lane) {
  unsigned o = static_cast<unsigned>(lane) * 16u;
  asm volatile("" : "+v"(o));
  return o;
}

// Filter value of transform q, register v, from the table [q][v][lane].
__device__ __forceinline__ double2 load_filter_value(const double* filt, int q, int v, unsigned l16) {
  const char* base = reinterpret_cast<const char*>(filt) + static_cast<size_t>(q) * (16 * 64 * 16);
  return *reinterpret_cast<const double2*>(base + (static_cast<unsigned>(v) * 1024u + l16));
}

// Filtered spectrum Z = m * f_hat for all 16 modes of a lane (FP64, |Z| < 2^8),
// split into the left operand of inverse pass A. The spectrum is re-read from
// LDS for every transform: an opaque lane offset keeps the compiler from
// hoisting the reads into 64 live VGPRs.
__device__ __forceinline__ void filtered_split(const double2* mv, const double2* fh, int lane, Split3 A[4]) {
  asm volatile("" : "+v"(lane));
#pragma unroll
  for (int v = 0; v < 16; v += 2) {
    const double2 m0 = mv[v], m1 = mv[v + 1];
    const double2 f0 = fh[v * 64 + lane], f1 = fh[(v + 1) * 64 + lane];
    const double yr0 = m0.x * f0.x - m0.y * f0.y, yi0 = m0.x * f0.y + m0.y * f0.x;
    const double yr1 = m1.x * f1.x - m1.y * f1.y, yi1 = m1.x * f1.y + m1.y * f1.x;
    put2(A[v >> 3], v & 7, split2_f64(yr0, yr1));
    put2(A[2 + (v >> 3)], v & 7, split2_f64(yi0, yi1));
  }
}

// LDS of the FX16 body: per wavefront the cell's spectrum as FP64 complex
// values in [register][lane] order, per workgroup the table of DFT-matrix lo
// and hi parts.
constexpr int kFhatLdsBytes = 16 * 64 * 16;
constexpr int kEoLdsBytes = 2 * kEoHiOffset * 16;

// FX16 body. Register budget: at most 256 VGPRs per lane, so that two
// wavefronts share each SIMD and the matrix-core work of one overlaps the
// vector work (splits, FP64 filtering and gain) of the other. The spectrum
// lives in LDS (`fh`, this wavefront's kFhatLdsBytes), the filters stream from
// L2 in mode pairs, and per transform the phases run in order: split of the
// filtered spectrum, inverse pass A, slicing, inverse pass B, gain.
//
// SPLIT (latency form, one cell per workgroup of four wavefronts): the four
// wavefronts compute the spectrum each, then share the cell's transforms
// (wavefront w takes the gain transforms q = w, w + 4, ...; the one with
// w = P mod 4 also the loss), and wavefront 0 sums the four partial results in
// a fixed order from LDS and runs the epilogue. first and stride then count
// cells per workgroup; fh is this wavefront's region of four consecutive ones.
template <int OUT, bool SPLIT = false>  // OUT: 0 eval float, 1 eval double (projection), 2 step, -1 from a.out_kind
__device__ __forceinline__ void fx16_t32_body(const KernelArgs& a, int64_t first, int64_t stride, double2* fh,
                                              const half8* eo) {
  const int lane = threadIdx.x & 63;
  const int wv = SPLIT ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;   // wavefront of the cell
  const int q0 = SPLIT ? (wv < a.P ? wv : a.P) : 0;   // first transform (clamped: a valid table entry)
  constexpr int qs = SPLIT ? 4 : 1;                   // transform step
  const bool own_loss = !SPLIT || wv == a.P % 4;

  // DFT-matrix operands (Er, Ei, -Ei; two K-slices; lead and hi per lane; the
  // lo parts in the LDS table eo).
  Lead E[3][2];
  {
    const half8* src = reinterpret_cast<const half8*>(a.econst) + lane * 18;
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        E[m][s].l = src[(m * 2 + s) * 3 + 0];
      }
  }

  for (int64_t cell = first; cell < a.cells; cell += stride) {
    f32x16 r0{}, r1{}, i0{}, i1{};
    Split3 A[4];
    int s_fh;
    {
      float fv[16];
      load_cell<Lay32>(a, cell, lane, fv);

      // ---- forward pass 1 (real input, contraction over the first axis)
      float fm = 0.0f;
#pragma unroll
      for (int v = 0; v < 16; ++v) fm = fmaxf(fm, fabsf(fv[v]));
      fm = wave_max(fm);
      const int a0 = 9 - exp_above(fm);
      const double cf = ldexp(1.0, a0);  // FP64: 2^a0 exceeds the FP32 range for max|f| < 2^-118
#pragma unroll
      for (int v = 0; v < 16; v += 2)
        put2(A[v >> 3], v & 7, split2_f64(static_cast<double>(fv[v]) * cf, static_cast<double>(fv[v + 1]) * cf));
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        mma6_lo_lds(A[s], E[kEr][s], eo + (kEr * 2 + s) * 64 + lane, r0, r1);
        mma6_lo_lds(A[s], E[kNEi][s], eo + (kNEi * 2 + s) * 64 + lane, i0, i1);
      }
      s_fh = -(a0 + 9);  // true value = accumulator * 2^s_fh
    }

    // ---- forward pass 2 (complex, contraction over the second axis)
    {
      const int a1 = 9 - exp_above(tile_absmax(r0, r1, i0, i1));
      slice_tiles(r0, r1, i0, i1, ldexpf(1.0f, a1), A);
      pass64_lo_lds(A, E, eo, kEr, kEi, kNEi, kEr, true, r0, r1, i0, i1);
      s_fh -= a1 + 9;
    }

    // unnormalised spectrum in FP64 to LDS, rescaled so that |f_hat| < 2^8
    {
      float fhm = 0.0f;
#pragma unroll
      for (int v = 0; v < 16; ++v)
        fhm = fmaxf(fhm, fmaxf(fabsf(r0[v] + r1[v]), fabsf(i0[v] + i1[v])));
      fhm = wave_max(fhm * 1.0000002f);
      const int bsh = 9 - (exp_above(fhm) + 1);
#pragma unroll
      for (int v = 0; v < 16; ++v)
        fh[v * 64 + lane] = make_double2(ldexp(static_cast<double>(r0[v]) + static_cast<double>(r1[v]), bsh),
                                         ldexp(static_cast<double>(i0[v]) + static_cast<double>(i1[v]), bsh));
      s_fh -= bsh;  // true f_hat = stored value * 2^s_fh
    }

    double gain[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) gain[v] = 0.0;

    // Packed transforms q = 0..P-1 contribute Re * Im of their inverse DFT to the
    // gain; entry P of the table is the real loss multiplier, whose inverse DFT
    // (real part) is the loss field.
    // Filter values [q][mode v][lane] (complex FP64, 1 KB per wavefront and
    // register): all 16 of a transform are loaded in one batch, those of
    // transform q+1 as soon as the operands of pass B of transform q are dead,
    // so that their latency overlaps the gain update. The loop is rotated so
    // that each batch is consumed in the iteration that loads it.
    {
      double2 mv[16];
      const unsigned l16 = opaque_lane16(lane);
#pragma unroll
      for (int v = 0; v < 16; ++v) mv[v] = load_filter_value(a.filt, q0, v, l16);
      filtered_split(mv, fh, lane, A);
    }
    for (int q = (SPLIT ? wv : 0); q < a.P; q += qs) {
      const int qn = q + qs < a.P ? q + qs : a.P;   // next transform of this wavefront (or the loss entry)
      // inverse pass A (contraction over the first axis)
      pass64_lo_lds(A, E, eo, kEr, kNEi, kEi, kEr, true, r0, r1, i0, i1);
      const int a2 = 9 - exp_above(tile_absmax(r0, r1, i0, i1));
      slice_tiles(r0, r1, i0, i1, ldexpf(1.0f, a2), A);
      // inverse pass B (second axis)
      pass64_lo_lds(A, E, eo, kEr, kNEi, kEi, kEr, true, r0, r1, i0, i1);
      const int sd = a.filt_exp[q] + s_fh - 9 - a2 - 9;  // true field = accumulator * 2^sd
      // first half of the next filter in flight during the gain update, the
      // second half once the accumulators are consumed
      __builtin_amdgcn_sched_barrier(0);
      double2 mv[16];
      const unsigned l16 = opaque_lane16(lane);
#pragma unroll
      for (int v = 0; v < 8; ++v) mv[v] = load_filter_value(a.filt, qn, v, l16);
      __builtin_amdgcn_sched_barrier(0);
      const double w = ldexp(1.0, 2 * sd);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const double re = static_cast<double>(r0[v]) + static_cast<double>(r1[v]);
        const double im = static_cast<double>(i0[v]) + static_cast<double>(i1[v]);
        gain[v] = fma(re * w, im, gain[v]);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int v = 8; v < 16; ++v) mv[v] = load_filter_value(a.filt, qn, v, l16);
      __builtin_amdgcn_sched_barrier(0);
      filtered_split(mv, fh, lane, A);
    }
    float fv[16];
    if (own_loss) {   // wavefront-uniform
      // the loss transform (entry P): only the real part of pass B is needed
      pass64_lo_lds(A, E, eo, kEr, kNEi, kEi, kEr, true, r0, r1, i0, i1);
      const int a2l = 9 - exp_above(tile_absmax(r0, r1, i0, i1));
      slice_tiles(r0, r1, i0, i1, ldexpf(1.0f, a2l), A);
      pass64_lo_lds(A, E, eo, kEr, kNEi, kEi, kEr, false, r0, r1, i0, i1);
      const int sd_loss = a.filt_exp[a.P] + s_fh - 9 - a2l - 9;
      // the last transform is the loss field: Q = gain - f * loss
      load_cell<Lay32>(a, cell, lane, fv, r0[0]);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const double lf = ldexp(static_cast<double>(r0[v]) + static_cast<double>(r1[v]), sd_loss);
        gain[v] = gain[v] - static_cast<double>(fv[v]) * lf;
      }
    }
    if constexpr (SPLIT) {
      // partial results through LDS (each wavefront's spectrum region, free
      // now); wavefront 0 adds them in the order 0, 1, 2, 3
      double* part = reinterpret_cast<double*>(fh);
#pragma unroll
      for (int v = 0; v < 16; ++v) part[v * 64 + lane] = gain[v];
      __syncthreads();
      if (wv == 0) {
#pragma unroll
        for (int k = 1; k < 4; ++k) {
          const double* other = reinterpret_cast<const double*>(fh + k * (kFhatLdsBytes / 16));
#pragma unroll
          for (int v = 0; v < 16; ++v) gain[v] += other[v * 64 + lane];
        }
        load_cell<Lay32>(a, cell, lane, fv, static_cast<float>(gain[0]));
        finish_cell<OUT, Lay32>(a, cell, fv, gain, lane);
      }
      __syncthreads();   // the regions are rewritten by the next cell's spectrum
    } else {
      finish_cell<OUT, Lay32>(a, cell, fv, gain, lane);
    }
  }
}

// ------------------------------------------------------------ FX16 ping-pong
//
// The same computation with eight wavefronts per workgroup, two per SIMD, run
// in alternating phases. A cell's work is a strict alternation of matrix-core
// phases (a DFT pass: 12 or 48 MFMAs) and vector phases (slicing, spectrum
// store and filtered split, gain update, epilogue); every phase ends at a
// workgroup barrier. Wavefronts 4..7 start one phase late, so while the
// wavefront of one pair on a SIMD runs a DFT pass the other runs the vector
// phase before it: the matrix core and the vector ALU of each SIMD work at the
// same time by construction instead of by chance. All wavefronts execute the
// same number of barriers: `kmax` cells each (a wavefront with fewer cells
// works on a clamped cell and stores nothing), one stagger barrier at the
// start (late group) or the end (early group).

__device__ __forceinline__ void pp_phase_end() {
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
}

template <int OUT>
__device__ __forceinline__ void fx16_t32_body_pp(const KernelArgs& a, int64_t first, int64_t stride, int64_t kmax,
                                                 bool late, double2* fh, const half8* eo) {
  const int lane = threadIdx.x & 63;
  Lead E[3][2];
  {
    const half8* src = reinterpret_cast<const half8*>(a.econst) + lane * 18;
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        E[m][s].l = src[(m * 2 + s) * 3 + 0];
      }
  }
  if (late) pp_phase_end();

  for (int64_t k = 0; k < kmax; ++k) {
    const int64_t want = first + k * stride;
    const bool valid = want < a.cells;
    const int64_t cell = valid ? want : a.cells - 1;
    f32x16 r0{}, r1{}, i0{}, i1{};
    Split3 A[4];
    int s_fh;
    // [matrix] forward pass 1 (real input, contraction over the first axis)
    {
      float fv[16];
      load_cell<Lay32>(a, cell, lane, fv);
      float fm = 0.0f;
#pragma unroll
      for (int v = 0; v < 16; ++v) fm = fmaxf(fm, fabsf(fv[v]));
      fm = wave_max(fm);
      const int a0 = 9 - exp_above(fm);
      const double cf = ldexp(1.0, a0);  // FP64: 2^a0 exceeds the FP32 range for max|f| < 2^-118
#pragma unroll
      for (int v = 0; v < 16; v += 2)
        put2(A[v >> 3], v & 7, split2_f64(static_cast<double>(fv[v]) * cf, static_cast<double>(fv[v + 1]) * cf));
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        mma6_lo_lds(A[s], E[kEr][s], eo + (kEr * 2 + s) * 64 + lane, r0, r1);
        mma6_lo_lds(A[s], E[kNEi][s], eo + (kNEi * 2 + s) * 64 + lane, i0, i1);
      }
      s_fh = -(a0 + 9);
    }
    pp_phase_end();
    // [vector] slice
    int a1;
    {
      a1 = 9 - exp_above(tile_absmax(r0, r1, i0, i1));
      slice_tiles(r0, r1, i0, i1, ldexpf(1.0f, a1), A);
    }
    pp_phase_end();
    // [matrix] forward pass 2 (complex, contraction over the second axis)
    pass64_lo_lds(A, E, eo, kEr, kEi, kNEi, kEr, true, r0, r1, i0, i1);
    s_fh -= a1 + 9;
    pp_phase_end();
    // [vector] spectrum to LDS (FP64, |f_hat| < 2^8), first filtered split
    double gain[16];
    {
      float fhm = 0.0f;
#pragma unroll
      for (int v = 0; v < 16; ++v)
        fhm = fmaxf(fhm, fmaxf(fabsf(r0[v] + r1[v]), fabsf(i0[v] + i1[v])));
      fhm = wave_max(fhm * 1.0000002f);
      const int bsh = 9 - (exp_above(fhm) + 1);
#pragma unroll
      for (int v = 0; v < 16; ++v)
        fh[v * 64 + lane] = make_double2(ldexp(static_cast<double>(r0[v]) + static_cast<double>(r1[v]), bsh),
                                         ldexp(static_cast<double>(i0[v]) + static_cast<double>(i1[v]), bsh));
      s_fh -= bsh;
#pragma unroll
      for (int v = 0; v < 16; ++v) gain[v] = 0.0;
      double2 mv[16];
      const unsigned l16 = opaque_lane16(lane);
#pragma unroll
      for (int v = 0; v < 16; ++v) mv[v] = load_filter_value(a.filt, 0, v, l16);
      filtered_split(mv, fh, lane, A);
    }
    pp_phase_end();
    for (int q = 0; q < a.P; ++q) {
      // [matrix] inverse pass A
      pass64_lo_lds(A, E, eo, kEr, kNEi, kEi, kEr, true, r0, r1, i0, i1);
      pp_phase_end();
      // [vector] slice
      const int a2 = 9 - exp_above(tile_absmax(r0, r1, i0, i1));
      slice_tiles(r0, r1, i0, i1, ldexpf(1.0f, a2), A);
      pp_phase_end();
      // [matrix] inverse pass B
      pass64_lo_lds(A, E, eo, kEr, kNEi, kEi, kEr, true, r0, r1, i0, i1);
      const int sd = a.filt_exp[q] + s_fh - 9 - a2 - 9;
      pp_phase_end();
      // [vector] gain update and the next filtered split; first half of the
      // next filter in flight during the gain update, the second half once the
      // accumulators are consumed
      __builtin_amdgcn_sched_barrier(0);
      double2 mv[16];
      const unsigned l16 = opaque_lane16(lane);
#pragma unroll
      for (int v = 0; v < 8; ++v) mv[v] = load_filter_value(a.filt, q + 1, v, l16);
      __builtin_amdgcn_sched_barrier(0);
      const double w = ldexp(1.0, 2 * sd);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const double re = static_cast<double>(r0[v]) + static_cast<double>(r1[v]);
        const double im = static_cast<double>(i0[v]) + static_cast<double>(i1[v]);
        gain[v] = fma(re * w, im, gain[v]);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int v = 8; v < 16; ++v) mv[v] = load_filter_value(a.filt, q + 1, v, l16);
      __builtin_amdgcn_sched_barrier(0);
      filtered_split(mv, fh, lane, A);
      pp_phase_end();
    }
    // the loss transform (entry P): [matrix] pass A, [vector] slice, [matrix]
    // the real part of pass B; the epilogue below is its vector phase
    pass64_lo_lds(A, E, eo, kEr, kNEi, kEi, kEr, true, r0, r1, i0, i1);
    pp_phase_end();
    const int a2l = 9 - exp_above(tile_absmax(r0, r1, i0, i1));
    slice_tiles(r0, r1, i0, i1, ldexpf(1.0f, a2l), A);
    pp_phase_end();
    pass64_lo_lds(A, E, eo, kEr, kNEi, kEi, kEr, false, r0, r1, i0, i1);
    const int sd_loss = a.filt_exp[a.P] + s_fh - 9 - a2l - 9;
    pp_phase_end();
    // [vector] epilogue: Q = gain - f * loss
    {
      float fv[16];
      load_cell<Lay32>(a, cell, lane, fv, r0[0]);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const double lf = ldexp(static_cast<double>(r0[v]) + static_cast<double>(r1[v]), sd_loss);
        gain[v] = gain[v] - static_cast<double>(fv[v]) * lf;
      }
      if (valid) finish_cell<OUT, Lay32>(a, cell, fv, gain, lane);
    }
    pp_phase_end();
  }
  if (!late) pp_phase_end();
}

// ------------------------------------------------------------ FP32 variant

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

template <int OUT>  // OUT: 0 eval float, 1 eval double (projection), 2 step, -1 from a.out_kind
__device__ __forceinline__ void fp32_t32_body(const KernelArgs& a, int64_t first, int64_t stride) {
  const int lane = threadIdx.x & 63;
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
    // gain transforms q < P, then the loss multiplier (entry P, real part
    // only), issued after the loop so that the loop body has no branch on the
    // kind of transform
    auto transform = [&](int q, auto gain_kind) {
      constexpr bool loss = !decltype(gain_kind)::value;
      float zr[16], zi[16];
      if constexpr (!loss) {
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
        if constexpr (!loss) {
          yi = mfma32(dr[v], Ei[v], yi);
          yi = mfma32(di[v], Er[v], yi);
        }
      }
      if constexpr (!loss) {
#pragma unroll
        for (int v = 0; v < 16; ++v) gain[v] += static_cast<double>(yr[v] * yi[v]);
      } else {
#pragma unroll
        for (int v = 0; v < 16; ++v)
          gain[v] = gain[v] - static_cast<double>(fv[v]) * static_cast<double>(yr[v]);
      }
    };
    for (int q = 0; q < a.P; ++q) transform(q, std::true_type{});
    transform(a.P, std::false_type{});
    finish_cell<OUT, Lay32>(a, cell, fv, gain, lane);
  }
}

}  // namespace
}  // namespace qcoll
