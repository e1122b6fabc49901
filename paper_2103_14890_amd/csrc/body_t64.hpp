// Per-cell body of the 2D kernels for grids of n = 2 n' points per axis with
// n' <= 32 (n = 36..64, e.g. 48 and 64), shared by the single-plan kernels and
// the batched multi-plan kernel.
//
// One workgroup of four wavefronts evaluates one cell. The n-point DFTs are
// split once by parity (radix 2) into n'-point DFTs that run on the
// register-resident 32x32-tile machinery of the N <= 32 kernels:
//
//   forward:  f_hat[k' + n'a] = sum_p (-1)^(a.p) w^(-k'.p) F_p[k'],
//             F_p = n'-point 2D DFT of the sub-grid f[2m + p]
//   inverse:  y[2m + p] = n'-point 2D inverse DFT over k' of
//             G_p[k'] = w^(k'.p) sum_a (-1)^(a.p) Z[k' + n'a]
//
// with w = exp(2 pi i / n), a, p in {0,1}^2 (one per axis) and k' in
// [0, n')^2. Wavefront w = 2 w1 + w2 holds the mode quarter a = (w1, w2) of
// the spectrum (f_hat and the filter values there) and computes the output
// parity class p = (w1, w2) of the grid. Between the two roles the quarters
// are exchanged through LDS in FP64 (true values), once for the forward
// transform and once per filter. The row twiddle w^(k1' p1) comes from a small
// broadcast table in LDS, the column twiddle w^(k2' p2) is one complex number
// per lane.

#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "body_t32.hpp"

namespace qcoll {
namespace {

// LDS (79 KB, so that two cells' workgroups share a CU): four complex FP64
// 32x32 slots in [slot][register][lane] order (a lane's 16-byte value for
// register v of slot s sits at (s * 16 + v) * 64 + lane), the row-twiddle table
// [p1][k1'], a small reduction area and the DFT-matrix table. A mode's twiddle
// w^(k'.p) is formed where it is used, as the row twiddle (broadcast from the
// table) times the lane's column twiddle.
constexpr int kZSlot = 16 * 64;                      // complex values per slot
constexpr int kT64LdsBytes = (4 * kZSlot + 2 * 32 + 8 * 4) * 16 + kEoLdsBytes;

// 16-byte aligned, so that a lane's complex value is one ds_read_b128 /
// ds_write_b128 (two 8-byte halves with a 16-byte lane stride conflict in
// the LDS banks)
struct alignas(16) Cd {
  double x, y;
};

typedef double dbl2v __attribute__((ext_vector_type(2)));   // 16-byte store units
typedef float flt4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ Cd cmul(Cd a, Cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// Parity sub-grid x[m1][m2] = f[2 m1 + p1][2 m2 + p2] of one cell in the 32x32
// result-tile layout, zero outside n' x n'. The lane index is opaque so that the
// addresses are formed here rather than hoisted out of the cell loop.
__device__ __forceinline__ void load_subgrid(const KernelArgs& a, int64_t cell, int p1, int p2, float* fv) {
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  const int h = lane >> 5, c = lane & 31;
  const int n = a.n, np = n >> 1;
  const float* fc = a.f + cell * static_cast<int64_t>(n) * n;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int r = rrow(v, h);
    fv[v] = load_or_zero(fc, r < np && c < np, (2 * r + p1) * n + 2 * c + p2);
  }
}

// Per-lane operands of the n'-point DFT matrices for the FP32 variant
// (v_mfma_f32_32x32x2f32): for register v, E[rrow(v, h)][c] of cos, sin and
// -sin, zero outside n' x n'.
struct E32 {
  float r[16], i[16], n[16];
};

// The FP32 variant's forward (real input, then complex) and inverse (complex,
// twice) 32-point tile passes, as in the 32x32 FP32 kernel.
__device__ __forceinline__ void fwd_fp32(const E32& E, const float* fv, f32x16& fre, f32x16& fim) {
  f32x16 re{}, im{};
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    re = mfma32(fv[v], E.r[v], re);
    im = mfma32(fv[v], E.n[v], im);
  }
  fre = fim = f32x16{};
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    fre = mfma32(re[v], E.r[v], fre);
    fre = mfma32(im[v], E.i[v], fre);
    fim = mfma32(re[v], E.n[v], fim);
    fim = mfma32(im[v], E.r[v], fim);
  }
}

__device__ __forceinline__ void inv_fp32(const E32& E, const float* zr, const float* zi, bool want_im, f32x16& yr,
                                         f32x16& yi) {
  f32x16 dr{}, di{};
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    dr = mfma32(zr[v], E.r[v], dr);
    dr = mfma32(zi[v], E.n[v], dr);
    di = mfma32(zr[v], E.i[v], di);
    di = mfma32(zi[v], E.r[v], di);
  }
  yr = yi = f32x16{};
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    yr = mfma32(dr[v], E.r[v], yr);
    yr = mfma32(di[v], E.n[v], yr);
    if (want_im) {
      yi = mfma32(dr[v], E.i[v], yi);
      yi = mfma32(di[v], E.r[v], yi);
    }
  }
}

// FX = true: FX16 DFT-GEMMs (three-part FP16 splits, six products, power-of-two
// scales tracked as integers); FX = false: FP32 DFT-GEMMs, the plain FP32 path.
// Everything between the passes (quarter exchange, twiddles, filter products,
// gain) is FP64 in both; the FP32 variant rounds each pass's input to FP32.
// OUT: 0 eval float, 1 eval double (projection), 2 step, 3 IMEX RK stage, 4
// double without projection; -1 chosen at run time from a.out_kind among 0..2
// (the batched launches). Cells first, first + stride, ...; lds_raw is the
// workgroup's kT64LdsBytes of dynamic LDS (16-byte aligned).
//
// SPLIT (the latency form of batched launches): a.split workgroups share each
// cell: work item i is part i % a.split of cell i / a.split; every part computes
// the spectrum, part j the gain transforms q = j, j + a.split, ... and the part
// P mod a.split the loss; the parts leave their results in a.split_ws and count
// their arrivals in a.split_cnt; the last to arrive adds the parts in the order
// 0, 1, ... and runs the epilogue (first and stride then count work items).
// VEC: Q is written with 16-byte stores (the caller has checked that the output
// is 16-byte aligned; n even makes every cell so), else with element stores.
template <int OUT, bool FX, bool SPLIT = false, bool VEC = false>
__device__ __forceinline__ void t64_body(const KernelArgs& a, int64_t first, int64_t stride, double2* lds_raw) {
  const int kind = OUT < 0 ? a.out_kind : OUT;
  auto can = [](int k) { return OUT == k || (OUT < 0 && k <= 2); };
  double* lds = reinterpret_cast<double*>(lds_raw);
  Cd* zs = reinterpret_cast<Cd*>(lds);                 // [4][16][64]
  Cd* tw = zs + 4 * kZSlot;                            // [2][32]
  double* red = reinterpret_cast<double*>(tw + 64);    // [4 waves][4]
  half8* eo = reinterpret_cast<half8*>(reinterpret_cast<Cd*>(red + 32));  // DFT lo parts

  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (scalar registers)
  const int p1 = w >> 1, p2 = w & 1;                   // parity class = mode quarter
  const int h = lane >> 5, c = lane & 31;
  const int n = a.n, np = n >> 1;

  // row twiddles w^(k1' p1) for both parities, column twiddle of this lane
  for (int i = threadIdx.x; i < 64; i += blockDim.x) tw[i] = {a.tw[2 * i], a.tw[2 * i + 1]};
  const Cd c2 = {a.tw[2 * (32 * p2 + c)], a.tw[2 * (32 * p2 + c) + 1]};
  __syncthreads();
  auto twv = [&](int v) { return cmul(tw[32 * p1 + rrow(v, h)], c2); };

  Lead E[3][2];
  E32 E3;
  if constexpr (FX) {
    load_eo_table(a, eo);
    const half8* src = reinterpret_cast<const half8*>(a.econst) + lane * 18;
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        E[m][s].l = src[(m * 2 + s) * 3 + 0];
      }
  } else {
    (void)eo;
    const float* src = reinterpret_cast<const float*>(a.econst) + lane * 48;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      E3.r[v] = src[v];
      E3.i[v] = src[16 + v];
      E3.n[v] = src[32 + v];
    }
  }
  const double sgn[4] = {1.0, (p2 ? -1.0 : 1.0), (p1 ? -1.0 : 1.0), ((p1 ^ p2) ? -1.0 : 1.0)};

  const int S = SPLIT ? a.split : 1;
  for (int64_t item = first; item < a.cells * S; item += stride) {
    const int64_t cell = SPLIT ? item / S : item;
    const int part = SPLIT ? static_cast<int>(item - cell * S) : 0;
    // ---- own parity sub-grid x[m1][m2] = f[2 m1 + p1][2 m2 + p2]
    float fv[16];
    load_subgrid(a, cell, p1, p2, fv);
    // ---- n'-point 2D DFT of the sub-grid (as in the N <= 32 kernels); the
    // true values are acc * 2^sc (acc = r0 + r1, i0 + i1)
    Split3 A[4];
    f32x16 r0{}, r1{}, i0{}, i1{};
    int sc = 0;
    if constexpr (FX) {
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
      sc = -(a0 + 9);
      const int a1 = 9 - exp_above(tile_absmax(r0, r1, i0, i1));
      slice_tiles(r0, r1, i0, i1, ldexpf(1.0f, a1), A);
      pass64_lo_lds(A, E, eo, kEr, kEi, kNEi, kEr, true, r0, r1, i0, i1);
      sc = sc - a1 - 9;
    } else {
      fwd_fp32(E3, fv, r0, i0);
    }
    // ---- twiddle w^(-k'.p) and exchange: T_p -> f_hat quarter a = w
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const Cd t = twv(v);
      const Cd F = {ldexp(static_cast<double>(r0[v]) + static_cast<double>(r1[v]), sc),
                    ldexp(static_cast<double>(i0[v]) + static_cast<double>(i1[v]), sc)};
      zs[(w * 16 + v) * 64 + lane] = cmul({t.x, -t.y}, F);
    }
    __syncthreads();
    // This wave's spectrum quarter f_hat_a lives in the wave's exchange slot
    // between transforms (the slot is free while the inverse passes run), not
    // in registers: held in registers it spilled 16 VGPRs per lane, whose
    // scratch traffic went to HBM (2.8x the algorithmic bytes per launch, for a
    // launch 3% shorter).
    double fr[16], fi[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const Cd t = zs[(s * 16 + v) * 64 + lane];
        sr += sgn[s] * t.x;
        si += sgn[s] * t.y;
      }
      fr[v] = sr;
      fi[v] = si;
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 16; ++v) zs[(w * 16 + v) * 64 + lane] = {fr[v], fi[v]};

    double gain[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) gain[v] = 0.0;
    int sd_last = 0;
    // one transform: q < P a gain transform (Re * Im of its inverse DFT), q = P
    // the loss multiplier (real part only); the loss transform is issued after
    // the loop so that the loop body has no branch on the kind of transform
    auto transform = [&](int q, auto gain_kind) {
      constexpr bool G = decltype(gain_kind)::value;
      // filtered quarter Z_a (true values) to LDS, with its max |component|
      // filter values of this quarter: [q][quarter][register v][lane] complex,
      // loaded in two batches of eight (the register budget of two workgroups
      // per CU; the other workgroup covers the latency)
      const double2* mq = reinterpret_cast<const double2*>(a.filt) + (static_cast<int64_t>(q) * 4 + w) * kZSlot;
      int ml = lane;
      asm volatile("" : "+v"(ml));
      constexpr int kMv = 8;
      double2 mvv[16];
#pragma unroll
      for (int v = 0; v < kMv; ++v) mvv[v] = mq[v * 64 + ml];
      __builtin_amdgcn_sched_barrier(0);
      // FX16: Z_a is kept as filter mantissas times the spectrum (the filter's
      // power of two 2^filt_exp[q] goes into the slicing scale below, exactly);
      // FP32: true values. The maximum |component| comes from the high words of
      // the doubles: as FP32 bit patterns with the sign cleared they order like
      // the magnitudes (true values can lie outside the FP32 range)
      const double zsc = FX ? 1.0 : ldexp(1.0, a.filt_exp[q]);
      float zmh = 0.0f;
      Cd fq[16];   // f_hat_a, from this wave's slot, which then takes Z_a
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        if (v == kMv) {
#pragma unroll
          for (int u = kMv; u < 16; ++u) mvv[u] = mq[u * 64 + ml];
          __builtin_amdgcn_sched_barrier(0);
        }
        fq[v] = zs[(w * 16 + v) * 64 + lane];
        const double mr = FX ? mvv[v].x : mvv[v].x * zsc, mi = FX ? mvv[v].y : mvv[v].y * zsc;
        const Cd z = {mr * fq[v].x - mi * fq[v].y, mr * fq[v].y + mi * fq[v].x};
        zs[(w * 16 + v) * 64 + lane] = z;
        if (FX)   // one v_max3_f32 with |.| operand modifiers (in C the abs becomes an integer and)
          asm("v_max3_f32 %0, |%1|, |%2|, %3"
              : "=v"(zmh)
              : "v"(__double2hiint(z.x)), "v"(__double2hiint(z.y)), "v"(zmh));
        if (v & 1) __builtin_amdgcn_sched_barrier(0);
      }
      if constexpr (FX) {
        // an upper bound of the wave's maximum (the high word rounded up)
        const int hb = __float_as_int(wave_max(zmh));
        if (lane == 0) red[w * 4 + 3] = hb > 0 ? __hiloint2double(hb + 1, 0) : 0.0;
      }
      __syncthreads();
      // |G_p| <= sum_a max |Z_a| (twiddles have modulus one): common slicing scale
      int b = 0;
      if constexpr (FX) b = 9 - (exp_above_d((red[3] + red[7] + red[11] + red[15]) * 1.0000005) + 1);
      // G_p = w^(k'.p) sum_a (-1)^(a.p) Z_a for this wave's parity class, split
      // into the left operand of the first inverse pass as it is formed (FP32:
      // rounded to the FP32 operand)
      // (FX16: the scale 2^b rides on the lane's column twiddle, exactly)
      const Cd c2b = FX ? Cd{ldexp(c2.x, b), ldexp(c2.y, b)} : c2;
      float zr[16], zi[16];
#pragma unroll
      for (int v = 0; v < 16; v += 2) {
        double gr[2], gi[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          double sr = 0.0, si = 0.0;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const Cd t = zs[(s * 16 + v + u) * 64 + lane];
            sr += sgn[s] * t.x;
            si += sgn[s] * t.y;
          }
          const Cd g = cmul(cmul(tw[32 * p1 + rrow(v + u, h)], c2b), {sr, si});
          gr[u] = g.x;
          gi[u] = g.y;
        }
        if constexpr (FX) {
          put2(A[v >> 3], v & 7, split2_f64(gr[0], gr[1]));
          put2(A[2 + (v >> 3)], v & 7, split2_f64(gi[0], gi[1]));
        } else {
          zr[v] = static_cast<float>(gr[0]);
          zr[v + 1] = static_cast<float>(gr[1]);
          zi[v] = static_cast<float>(gi[0]);
          zi[v + 1] = static_cast<float>(gi[1]);
        }
        __builtin_amdgcn_sched_barrier(0);  // bound the LDS reads in flight
      }
      __syncthreads();
      // every wave has read the Z slots: f_hat_a back into this wave's slot
#pragma unroll
      for (int v = 0; v < 16; ++v) zs[(w * 16 + v) * 64 + lane] = fq[v];
      if constexpr (FX) {
        pass64_lo_lds(A, E, eo, kEr, kNEi, kEi, kEr, true, r0, r1, i0, i1);
        int sd = a.filt_exp[q] - b - 9;   // Z_a carried the filter mantissas
        const int a2 = 9 - exp_above(tile_absmax(r0, r1, i0, i1));
        slice_tiles(r0, r1, i0, i1, ldexpf(1.0f, a2), A);
        pass64_lo_lds(A, E, eo, kEr, kNEi, kEi, kEr, G, r0, r1, i0, i1);  // loss: real part only
        sd = sd - a2 - 9;
        if constexpr (G) {
          const double wq = ldexp(1.0, 2 * sd);
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            double re = static_cast<double>(r0[v]) + static_cast<double>(r1[v]);
            double im = static_cast<double>(i0[v]) + static_cast<double>(i1[v]);
            gain[v] = fma(re * wq, im, gain[v]);
          }
        } else {
          sd_last = sd;
        }
      } else {
        inv_fp32(E3, zr, zi, G, r0, i0);   // loss: real part only
        if constexpr (G) {
#pragma unroll
          for (int v = 0; v < 16; ++v) gain[v] += static_cast<double>(r0[v] * i0[v]);
        }
      }
    };
    // the loss transform first (the loss term -f * L starts the gain sum), so
    // that its read of f follows the first one closely enough to hit the
    // cache: evaluations fetch f from memory once per cell. Then the gain
    // transforms. (The split form keeps the loss last: its part P mod S.)
    const bool own_loss = !SPLIT || part == a.P % S;   // workgroup-uniform
    auto loss_term = [&]() {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const double lf = FX ? ldexp(static_cast<double>(r0[v]) + static_cast<double>(r1[v]), sd_last)
                             : static_cast<double>(r0[v]);
        gain[v] -= static_cast<double>(fv[v]) * lf;
      }
    };
    if constexpr (!SPLIT) {
      transform(a.P, std::false_type{});
      load_subgrid(a, cell, p1, p2, fv);   // not held in registers through the forward transform
      loss_term();
    }
    for (int q = part; q < a.P; q += S) transform(q, std::true_type{});
    if constexpr (SPLIT) {
      if (own_loss) transform(a.P, std::false_type{});
      load_subgrid(a, cell, p1, p2, fv);
      if (own_loss) loss_term();
    } else if ((can(2) && kind == 2) || (can(3) && kind == 3)) {
      load_subgrid(a, cell, p1, p2, fv);   // the updates read f again (not held through the transforms)
    }
    if constexpr (SPLIT) {
      double* mine = a.split_ws + ((cell * S + part) * 4 + w) * 1024;
#pragma unroll
      for (int v = 0; v < 16; ++v) mine[v * 64 + lane] = gain[v];
      __threadfence();   // the part is visible device-wide before it is counted
      __syncthreads();
      if (threadIdx.x == 0) red[20] = atomicAdd(&a.split_cnt[cell], 1) == S - 1 ? 1.0 : 0.0;
      __syncthreads();
      const bool last = red[20] != 0.0;
      __syncthreads();   // red is reused by the epilogue
      if (!last) continue;
      __threadfence();   // the other parts' results are read after their counts
#pragma unroll
      for (int v = 0; v < 16; ++v) gain[v] = 0.0;
      for (int j = 0; j < S; ++j) {
        const double* pj = a.split_ws + ((cell * S + j) * 4 + w) * 1024;
#pragma unroll
        for (int v = 0; v < 16; ++v) gain[v] += pj[v * 64 + lane];
      }
      if (threadIdx.x == 0) a.split_cnt[cell] = 0;   // zero for the next launch
    }

    // ---- epilogue on this wave's parity class; cell-wide sums through LDS.
    // Results and stage slots stream through L2 with non-temporal accesses, so
    // that they do not evict the filter table all cells of a CU share. The
    // lane indices are re-derived from an opaque copy so that the per-point
    // velocities and addresses are not hoisted out of the cell loop.
    int elane = lane;
    asm volatile("" : "+v"(elane));
    const int h = elane >> 5, c = elane & 31;
    const double v2c = -a.L + a.dv * (2 * c + p2);
    // Q leaves through LDS: each wave puts its parity class in row-major order
    // into the exchange slots (free after the last transform), then the
    // workgroup writes whole rows. Stored directly, the classes interleave at
    // every other element, and each cache line reaches memory in halves.
    auto store_q = [&](auto* Qc, auto value) {
      using T = std::remove_reference_t<decltype(*Qc)>;
      T* st = reinterpret_cast<T*>(zs);
      __syncthreads();   // every wave has written its slot back
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = rrow(v, h);
        if (r < np && c < np) st[(2 * r + p1) * n + 2 * c + p2] = value(v);
      }
      __syncthreads();
      // consecutive lanes at consecutive addresses (whole rows)
      if constexpr (VEC) {
        using T4 = typename std::conditional<sizeof(T) == 8, dbl2v, flt4v>::type;
        constexpr int kPer = 16 / sizeof(T);
        const T4* st4 = reinterpret_cast<const T4*>(st);
        T4* q4 = reinterpret_cast<T4*>(Qc);
        for (int i = threadIdx.x; i < n * n / kPer; i += blockDim.x) __builtin_nontemporal_store(st4[i], &q4[i]);
      } else {
        for (int i = threadIdx.x; i < n * n; i += blockDim.x) __builtin_nontemporal_store(st[i], &Qc[i]);
      }
      __syncthreads();   // the next cell writes the slots
    };
    if (can(4) && kind == 4) {  // double Q without projection (fine-grid stage of the Galerkin variant)
      double* Qc = reinterpret_cast<double*>(a.q) + cell * static_cast<int64_t>(n) * n;
      store_q(Qc, [&](int v) { return gain[v]; });
    } else if (can(0) && kind == 0) {
      float* Qc = reinterpret_cast<float*>(a.q) + cell * static_cast<int64_t>(n) * n;
      store_q(Qc, [&](int v) { return static_cast<float>(gain[v]); });
    } else if (can(1) && kind == 1) {
      double m[4] = {0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const double v1 = -a.L + a.dv * (2 * rrow(v, h) + p1);
        m[0] += gain[v];
        m[1] += v1 * gain[v];
        m[2] += v2c * gain[v];
        m[3] += (v1 * v1 + v2c * v2c) * gain[v];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) m[i] = wave_sum(m[i]);
      if (lane == 0)
        for (int i = 0; i < 4; ++i) red[w * 4 + i] = m[i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 4; ++i) m[i] = red[i] + red[4 + i] + red[8 + i] + red[12 + i];
      __syncthreads();
      double lam[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        lam[i] = a.gram_inv[i * 4 + 0] * m[0] + a.gram_inv[i * 4 + 1] * m[1] + a.gram_inv[i * 4 + 2] * m[2] +
                 a.gram_inv[i * 4 + 3] * m[3];
      double* Qc = reinterpret_cast<double*>(a.q) + cell * static_cast<int64_t>(n) * n;
      store_q(Qc, [&](int v) {
        const double v1 = -a.L + a.dv * (2 * rrow(v, h) + p1);
        return gain[v] - (lam[0] + lam[1] * v1 + lam[2] * v2c + lam[3] * (v1 * v1 + v2c * v2c));
      });
    } else if (can(3) && kind == 3) {
      // stage l of the penalised IMEX RK step (as finish_cell<3> of the 32x32
      // kernels); fv holds the input F_{l-1}, gain its Q (FP64)
      // The scheme and stage indices are made opaque here, so that the tableau
      // coefficients are loaded in the epilogue of each cell: hoisted out of
      // the cell loop they would occupy scalar registers through the filter
      // loop, whose spills to vector lanes cost it its overlapped LDS reads.
      int sch = a.rk_scheme - 1, l = a.rk_stage;
      asm volatile("" : "+s"(sch), "+s"(l));
      const int ns = sch == 0 ? 3 : 5;   // stages of the scheme
      const double* At = kRkAt[sch][l - 1];
      const double* Ai = kRkA[sch][l - 1];
      const int64_t base = cell * static_cast<int64_t>(n) * n;
      float* fnp = a.rk_fn + base;
      // f^n is read twice (moments, then the update) instead of being held in
      // registers through the stage sums
      double sm[4] = {0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = rrow(v, h);
        const double v1 = -a.L + a.dv * (2 * r + p1);
        const double fnv = (r < np && c < np) ? static_cast<double>(fnp[(2 * r + p1) * n + 2 * c + p2]) : 0.0;
        sm[0] += fnv;
        sm[1] += v1 * fnv;
        sm[2] += v2c * fnv;
        sm[3] += (v1 * v1 + v2c * v2c) * fnv;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) sm[i] = wave_sum(sm[i]);
      if (lane == 0)
        for (int i = 0; i < 4; ++i) red[w * 4 + i] = sm[i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 4; ++i) sm[i] = red[i] + red[4 + i] + red[8 + i] + red[12 + i];
      __syncthreads();
      const double rho = sm[0] * a.dv * a.dv, u1 = sm[1] / sm[0], u2 = sm[2] / sm[0];
      const double Tm = 0.5 * (sm[3] / sm[0] - u1 * u1 - u2 * u2);
      const double nu = rho, k = a.dt_eps;
      const double cM = rho / (2.0 * 3.14159265358979323846 * Tm);
      const double den = 1.0 + Ai[l - 1] * k * nu;
      const double* ec = exp_consts();
      // the Maxwellian factors by velocity axis, M = cM e1(v1) e2(v2): this
      // lane's column factor, and the factor of this wave's row 2 (lane mod 32)
      // + p1, which the rows fetch from that lane
      const double e2 = exp_nonpos(-(v2c - u2) * (v2c - u2) / (2.0 * Tm), ec);
      const double vr = -a.L + a.dv * (2 * (lane & 31) + p1);
      const double e1 = exp_nonpos(-(vr - u1) * (vr - u1) / (2.0 * Tm), ec);
      int bad = 0;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = rrow(v, h);
        const double M = cM * __shfl(e1, r) * e2;   // (every lane takes part in the exchange)
        if (!(r < np && c < np)) continue;
        const int o = (2 * r + p1) * n + 2 * c + p2;
        const double fnv = static_cast<double>(fnp[o]);
        double rhs = fnv + Ai[l - 1] * k * nu * M;
        for (int m = 1; m < l; ++m) {
          const double Fm = m == 1 ? fnv
                            : (m == l - 1 ? static_cast<double>(fv[v])
                                          : static_cast<double>(__builtin_nontemporal_load(&a.rk_work[(m - 2) * a.rk_stride + base + o])));
          const double Sm = nu * (M - Fm);
          double acc = Ai[m - 1] * Sm;
          if (At[m - 1] != 0.0) {
            const double Qm =
                m == l - 1 ? gain[v] : static_cast<double>(__builtin_nontemporal_load(&a.rk_work[(ns - 3 + m) * a.rk_stride + base + o]));
            acc += At[m - 1] * (Qm - Sm);
          }
          rhs += k * acc;
        }
        const float Fl = static_cast<float>(rhs / den);
        if (l == ns) {
          bad |= !(fabsf(Fl) <= 3.0e38f);
          __builtin_nontemporal_store(Fl, &fnp[o]);
        } else {
          __builtin_nontemporal_store(Fl, &a.rk_work[(l - 2) * a.rk_stride + base + o]);
          __builtin_nontemporal_store(static_cast<float>(gain[v]), &a.rk_work[(ns - 3 + (l - 1)) * a.rk_stride + base + o]);
        }
      }
      if (l == ns && a.status) {
        bad = __any(bad) ? 1 : 0;
        if (lane == 0) red[w * 4 + 1] = bad;
        __syncthreads();
        if (threadIdx.x == 0) a.status[cell] = (red[1] + red[5] + red[9] + red[13]) > 0 ? 1 : 0;
        __syncthreads();
      }
    } else {
      double rho = 0.0;
#pragma unroll
      for (int v = 0; v < 16; ++v) rho += static_cast<double>(fv[v]);
      rho = wave_sum(rho);
      if (lane == 0) red[w * 4] = rho;
      __syncthreads();
      rho = (red[0] + red[4] + red[8] + red[12]) * a.dv * a.dv;
      __syncthreads();
      const double k = a.scheme == 1 ? a.dt_eps / (1.0 + a.dt_eps * rho) : a.dt_eps;
      float* fcell = const_cast<float*>(a.f) + cell * static_cast<int64_t>(n) * n;
      int bad = 0;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = rrow(v, h);
        const float nv = static_cast<float>(static_cast<double>(fv[v]) + k * gain[v]);
        if (r < np && c < np) {
          bad |= !(fabsf(nv) <= 3.0e38f);
          __builtin_nontemporal_store(nv, &fcell[(2 * r + p1) * n + 2 * c + p2]);
        }
      }
      if (a.status) {
        bad = __any(bad) ? 1 : 0;
        if (lane == 0) red[w * 4 + 1] = bad;
        __syncthreads();
        if (threadIdx.x == 0)
          a.status[cell] = (red[1] + red[5] + red[9] + red[13]) > 0 ? 1 : 0;
        __syncthreads();
      }
    }
  }
}


}  // namespace
}  // namespace qcoll
