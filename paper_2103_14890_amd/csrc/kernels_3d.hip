// Fast spectral collision operator on 3D velocity grids, gfx950.
//
// Grids of n <= 32 points per axis run zero-padded in a T^3 tile (T = 16 for
// n <= 16, else 32); the DFT matrices are zero outside n x n, so the padding
// never mixes into the result. One workgroup of four wavefronts evaluates one
// cell; cells of several plans (grids) share one launch through a slot table.
//
// The 3D DFT is three passes, one per axis, each a batch of 1-D complex DFTs
// done as MFMA GEMMs over tiles of T lines (section 3.3: the kernel modes
// become A products in Fourier space, each evaluated by FFT-sized transforms):
// FP32 MFMA, or in the FX16 variant split-FP16 MFMA with the FP32 data layout.
// A cell's complex spectrum, the work fields between passes and the FP64 gain
// live in a per-workgroup scratch area (global memory, cached in L2/MALL):
// a 32^3 complex field is 256 KB, more than the LDS of a CU.
//
// Layouts: fields are [i0][i1][i2] with i2 fastest (f and Q use the same order
// with n instead of T). Passes along axes 0 and 1 use the data as the right
// MFMA operand (lines on the lanes: coalesced loads and stores); the pass along
// axis 2 uses the data as the left operand, so that its output has the lines in
// registers and the transformed index on the lanes (coalesced stores). The
// per-lane DFT-matrix values are the same in both roles since E is symmetric.
//
// Per cell: forward passes axis 2, 1, 0 -> spectrum; for each group of packed
// transforms the inverse passes axis 0 (multiplying the spectrum by each
// filter on load), then 1 and 2 plane by plane (accumulating Re * Im into the
// gain, FP64); the last transform is the loss multiplier, whose real field
// gives Q = gain - f * loss. Then the FP64 conservation projection or the
// stage update, as in the 2D kernels.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels_common.hpp"

namespace qcoll {
namespace {

template <int T>
struct Sh;

// v_mfma_f32_32x32x2f32: A 32x2 (lane: row l%32, k l/32), B 2x32 (k l/32,
// column l%32), D 32x32 with column l%32 and 16 rows per lane.
template <>
struct Sh<32> {
  static constexpr int KS = 2, NS = 16, NR = 16;
  typedef f32x16 acc;
  __device__ static int row(int v, int l) { return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3); }
  __device__ static acc mfma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
};

// v_mfma_f32_16x16x4f32: A 16x4 (row l%16, k l/16), B 4x16 (k l/16, column
// l%16), D 16x16 with column l%16 and rows 4 (l/16) + v.
template <>
struct Sh<16> {
  static constexpr int KS = 4, NS = 4, NR = 4;
  typedef f32x4 acc;
  __device__ static int row(int v, int l) { return 4 * (l >> 4) + v; }
  __device__ static acc mfma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

// Per-lane DFT-matrix values: for step s, e(x, j) with x = lane % T and
// j = KS s + lane / T, as cos, sin and -sin of 2 pi x j / n.
template <int T>
struct Emat {
  float c[Sh<T>::NS], s[Sh<T>::NS], ns[Sh<T>::NS];
};

// One complex pass over a tile. Inputs xr, xi: per step, point j of line x
// (DB: data as the right operand, D = E X; otherwise the left operand, D = X E).
// Forward E = C - iS, inverse E = C + iS.
template <int T, bool DB, bool INV, bool REAL_IN>
__device__ __forceinline__ void tile_dft(const Emat<T>& E, const float* xr, const float* xi,
                                         typename Sh<T>::acc& dr, typename Sh<T>::acc& di) {
  using S = Sh<T>;
  dr = typename S::acc{};
  di = typename S::acc{};
#pragma unroll
  for (int s = 0; s < S::NS; ++s) {
    const float c = E.c[s];
    const float sr = INV ? E.ns[s] : E.s[s];  // multiplies xi in the real part
    const float si = INV ? E.s[s] : E.ns[s];  // multiplies xr in the imaginary part
    if (DB) {
      dr = S::mfma(c, xr[s], dr);
      di = S::mfma(si, xr[s], di);
      if (!REAL_IN) {
        dr = S::mfma(sr, xi[s], dr);
        di = S::mfma(c, xi[s], di);
      }
    } else {
      dr = S::mfma(xr[s], c, dr);
      di = S::mfma(xr[s], si, di);
      if (!REAL_IN) {
        dr = S::mfma(xi[s], sr, dr);
        di = S::mfma(xi[s], c, di);
      }
    }
  }
}

// ---- FX16 variant of a 32 x 32 tile pass. The DFT-matrix operands are held
// as three-part FP16 splits of 2^9 e (a lead on the integer grid, hi and lo of
// the remainder) in a workgroup LDS table [cos, sin, -sin][K half][part][lane];
// the tile's data are scaled by a power of two so that |x| < 2^9 and split the
// same way. Six products per operand pair on v_mfma_f32_32x32x16_f16: the lead
// products, exact in FP32, in one accumulator, the five corrections in a
// second. Slot j of K half i on lane l carries the point 2 (8 i + j) + l / 32,
// i.e. step s = 8 i + j of the FP32 layout, so the data arrays of that layout
// are packed without moving between lanes, and the result tile has the FP32
// kernel's layout.
constexpr int kEtabHalf8 = 3 * 2 * 3 * 64;   // 18 KB of LDS

struct EmatFx {
  const half8* tab;   // the LDS table
};

// 16 x 16 tiles: one v_mfma_f32_16x16x32_f16 contracts a line's real and
// imaginary parts together. On lane l (x = l % 16, g = l / 16), K slot j < 4
// carries the real part of point 4 j + g and slot 4 + j its imaginary part:
// the FP32 layout's steps, so again no data move between lanes. The LDS table
// holds, per lane, the matching operand rows [C | S_r] of the real output and
// [S_i | C] of the imaginary output, forward and inverse:
// [dr fwd, dr inv, di fwd, di inv][part][lane].
constexpr int kEtab16Half8 = 4 * 3 * 64;   // 12 KB of LDS

struct EmatFx16 {
  const half8* tab;
};

template <int T, bool FX>
struct EmatOf {
  typedef Emat<T> type;
};
template <>
struct EmatOf<32, true> {
  typedef EmatFx type;
};
template <>
struct EmatOf<16, true> {
  typedef EmatFx16 type;
};

__device__ __forceinline__ f32x4 mfma_h16(half8 a, half8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void mma6_3d16(const Split3& a, const Split3& b, f32x4& acc0, f32x4& acc1) {
  acc0 = mfma_h16(a.l, b.l, acc0);
  acc1 = mfma_h16(a.l, b.h, acc1);
  acc1 = mfma_h16(a.h, b.l, acc1);
  acc1 = mfma_h16(a.l, b.o, acc1);
  acc1 = mfma_h16(a.h, b.h, acc1);
  acc1 = mfma_h16(a.o, b.l, acc1);
}

__device__ __forceinline__ f32x16 mfma_h(half8 a, half8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// acc0 += a.l b.l (exact); acc1 += the five remaining products.
__device__ __forceinline__ void mma6_3d(const Split3& a, const Split3& b, f32x16& acc0, f32x16& acc1) {
  acc0 = mfma_h(a.l, b.l, acc0);
  acc1 = mfma_h(a.l, b.h, acc1);
  acc1 = mfma_h(a.h, b.l, acc1);
  acc1 = mfma_h(a.l, b.o, acc1);
  acc1 = mfma_h(a.h, b.h, acc1);
  acc1 = mfma_h(a.o, b.l, acc1);
}

__device__ __forceinline__ Split3 etab_load(const EmatFx& E, int m, int i, int lane) {
  const half8* q = E.tab + ((m * 2 + i) * 3) * 64 + lane;
  Split3 r;
  r.l = q[0];
  r.h = q[64];
  r.o = q[128];
  return r;
}

// ya, yb scaled so that |y| < 2^9 (FP32 inputs: the split is exact).
__device__ __forceinline__ P3 split2_f32(float ya, float yb) {
  const float na = __builtin_rintf(ya), nb = __builtin_rintf(yb);
  return finish_pair(na, nb, ya - na, yb - nb);
}

template <int T, bool DB, bool INV, bool REAL_IN>
__device__ __forceinline__ void tile_dft(const EmatFx& E, const float* xr, const float* xi, f32x16& dr,
                                         f32x16& di) {
  static_assert(T == 32, "the FX16 tile pass is 32 x 32");
  float m = 0.0f;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    m = fmaxf(m, fabsf(xr[s]));
    if (!REAL_IN) m = fmaxf(m, fabsf(xi[s]));
  }
  m = wave_max(m);
  // 2^sa stays finite: tiles with max |x| < 2^-118 are split with fewer
  // significant bits (the fields are FP32, whose normal range ends at 2^-126)
  const int sa = min(9 - exp_above(m), 127);
  const float c = ldexpf(1.0f, sa);
  Split3 Xr[2], Xi[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
      put2(Xr[i], j, split2_f32(xr[8 * i + j] * c, xr[8 * i + j + 1] * c));
      if (!REAL_IN) put2(Xi[i], j, split2_f32(xi[8 * i + j] * c, xi[8 * i + j + 1] * c));
    }
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  f32x16 r0{}, r1{}, i0{}, i1{};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const Split3 C = etab_load(E, 0, i, lane);
    const Split3 Si = etab_load(E, INV ? 1 : 2, i, lane);  // multiplies xr in the imaginary part
    if (DB) {
      mma6_3d(C, Xr[i], r0, r1);
      mma6_3d(Si, Xr[i], i0, i1);
    } else {
      mma6_3d(Xr[i], C, r0, r1);
      mma6_3d(Xr[i], Si, i0, i1);
    }
    if (!REAL_IN) {
      const Split3 Sr = etab_load(E, INV ? 2 : 1, i, lane);  // multiplies xi in the real part
      if (DB) {
        mma6_3d(Sr, Xi[i], r0, r1);
        mma6_3d(C, Xi[i], i0, i1);
      } else {
        mma6_3d(Xi[i], Sr, r0, r1);
        mma6_3d(Xi[i], C, i0, i1);
      }
    }
  }
  const float inv = ldexpf(1.0f, -(sa + 9));
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    dr[v] = (r0[v] + r1[v]) * inv;
    di[v] = (i0[v] + i1[v]) * inv;
  }
}

template <int T, bool DB, bool INV, bool REAL_IN>
__device__ __forceinline__ void tile_dft(const EmatFx16& E, const float* xr, const float* xi, f32x4& dr,
                                         f32x4& di) {
  static_assert(T == 16, "the 16-point FX16 tile pass");
  float m = 0.0f;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    m = fmaxf(m, fabsf(xr[s]));
    if (!REAL_IN) m = fmaxf(m, fabsf(xi[s]));
  }
  m = wave_max(m);
  // 2^sa stays finite: tiles with max |x| < 2^-118 are split with fewer
  // significant bits (the fields are FP32, whose normal range ends at 2^-126)
  const int sa = min(9 - exp_above(m), 127);
  const float c = ldexpf(1.0f, sa);
  Split3 X;
  put2(X, 0, split2_f32(xr[0] * c, xr[1] * c));
  put2(X, 2, split2_f32(xr[2] * c, xr[3] * c));
  if (REAL_IN) {
    put2(X, 4, split2_f32(0.0f, 0.0f));
    put2(X, 6, split2_f32(0.0f, 0.0f));
  } else {
    put2(X, 4, split2_f32(xi[0] * c, xi[1] * c));
    put2(X, 6, split2_f32(xi[2] * c, xi[3] * c));
  }
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  auto row = [&](int k) {
    const half8* q = E.tab + (k * 3) * 64 + lane;
    Split3 r;
    r.l = q[0];
    r.h = q[64];
    r.o = q[128];
    return r;
  };
  const Split3 Er = row(INV ? 1 : 0), Ei = row(INV ? 3 : 2);
  f32x4 r0{}, r1{}, i0{}, i1{};
  if (DB) {
    mma6_3d16(Er, X, r0, r1);
    mma6_3d16(Ei, X, i0, i1);
  } else {
    mma6_3d16(X, Er, r0, r1);
    mma6_3d16(X, Ei, i0, i1);
  }
  const float inv = ldexpf(1.0f, -(sa + 9));
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    dr[v] = (r0[v] + r1[v]) * inv;
    di[v] = (i0[v] + i1[v]) * inv;
  }
}

// Sum over the workgroup (four wavefronts) of K values per thread.
template <int K>
__device__ __forceinline__ void block_sum(double* x, double* red) {
#pragma unroll
  for (int i = 0; i < K; ++i) x[i] = wave_sum(x[i]);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int i = 0; i < K; ++i) red[w * 8 + i] = x[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < K; ++i) x[i] = red[i] + red[8 + i] + red[16 + i] + red[24 + i];
}

// Per-lane indices are re-derived from an opaque copy of the lane id at the top
// of every tile loop, so that per-lane addresses are formed where they are
// used instead of being hoisted out of the transform loop into hundreds of
// live VGPRs.
#define OPAQUE_LANE()               \
  int lane = threadIdx.x & 63;      \
  asm volatile("" : "+v"(lane));    \
  const int x = lane % T, jl = lane / T; \
  (void)jl

// All tiles t = w, w+4, ... of one axis pass for this wavefront, with the next
// tile's inputs loaded while the current tile's MFMAs run. load(t, xr, xi)
// fetches a tile's inputs, store(t, dr, di) disposes of its outputs; tiles of
// one wavefront touch disjoint lines, so prefetching ahead of the stores is safe.
template <int T, bool DB, bool INV, bool REAL_IN, class EM, class Load, class Store>
__device__ __forceinline__ void pass_tiles(const EM& E, int w, Load load, Store store) {
  using S = Sh<T>;
  float ar[S::NS], ai[S::NS], br[S::NS], bi[S::NS];
  load(w, ar, ai);
#pragma unroll 1
  for (int t = w; t < T; t += 4) {
    if (t + 4 < T) load(t + 4, br, bi);
    typename S::acc dr, di;
    tile_dft<T, DB, INV, REAL_IN>(E, ar, ai, dr, di);
    store(t, dr, di);
#pragma unroll
    for (int s = 0; s < S::NS; ++s) {
      ar[s] = br[s];
      ai[s] = bi[s];
    }
  }
}

// A plane in LDS has rows of T + 1 values: the axis-2 pass reads it by
// columns (lane x takes row x), and with a row stride of T values the lanes of
// a half-wavefront would all fall on the same two LDS banks; with T + 1 they
// fall on distinct ones, while the row-wise writes stay contiguous.
constexpr int kPlaneLds = 32 * 33;

// The inverse passes along axes 1 and 2 of one plane i0 = t (tiles t = w,
// w+4, ... of this wavefront) run back to back: the axis-1 result goes through
// a T x T plane in this wavefront's LDS (its layout has the lines in registers,
// the axis-2 pass needs them on the lanes) instead of through the scratch
// field, so the field is read once and never written between the two passes.
// load(t, xr, xi) fetches plane t's axis-1 inputs (the next plane's while the
// current one computes); store(t, dr, di) disposes of the axis-2 outputs.
template <int T, class EM, class Load, class Store>
__device__ __forceinline__ void plane_passes(const EM& E, int w, float2* plane, Load load, Store store) {
  using S = Sh<T>;
  float ar[S::NS], ai[S::NS], br[S::NS], bi[S::NS];
  load(w, ar, ai);
#pragma unroll 1
  for (int t = w; t < T; t += 4) {
    if (t + 4 < T) load(t + 4, br, bi);
    typename S::acc dr, di;
    tile_dft<T, true, true, false>(E, ar, ai, dr, di);
    {
      OPAQUE_LANE();
#pragma unroll
      for (int v = 0; v < S::NR; ++v) plane[S::row(v, lane) * (T + 1) + x] = make_float2(dr[v], di[v]);
    }
    {
      OPAQUE_LANE();
#pragma unroll
      for (int s = 0; s < S::NS; ++s) {
        const float2 z = plane[x * (T + 1) + S::KS * s + jl];
        ar[s] = z.x;
        ai[s] = z.y;
      }
    }
    tile_dft<T, false, true, false>(E, ar, ai, dr, di);
    store(t, dr, di);
#pragma unroll
    for (int s = 0; s < S::NS; ++s) {
      ar[s] = br[s];
      ai[s] = bi[s];
    }
  }
}

// Up to k3dGroup transforms at once: plane t of each work field in turn through
// the axis-1 and axis-2 passes (the next field's plane, or the next plane's
// first field, prefetched during the current one), the products Re * Im of
// the group summed in FP64 registers; store(t, g) receives the plane's sum, so
// the FP64 gain is read and written once per group.
template <int T, class EM, class Load, class Store>
__device__ __forceinline__ void plane_passes_group(const EM& E, int w, float2* plane, int g, Load load,
                                                   Store store) {
  using S = Sh<T>;
  float ar[S::NS], ai[S::NS], br[S::NS], bi[S::NS];
  load(0, w, ar, ai);
#pragma unroll 1
  for (int t = w; t < T; t += 4) {
    double acc[S::NR];
#pragma unroll
    for (int v = 0; v < S::NR; ++v) acc[v] = 0.0;
#pragma unroll 1
    for (int f = 0; f < g; ++f) {
      if (f + 1 < g) load(f + 1, t, br, bi);
      else if (t + 4 < T) load(0, t + 4, br, bi);
      typename S::acc dr, di;
      tile_dft<T, true, true, false>(E, ar, ai, dr, di);
      {
        OPAQUE_LANE();
#pragma unroll
        for (int v = 0; v < S::NR; ++v) plane[S::row(v, lane) * (T + 1) + x] = make_float2(dr[v], di[v]);
      }
      {
        OPAQUE_LANE();
#pragma unroll
        for (int s = 0; s < S::NS; ++s) {
          const float2 z = plane[x * (T + 1) + S::KS * s + jl];
          ar[s] = z.x;
          ai[s] = z.y;
        }
      }
      tile_dft<T, false, true, false>(E, ar, ai, dr, di);
#pragma unroll
      for (int v = 0; v < S::NR; ++v) acc[v] += static_cast<double>(dr[v]) * static_cast<double>(di[v]);
#pragma unroll
      for (int s = 0; s < S::NS; ++s) {
        ar[s] = br[s];
        ai[s] = bi[s];
      }
    }
    store(t, acc);
  }
}

template <int T, bool FX>
__device__ void cell_3d(const Slot3& a, int64_t cell, char* scratch, double* red, float2* plane,
                        const half8* etab) {
  using S = Sh<T>;
  constexpr int T2 = T * T, T3 = T * T * T;
  const int w = threadIdx.x >> 6;
  const int n = a.n;
  float2* fh = reinterpret_cast<float2*>(scratch);
  float2* work = fh + T3;
  double* gain = reinterpret_cast<double*>(work + T3);
  float2* work_g = reinterpret_cast<float2*>(gain + T3);  // further work fields of a transform group
  // work field f of a group: f = 0 is `work`, f >= 1 follow the gain
  auto wfield = [&](int f) { return f == 0 ? work : work_g + static_cast<int64_t>(f - 1) * T3; };
  const float* fc = a.f + cell * static_cast<int64_t>(n) * n * n;

  typename EmatOf<T, FX>::type E;
  if constexpr (FX) {
    E.tab = etab;
  } else {
    (void)etab;
    const int lane = threadIdx.x & 63;
    const float* src = a.econst + lane * 3 * S::NS;
#pragma unroll
    for (int s = 0; s < S::NS; ++s) {
      E.c[s] = src[s];
      E.s[s] = src[S::NS + s];
      E.ns[s] = src[2 * S::NS + s];
    }
  }
  // ---- forward pass, axis 2 (real input; data as the left operand); tile t = i0
  double fsum = 0.0;
  pass_tiles<T, false, false, true>(
      E, w,
      [&](int t, float* xr, float* xi) {
        OPAQUE_LANE();
#pragma unroll
        for (int s = 0; s < S::NS; ++s) {
          const int j = S::KS * s + jl;
          xr[s] = load_or_zero(fc, t < n && x < n && j < n, (t * n + x) * n + j);
          xi[s] = 0.0f;
          fsum += static_cast<double>(xr[s]);
        }
      },
      [&](int t, const typename S::acc& dr, const typename S::acc& di) {
        OPAQUE_LANE();
#pragma unroll
        for (int v = 0; v < S::NR; ++v) work[t * T2 + S::row(v, lane) * T + x] = make_float2(dr[v], di[v]);
      });
  __syncthreads();
  // ---- forward pass, axis 1 (tile t = i0, lanes over i2), in place
  auto load_axis1 = [&](int t, float* xr, float* xi) {
    OPAQUE_LANE();
#pragma unroll
    for (int s = 0; s < S::NS; ++s) {
      const float2 z = work[t * T2 + (S::KS * s + jl) * T + x];
      xr[s] = z.x;
      xi[s] = z.y;
    }
  };
  auto store_axis1 = [&](int t, const typename S::acc& dr, const typename S::acc& di) {
    OPAQUE_LANE();
#pragma unroll
    for (int v = 0; v < S::NR; ++v) work[t * T2 + S::row(v, lane) * T + x] = make_float2(dr[v], di[v]);
  };
  pass_tiles<T, true, false, false>(E, w, load_axis1, store_axis1);
  __syncthreads();
  // ---- forward pass, axis 0 (tile t = i1, lanes over i2) -> spectrum
  pass_tiles<T, true, false, false>(
      E, w,
      [&](int t, float* xr, float* xi) {
        OPAQUE_LANE();
#pragma unroll
        for (int s = 0; s < S::NS; ++s) {
          const float2 z = work[(S::KS * s + jl) * T2 + t * T + x];
          xr[s] = z.x;
          xi[s] = z.y;
        }
      },
      [&](int t, const typename S::acc& dr, const typename S::acc& di) {
        OPAQUE_LANE();
#pragma unroll
        for (int v = 0; v < S::NR; ++v) fh[S::row(v, lane) * T2 + t * T + x] = make_float2(dr[v], di[v]);
      });
  __syncthreads();

  double mom[5] = {0, 0, 0, 0, 0};
  // Gain transforms in groups of up to k3dGroup: one axis-0 pass reads the
  // spectrum once for the whole group (one work field per transform), one plane
  // pass reads and writes the FP64 gain once for the group. The loss transform
  // runs alone below.
  int q0 = 0;
  for (; q0 < a.P; q0 += k3dGroup) {
    const int g = a.P - q0 < k3dGroup ? a.P - q0 : k3dGroup;
    const float2* mg = reinterpret_cast<const float2*>(a.filt) + static_cast<int64_t>(q0) * T3;
    {
      // ---- inverse pass, axis 0, every transform of the group (tile t = k1)
      float zr[S::NS], zi[S::NS];
      float2 mb[S::NS];
      auto load_z = [&](int t) {
        OPAQUE_LANE();
#pragma unroll
        for (int s = 0; s < S::NS; ++s) {
          const float2 z = fh[(S::KS * s + jl) * T2 + t * T + x];
          zr[s] = z.x;
          zi[s] = z.y;
        }
      };
      auto load_m = [&](int f, int t) {
        OPAQUE_LANE();
        const float2* m = mg + static_cast<int64_t>(f) * T3;
#pragma unroll
        for (int s = 0; s < S::NS; ++s) mb[s] = m[(S::KS * s + jl) * T2 + t * T + x];
      };
      load_z(w);
      load_m(0, w);
#pragma unroll 1
      for (int t = w; t < T; t += 4) {
#pragma unroll 1
        for (int f = 0; f < g; ++f) {
          float xr[S::NS], xi[S::NS];
#pragma unroll
          for (int s = 0; s < S::NS; ++s) {
            xr[s] = mb[s].x * zr[s] - mb[s].y * zi[s];
            xi[s] = mb[s].x * zi[s] + mb[s].y * zr[s];
          }
          // during this DFT: the next transform's filter tile, or the next tile's
          // spectrum and first filter
          if (f + 1 < g) {
            load_m(f + 1, t);
          } else if (t + 4 < T) {
            load_z(t + 4);
            load_m(0, t + 4);
          }
          typename S::acc dr, di;
          tile_dft<T, true, true, false>(E, xr, xi, dr, di);
          {
            OPAQUE_LANE();
            float2* wf = wfield(f);
#pragma unroll
            for (int v = 0; v < S::NR; ++v) wf[S::row(v, lane) * T2 + t * T + x] = make_float2(dr[v], di[v]);
          }
        }
      }
    }
    __syncthreads();
    // ---- axis-1 and axis-2 passes of each plane, every transform of the group, and the gain
    plane_passes_group<T>(E, w, plane, g,
                          [&](int f, int t, float* xr, float* xi) {
                            OPAQUE_LANE();
                            const float2* wf = wfield(f);
#pragma unroll
                            for (int s = 0; s < S::NS; ++s) {
                              const float2 z = wf[t * T2 + (S::KS * s + jl) * T + x];
                              xr[s] = z.x;
                              xi[s] = z.y;
                            }
                          },
                          [&](int t, const double* acc) {
                            OPAQUE_LANE();
#pragma unroll
                            for (int v = 0; v < S::NR; ++v) {
                              const int o = t * T2 + S::row(v, lane) * T + x;
                              gain[o] = q0 == 0 ? acc[v] : gain[o] + acc[v];
                            }
                          });
    __syncthreads();
  }
  {
    // ---- the loss transform (entry P of the table): inverse pass along axis 0
    // with the filter times the spectrum on load (tile t = k1)
    const float2* mq = reinterpret_cast<const float2*>(a.filt) + static_cast<int64_t>(a.P) * T3;
    pass_tiles<T, true, true, false>(
        E, w,
        [&](int t, float* xr, float* xi) {
          OPAQUE_LANE();
#pragma unroll
          for (int s = 0; s < S::NS; ++s) {
            const int o = (S::KS * s + jl) * T2 + t * T + x;
            const float2 z = fh[o], m = mq[o];
            xr[s] = m.x * z.x - m.y * z.y;
            xi[s] = m.x * z.y + m.y * z.x;
          }
        },
        [&](int t, const typename S::acc& dr, const typename S::acc& di) {
          OPAQUE_LANE();
#pragma unroll
          for (int v = 0; v < S::NR; ++v) work[S::row(v, lane) * T2 + t * T + x] = make_float2(dr[v], di[v]);
        });
    __syncthreads();
    // ---- inverse passes along axis 1 and axis 2 of each plane t = i0 (axis 2
    // with the data as the left operand: lines i1 = x on the lanes, output
    // point (t, row, x)); the real loss field gives Q = gain - f * loss on the
    // grid points, zero elsewhere
    plane_passes<T>(
        E, w, plane, load_axis1,
        [&](int t, const typename S::acc& dr, const typename S::acc& /* imaginary part: unused */) {
          OPAQUE_LANE();
#pragma unroll
          for (int v = 0; v < S::NR; ++v) {
            const int r = S::row(v, lane);
            const int o = t * T2 + r * T + x;
            double Q = 0.0;
            if (t < n && r < n && x < n) {
              const double fv = static_cast<double>(fc[(t * n + r) * n + x]);
              Q = (a.P > 0 ? gain[o] : 0.0) - fv * static_cast<double>(dr[v]);
              const double v0 = -a.L + a.dv * t, v1 = -a.L + a.dv * r, v2 = -a.L + a.dv * x;
              mom[0] += Q;
              mom[1] += v0 * Q;
              mom[2] += v1 * Q;
              mom[3] += v2 * Q;
              mom[4] += (v0 * v0 + v1 * v1 + v2 * v2) * Q;
            }
            gain[o] = Q;
          }
        });
    __syncthreads();
  }

  // ---- epilogue over this thread's points (those it wrote in the last pass)
  OPAQUE_LANE();
  const int64_t base = cell * static_cast<int64_t>(n) * n * n;
  if (a.out_kind == 0) {
    float* Qc = reinterpret_cast<float*>(a.q) + base;
    for (int t = w; t < T; t += 4)
#pragma unroll
      for (int v = 0; v < S::NR; ++v) {
        const int r = S::row(v, lane);
        if (t < n && r < n && x < n) Qc[(t * n + r) * n + x] = static_cast<float>(gain[t * T2 + r * T + x]);
      }
  } else if (a.out_kind == 1) {
    block_sum<5>(mom, red);
    double lam[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      lam[i] = 0.0;
#pragma unroll
      for (int j = 0; j < 5; ++j) lam[i] += a.gram_inv[i * 5 + j] * mom[j];
    }
    double* Qc = reinterpret_cast<double*>(a.q) + base;
    for (int t = w; t < T; t += 4)
#pragma unroll
      for (int v = 0; v < S::NR; ++v) {
        const int r = S::row(v, lane);
        if (t < n && r < n && x < n) {
          const double v0 = -a.L + a.dv * t, v1 = -a.L + a.dv * r, v2 = -a.L + a.dv * x;
          const double corr = lam[0] + lam[1] * v0 + lam[2] * v1 + lam[3] * v2 + lam[4] * (v0 * v0 + v1 * v1 + v2 * v2);
          Qc[(t * n + r) * n + x] = gain[t * T2 + r * T + x] - corr;
        }
      }
  } else if (a.out_kind == 3) {
    // stage l of the penalised IMEX RK step (as finish_cell<3> of the 2D
    // kernels): M from the discrete moments of f^n, nu = rho(f^n); gain holds
    // Q(F_{l-1}) in FP64 and fc the input F_{l-1}
    // opaque stage indices: the tableau coefficients are loaded here, per cell,
    // not hoisted into scalar registers held through the transform loops
    int sch = a.rk_scheme - 1, l = a.rk_stage;
    asm volatile("" : "+s"(sch), "+s"(l));
    const int S = sch == 0 ? 3 : 5;
    const double* At = kRkAt[sch][l - 1];
    const double* Ai = kRkA[sch][l - 1];
    float* fnp = a.rk_fn + base;
    double sm[5] = {0, 0, 0, 0, 0};
    for (int t = w; t < T; t += 4)
#pragma unroll
      for (int v = 0; v < S::NR; ++v) {
        const int r = S::row(v, lane);
        if (t < n && r < n && x < n) {
          const double fv = static_cast<double>(fnp[(t * n + r) * n + x]);
          const double v0 = -a.L + a.dv * t, v1 = -a.L + a.dv * r, v2 = -a.L + a.dv * x;
          sm[0] += fv;
          sm[1] += v0 * fv;
          sm[2] += v1 * fv;
          sm[3] += v2 * fv;
          sm[4] += (v0 * v0 + v1 * v1 + v2 * v2) * fv;
        }
      }
    block_sum<5>(sm, red);
    const double rho = sm[0] * a.dv * a.dv * a.dv;
    const double u0 = sm[1] / sm[0], u1 = sm[2] / sm[0], u2 = sm[3] / sm[0];
    const double Tm = (sm[4] / sm[0] - u0 * u0 - u1 * u1 - u2 * u2) / 3.0;
    const double nu = rho, k = a.dt_eps;
    const double tp = 2.0 * 3.14159265358979323846 * Tm;
    const double cM = rho / (tp * sqrt(tp));
    const double den = 1.0 + Ai[l - 1] * k * nu;
    const double* ec = exp_consts();
    int bad = 0;
    for (int t = w; t < T; t += 4)
#pragma unroll
      for (int v = 0; v < S::NR; ++v) {
        const int r = S::row(v, lane);
        if (!(t < n && r < n && x < n)) continue;
        const int o = (t * n + r) * n + x;
        const double v0 = -a.L + a.dv * t, v1 = -a.L + a.dv * r, v2 = -a.L + a.dv * x;
        const double c2 = (v0 - u0) * (v0 - u0) + (v1 - u1) * (v1 - u1) + (v2 - u2) * (v2 - u2);
        const double M = cM * exp_nonpos(-c2 / (2.0 * Tm), ec);
        const double fn = static_cast<double>(fnp[o]);
        double rhs = fn + Ai[l - 1] * k * nu * M;
        for (int m = 1; m < l; ++m) {
          const double Fm = m == 1 ? fn
                            : (m == l - 1 ? static_cast<double>(fc[o])
                                          : static_cast<double>(a.rk_work[(m - 2) * a.rk_stride + base + o]));
          const double Sm = nu * (M - Fm);
          double acc = Ai[m - 1] * Sm;
          if (At[m - 1] != 0.0) {
            const double Qm = m == l - 1 ? gain[t * T2 + r * T + x]
                                         : static_cast<double>(a.rk_work[(S - 3 + m) * a.rk_stride + base + o]);
            acc += At[m - 1] * (Qm - Sm);
          }
          rhs += k * acc;
        }
        const float Fl = static_cast<float>(rhs / den);
        if (l == S) {
          bad |= !(fabsf(Fl) <= 3.0e38f);
          fnp[o] = Fl;
        } else {
          a.rk_work[(l - 2) * a.rk_stride + base + o] = Fl;
          a.rk_work[(S - 3 + (l - 1)) * a.rk_stride + base + o] = static_cast<float>(gain[t * T2 + r * T + x]);
        }
      }
    if (l == S && a.status) {
      double b[1] = {static_cast<double>(__any(bad) ? 1 : 0)};
      block_sum<1>(b, red);
      if (threadIdx.x == 0) a.status[cell] = b[0] > 0.0 ? 1 : 0;
    }
  } else {
    double rs[1] = {fsum};
    block_sum<1>(rs, red);
    const double rho = rs[0] * a.dv * a.dv * a.dv;
    const double k = a.scheme == 1 ? a.dt_eps / (1.0 + a.dt_eps * rho) : a.dt_eps;
    float* fw = const_cast<float*>(a.f) + base;
    int bad = 0;
    for (int t = w; t < T; t += 4)
#pragma unroll
      for (int v = 0; v < S::NR; ++v) {
        const int r = S::row(v, lane);
        if (t < n && r < n && x < n) {
          const int o = (t * n + r) * n + x;
          const float nv = static_cast<float>(static_cast<double>(fw[o]) + k * gain[t * T2 + r * T + x]);
          bad |= !(fabsf(nv) <= 3.0e38f);
          fw[o] = nv;
        }
      }
    if (a.status) {
      double b[1] = {static_cast<double>(__any(bad) ? 1 : 0)};
      block_sum<1>(b, red);
      if (threadIdx.x == 0) a.status[cell] = b[0] > 0.0 ? 1 : 0;
    }
  }
  __syncthreads();  // scratch and red are reused by the next cell
}

__global__ __launch_bounds__(256) void fp32_3d_kernel(Args3 A) {
  __shared__ double red[32];
  __shared__ float2 plane_lds[4][kPlaneLds];   // one T x T plane per wavefront
  float2* plane = plane_lds[threadIdx.x >> 6];
  char* scratch = A.scratch + static_cast<int64_t>(blockIdx.x) * A.scratch_stride;
  const int64_t total = A.cell_start[A.nslots];
  for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
    int s = 0;
#pragma unroll 1
    while (s + 1 < A.nslots && g >= A.cell_start[s + 1]) ++s;
    const Slot3& a = A.slot[s];
    const int64_t cell = g - A.cell_start[s];
    if (a.T == 32) cell_3d<32, false>(a, cell, scratch, red, plane, nullptr);
    else cell_3d<16, false>(a, cell, scratch, red, plane, nullptr);
  }
}

// FX16 slots (16^3 and 32^3 tiles): the LDS table of DFT-matrix splits is
// reloaded when a workgroup moves to a slot of another plan.
__global__ __launch_bounds__(256) void fx16_3d_kernel(Args3 A) {
  __shared__ double red[32];
  __shared__ float2 plane_lds[4][kPlaneLds];
  __shared__ half8 etab_lds[kEtabHalf8];   // the 32x32 table (the 16x16 one is smaller)
  float2* plane = plane_lds[threadIdx.x >> 6];
  char* scratch = A.scratch + static_cast<int64_t>(blockIdx.x) * A.scratch_stride;
  const int64_t total = A.cell_start[A.nslots];
  const void* loaded = nullptr;
  for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
    int s = 0;
#pragma unroll 1
    while (s + 1 < A.nslots && g >= A.cell_start[s + 1]) ++s;
    const Slot3& a = A.slot[s];
    const int64_t cell = g - A.cell_start[s];
    if (a.etab16 != loaded) {  // the previous cell ended with a workgroup barrier
      const half8* src = static_cast<const half8*>(a.etab16);
      const int len = a.T == 32 ? kEtabHalf8 : kEtab16Half8;
      for (int i = threadIdx.x; i < len; i += blockDim.x) etab_lds[i] = src[i];
      __syncthreads();
      loaded = a.etab16;
    }
    if (a.T == 32) cell_3d<32, true>(a, cell, scratch, red, plane, etab_lds);
    else cell_3d<16, true>(a, cell, scratch, red, plane, etab_lds);
  }
}

}  // namespace

// FP32 and FX16 slots go to their own kernels, one launch each (in that order,
// on the same stream: they share the scratch area).
int launch_3d(const Args3& args, hipStream_t stream) {
  for (int fx = 0; fx < 2; ++fx) {
    Args3 sub;
    sub.scratch = args.scratch;
    sub.scratch_stride = args.scratch_stride;
    sub.blocks = args.blocks;
    for (int i = 0; i < args.nslots; ++i) {
      if ((args.slot[i].fx16 != 0) != (fx != 0)) continue;
      sub.slot[sub.nslots] = args.slot[i];
      sub.cell_start[sub.nslots + 1] =
          sub.cell_start[sub.nslots] + (args.cell_start[i + 1] - args.cell_start[i]);
      ++sub.nslots;
    }
    const int64_t total = sub.cell_start[sub.nslots];
    if (total <= 0) continue;
    const int64_t blocks = total < sub.blocks ? total : sub.blocks;
    if (fx)
      hipLaunchKernelGGL(fx16_3d_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, sub);
    else
      hipLaunchKernelGGL(fp32_3d_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, sub);
    if (hipGetLastError() != hipSuccess) return -3;
  }
  return 0;
}

}  // namespace qcoll
