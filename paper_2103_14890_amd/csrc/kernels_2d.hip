// Fast spectral collision operator, 2D velocity grid N = 32, gfx950.
//
// One wavefront evaluates one cell; a 256-thread workgroup holds four cells
// and walks the cell range in a grid-stride loop. Between the load of f and
// the store of Q a cell stays on chip: its data tiles in registers and, in the
// FX16 variant, its FP64 spectrum in LDS.
//
// Dataflow per cell (section 3.3): forward 2D DFT of f -> f_hat; for every
// packed filter q the spectrum m_q * f_hat and its inverse 2D DFT, whose real
// and imaginary parts are the two real fields g and h of one or two collision
// directions (their product is the gain contribution); one more inverse DFT
// of l * f_hat gives the loss field; Q = gain - f * loss.
//
// Each 1-D DFT pass is a dense DFT-matrix GEMM on MFMA with the DATA as the
// left operand and the DFT matrix as the right operand. The MFMA result tile
// holds its column index on the lanes and its row index in registers, which
// is exactly the left-operand layout of the next MFMA with rows and columns
// swapped; so consecutive passes chain in registers and the transposition
// between the two axes of the 2D transform costs nothing. The register order
// of the contraction index is the result-tile row order
//   r(v, h) = 8 (v / 4) + 4 h + v % 4   (register v, lane half h),
// and the DFT-matrix operands are stored with their rows in that order.
//
// Two arithmetic variants compute the same operator:
//  * FX16: both GEMM operands are split into a fixed-point leading part on a
//    9-bit grid (|lead| <= 512, so the 64 lead*lead products of a K = 64
//    contraction sum exactly in FP32) plus an FP16 hi/lo remainder. Six MFMA
//    products feed two accumulators (exact lead*lead, and the rest). Spectra,
//    filters and elementwise arithmetic are FP64.
//  * FP32: plain FP32 MFMA (32x32x2) with FP32 spectra and filters.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "body_t32.hpp"

namespace qcoll {
namespace {

// Two wavefronts per SIMD (at most 256 VGPRs each). Dynamic LDS: the table of
// DFT-matrix lo parts, then one spectrum per wavefront.
template <int OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void fx16_t32_kernel(KernelArgs a) {
  extern __shared__ double2 lds[];
  half8* eo = reinterpret_cast<half8*>(lds);
  load_eo_table(a, eo);
  const int wpb = blockDim.x >> 6;
  const int w = threadIdx.x >> 6;
  fx16_t32_body<OUT>(a, static_cast<int64_t>(blockIdx.x) * wpb + w, static_cast<int64_t>(gridDim.x) * wpb,
                     lds + (kEoLdsBytes + w * kFhatLdsBytes) / 16, eo);
}

// Ping-pong variant: eight wavefronts (two per SIMD) in alternating phases.
// The two wavefronts that share a SIMD take opposite roles: each wavefront
// reads its SIMD from the hardware-ID register, and the second of the
// workgroup's wavefronts on a SIMD starts one phase late.
template <int OUT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void fx16_t32_pp_kernel(KernelArgs a) {
  extern __shared__ double2 lds[];
  __shared__ int wave_simd[8];
  half8* eo = reinterpret_cast<half8*>(lds);
  const int w = threadIdx.x >> 6;
  const int simd = (__builtin_amdgcn_s_getreg((31 << 11) | 4) >> 4) & 3;   // HW_ID bits 5:4
  if ((threadIdx.x & 63) == 0) wave_simd[w] = simd;
  load_eo_table(a, eo);   // ends with a workgroup barrier
  int rank = 0;
  for (int j = 0; j < w; ++j) rank += wave_simd[j] == simd ? 1 : 0;
  const int64_t first0 = static_cast<int64_t>(blockIdx.x) * 8;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 8;
  const int64_t kmax = (a.cells - first0 + stride - 1) / stride;   // cells of wavefront 0 (the most)
  fx16_t32_body_pp<OUT>(a, first0 + w, stride, kmax, (rank & 1) != 0, lds + (kEoLdsBytes + w * kFhatLdsBytes) / 16,
                        eo);
}

template <int OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void fp32_t32_kernel(KernelArgs a) {
  const int wpb = blockDim.x >> 6;
  fp32_t32_body<OUT>(a, static_cast<int64_t>(blockIdx.x) * wpb + (threadIdx.x >> 6),
                 static_cast<int64_t>(gridDim.x) * wpb);
}

}  // namespace

int launch_2d32(const KernelArgs& args, hipStream_t stream) {
  if (args.cells <= 0) return 0;
  const int wpb = args.waves_per_block;
  int64_t blocks = (args.cells + wpb - 1) / wpb;
  if (blocks > args.max_blocks) blocks = args.max_blocks;
  dim3 grid(static_cast<unsigned>(blocks)), block(64 * wpb);
  if (args.precision == 4 && wpb == 8) {
    const unsigned lds = kEoLdsBytes + kFhatLdsBytes * 8;
    static const bool attr_ok = [] {
      bool ok = true;
      ok &= hipFuncSetAttribute(reinterpret_cast<const void*>(fx16_t32_pp_kernel<0>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kEoLdsBytes + 8 * kFhatLdsBytes) == hipSuccess;
      ok &= hipFuncSetAttribute(reinterpret_cast<const void*>(fx16_t32_pp_kernel<1>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kEoLdsBytes + 8 * kFhatLdsBytes) == hipSuccess;
      ok &= hipFuncSetAttribute(reinterpret_cast<const void*>(fx16_t32_pp_kernel<2>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kEoLdsBytes + 8 * kFhatLdsBytes) == hipSuccess;
      ok &= hipFuncSetAttribute(reinterpret_cast<const void*>(fx16_t32_pp_kernel<3>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kEoLdsBytes + 8 * kFhatLdsBytes) == hipSuccess;
      ok &= hipFuncSetAttribute(reinterpret_cast<const void*>(fx16_t32_pp_kernel<4>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kEoLdsBytes + 8 * kFhatLdsBytes) == hipSuccess;
      return ok;
    }();
    if (!attr_ok) return -3;
    if (args.out_kind == 0) hipLaunchKernelGGL(fx16_t32_pp_kernel<0>, grid, block, lds, stream, args);
    else if (args.out_kind == 1) hipLaunchKernelGGL(fx16_t32_pp_kernel<1>, grid, block, lds, stream, args);
    else if (args.out_kind == 2) hipLaunchKernelGGL(fx16_t32_pp_kernel<2>, grid, block, lds, stream, args);
    else if (args.out_kind == 3) hipLaunchKernelGGL(fx16_t32_pp_kernel<3>, grid, block, lds, stream, args);
    else hipLaunchKernelGGL(fx16_t32_pp_kernel<4>, grid, block, lds, stream, args);
  } else if (args.precision == 4) {
    const unsigned lds = kEoLdsBytes + kFhatLdsBytes * wpb;
    static const bool attr_ok = [] {  // dynamic LDS above the 64 KB default (4 waves: 70 KB)
      const int mx = kEoLdsBytes + 4 * kFhatLdsBytes;
      bool ok = true;
      ok &= hipFuncSetAttribute(reinterpret_cast<const void*>(fx16_t32_kernel<0>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, mx) == hipSuccess;
      ok &= hipFuncSetAttribute(reinterpret_cast<const void*>(fx16_t32_kernel<1>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, mx) == hipSuccess;
      ok &= hipFuncSetAttribute(reinterpret_cast<const void*>(fx16_t32_kernel<2>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, mx) == hipSuccess;
      ok &= hipFuncSetAttribute(reinterpret_cast<const void*>(fx16_t32_kernel<3>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, mx) == hipSuccess;
      ok &= hipFuncSetAttribute(reinterpret_cast<const void*>(fx16_t32_kernel<4>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, mx) == hipSuccess;
      return ok;
    }();
    if (!attr_ok) return -3;
    if (args.out_kind == 0) hipLaunchKernelGGL(fx16_t32_kernel<0>, grid, block, lds, stream, args);
    else if (args.out_kind == 1) hipLaunchKernelGGL(fx16_t32_kernel<1>, grid, block, lds, stream, args);
    else if (args.out_kind == 2) hipLaunchKernelGGL(fx16_t32_kernel<2>, grid, block, lds, stream, args);
    else if (args.out_kind == 3) hipLaunchKernelGGL(fx16_t32_kernel<3>, grid, block, lds, stream, args);
    else hipLaunchKernelGGL(fx16_t32_kernel<4>, grid, block, lds, stream, args);
  } else {
    if (args.out_kind == 0) hipLaunchKernelGGL(fp32_t32_kernel<0>, grid, block, 0, stream, args);
    else if (args.out_kind == 1) hipLaunchKernelGGL(fp32_t32_kernel<1>, grid, block, 0, stream, args);
    else if (args.out_kind == 2) hipLaunchKernelGGL(fp32_t32_kernel<2>, grid, block, 0, stream, args);
    else if (args.out_kind == 3) hipLaunchKernelGGL(fp32_t32_kernel<3>, grid, block, 0, stream, args);
    else hipLaunchKernelGGL(fp32_t32_kernel<4>, grid, block, 0, stream, args);
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qcoll
