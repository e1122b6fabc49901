// Fast spectral collision operator, 2D velocity grid N = 16, gfx950.
//
// Same dataflow as the N = 32 kernels (one wavefront per cell, every pass a
// DFT-matrix GEMM with the data as the left MFMA operand, consecutive passes
// chained in registers), on the 16x16 MFMA shapes. A 16x16 result tile holds
// column n = lane % 16 on the lanes and rows 4 g + v (g = lane / 16, register
// v = 0..3) in registers. The left operand of the next pass takes its K = 32
// contraction values as [4 real rows | 4 imaginary rows] per lane, i.e. the
// real and imaginary result tiles concatenated: claimed index 8 g + t is
// (part t / 4, row 4 g + t % 4). The DFT-matrix operands are stored in that
// order, one set per output part:
//   forward  real out [Er; Ei],  imag out [-Ei; Er]   (multiplying by conj(E))
//   inverse  real out [Er; -Ei], imag out [Ei; Er]    (multiplying by E)
// The real-input first forward pass uses the forward set with a zero
// imaginary half in the left operand.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "body_t16.hpp"

namespace qcoll {
namespace {

template <int OUT>
__global__ __launch_bounds__(256) void fx16_t16_kernel(KernelArgs a) {
  const int wpb = blockDim.x >> 6;
  fx16_t16_body<OUT>(a, static_cast<int64_t>(blockIdx.x) * wpb + (threadIdx.x >> 6),
                 static_cast<int64_t>(gridDim.x) * wpb);
}

template <int OUT>
__global__ __launch_bounds__(256) void fp32_t16_kernel(KernelArgs a) {
  const int wpb = blockDim.x >> 6;
  fp32_t16_body<OUT>(a, static_cast<int64_t>(blockIdx.x) * wpb + (threadIdx.x >> 6),
                 static_cast<int64_t>(gridDim.x) * wpb);
}

}  // namespace

int launch_2d16(const KernelArgs& args, hipStream_t stream) {
  if (args.cells <= 0) return 0;
  const int wpb = args.waves_per_block;
  int64_t blocks = (args.cells + wpb - 1) / wpb;
  if (blocks > args.max_blocks) blocks = args.max_blocks;
  dim3 grid(static_cast<unsigned>(blocks)), block(64 * wpb);
  if (args.precision == 4) {
    if (args.out_kind == 0) hipLaunchKernelGGL(fx16_t16_kernel<0>, grid, block, 0, stream, args);
    else if (args.out_kind == 1) hipLaunchKernelGGL(fx16_t16_kernel<1>, grid, block, 0, stream, args);
    else if (args.out_kind == 2) hipLaunchKernelGGL(fx16_t16_kernel<2>, grid, block, 0, stream, args);
    else if (args.out_kind == 3) hipLaunchKernelGGL(fx16_t16_kernel<3>, grid, block, 0, stream, args);
    else hipLaunchKernelGGL(fx16_t16_kernel<4>, grid, block, 0, stream, args);
  } else {
    if (args.out_kind == 0) hipLaunchKernelGGL(fp32_t16_kernel<0>, grid, block, 0, stream, args);
    else if (args.out_kind == 1) hipLaunchKernelGGL(fp32_t16_kernel<1>, grid, block, 0, stream, args);
    else if (args.out_kind == 2) hipLaunchKernelGGL(fp32_t16_kernel<2>, grid, block, 0, stream, args);
    else if (args.out_kind == 3) hipLaunchKernelGGL(fp32_t16_kernel<3>, grid, block, 0, stream, args);
    else hipLaunchKernelGGL(fp32_t16_kernel<4>, grid, block, 0, stream, args);
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qcoll
