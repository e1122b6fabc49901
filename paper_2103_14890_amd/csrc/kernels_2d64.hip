// Single-plan launches of the 2D kernels for grids of 36..64 points per axis
// (the per-cell body is in body_t64.hpp), gfx950.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "body_t64.hpp"

namespace qcoll {
namespace {

// Two workgroups (cells) per CU: at most 256 registers per lane, which with
// the 79 KB of LDS lets the matrix work of one cell overlap the vector and LDS
// work of the other.
#define T64_BOUNDS __launch_bounds__(256, 2)
// VEC: 16-byte stores of Q (output kinds 0, 1 and 4 into a 16-byte aligned Q)
template <int OUT, bool VEC = false>
__global__ T64_BOUNDS void fx16_t64_kernel(KernelArgs a) {
  extern __shared__ double2 lds_raw[];
  t64_body<OUT, true, false, VEC>(a, blockIdx.x, gridDim.x, lds_raw);
}

template <int OUT, bool VEC = false>
__global__ T64_BOUNDS void fp32_t64_kernel(KernelArgs a) {
  extern __shared__ double2 lds_raw[];
  t64_body<OUT, false, false, VEC>(a, blockIdx.x, gridDim.x, lds_raw);
}

}  // namespace

template <template <int, bool> class K>
static bool set_lds_attr() {
  bool ok = true;
  auto set = [&](const void* fn) {
    ok &= hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kT64LdsBytes) == hipSuccess;
  };
  set(reinterpret_cast<const void*>(K<0, false>::fn));
  set(reinterpret_cast<const void*>(K<1, false>::fn));
  set(reinterpret_cast<const void*>(K<2, false>::fn));
  set(reinterpret_cast<const void*>(K<3, false>::fn));
  set(reinterpret_cast<const void*>(K<4, false>::fn));
  set(reinterpret_cast<const void*>(K<0, true>::fn));
  set(reinterpret_cast<const void*>(K<1, true>::fn));
  set(reinterpret_cast<const void*>(K<4, true>::fn));
  return ok;
}

template <int OUT, bool VEC>
struct Fx16T64 {
  static constexpr auto fn = fx16_t64_kernel<OUT, VEC>;
};

template <int OUT, bool VEC>
struct Fp32T64 {
  static constexpr auto fn = fp32_t64_kernel<OUT, VEC>;
};

template <template <int, bool> class K>
static void launch_t64(const KernelArgs& args, dim3 grid, hipStream_t stream) {
  const dim3 block(256);
  const bool vec = (reinterpret_cast<uintptr_t>(args.q) & 15) == 0;   // (Q outputs only)
  switch (args.out_kind) {
    case 0:
      if (vec) hipLaunchKernelGGL((K<0, true>::fn), grid, block, kT64LdsBytes, stream, args);
      else hipLaunchKernelGGL((K<0, false>::fn), grid, block, kT64LdsBytes, stream, args);
      break;
    case 1:
      if (vec) hipLaunchKernelGGL((K<1, true>::fn), grid, block, kT64LdsBytes, stream, args);
      else hipLaunchKernelGGL((K<1, false>::fn), grid, block, kT64LdsBytes, stream, args);
      break;
    case 2: hipLaunchKernelGGL((K<2, false>::fn), grid, block, kT64LdsBytes, stream, args); break;
    case 3: hipLaunchKernelGGL((K<3, false>::fn), grid, block, kT64LdsBytes, stream, args); break;
    default:
      if (vec) hipLaunchKernelGGL((K<4, true>::fn), grid, block, kT64LdsBytes, stream, args);
      else hipLaunchKernelGGL((K<4, false>::fn), grid, block, kT64LdsBytes, stream, args);
      break;
  }
}

int launch_2d64(const KernelArgs& args, hipStream_t stream) {
  if (args.cells <= 0) return 0;
  if (args.precision != 4 && args.precision != 1) return -4;
  int64_t blocks = args.cells;
  if (blocks > args.max_blocks) blocks = args.max_blocks;
  // 79 KB of dynamic LDS, above the 64 KB default
  static const bool attr_ok = set_lds_attr<Fx16T64>() && set_lds_attr<Fp32T64>();
  if (!attr_ok) return -3;
  const dim3 grid(static_cast<unsigned>(blocks));
  if (args.precision == 4) launch_t64<Fx16T64>(args, grid, stream);
  else launch_t64<Fp32T64>(args, grid, stream);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qcoll
