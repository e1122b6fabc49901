// Batched launch over several plans: cells of different velocity grids (and
// arithmetic variants) in one grid. The operator is cell-local (section 3.3),
// so every cell runs exactly the code of its single-plan launch and the
// results are bitwise equal to separate launches. Workgroups are assigned to
// slots by contiguous ranges; a workgroup finds its slot with a short scan of
// the slot table (at most kMaxSlots entries) and then walks its slot's cells:
// one cell per wavefront on 16x16 and 32x32 tiles, one cell per workgroup of
// four wavefronts on the 64-point grids (the tile-64 body).

#include <hip/hip_runtime.h>

#include <cstdint>

#include "body_t16.hpp"
#include "body_t32.hpp"
#include "body_t64.hpp"

namespace qcoll {
namespace {

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void multi_kernel(MultiArgs m) {
  extern __shared__ double2 lds[];
  const int64_t b = blockIdx.x;
  int s = 0;
#pragma unroll 1
  while (s + 1 < m.nslots && b >= m.block_start[s + 1]) ++s;
  const KernelArgs& a = m.slot[s];
  if (a.tile == 64) {  // one cell (or one part of one, in the split form) per workgroup of four wavefronts
    const int64_t first = b - m.block_start[s], stride = m.block_start[s + 1] - m.block_start[s];
    if (a.split > 1) {
      if (a.precision == 4) t64_body<-1, true, true>(a, first, stride, lds);
      else t64_body<-1, false, true>(a, first, stride, lds);
    } else {
      if (a.precision == 4) t64_body<-1, true>(a, first, stride, lds);
      else t64_body<-1, false>(a, first, stride, lds);
    }
    return;
  }
  if (a.split > 1) {  // 32x32 FX16 tiles, one cell per workgroup of four wavefronts sharing its transforms
    half8* eo = reinterpret_cast<half8*>(lds);
    load_eo_table(a, eo);
    fx16_t32_body<-1, true>(a, b - m.block_start[s], m.block_start[s + 1] - m.block_start[s],
                            lds + (kEoLdsBytes + (threadIdx.x >> 6) * kFhatLdsBytes) / 16, eo);
    return;
  }
  const int wpb = blockDim.x >> 6;
  const int64_t first = (b - m.block_start[s]) * wpb + (threadIdx.x >> 6);
  const int64_t stride = (m.block_start[s + 1] - m.block_start[s]) * wpb;
  if (a.tile == 32) {
    if (a.precision == 4) {  // block-uniform branch: the table load's barrier is safe
      half8* eo = reinterpret_cast<half8*>(lds);
      load_eo_table(a, eo);
      fx16_t32_body<-1>(a, first, stride, lds + (kEoLdsBytes + (threadIdx.x >> 6) * kFhatLdsBytes) / 16, eo);
    }
    else fp32_t32_body<-1>(a, first, stride);
  } else {
    if (a.precision == 4) fx16_t16_body<-1>(a, first, stride);
    else fp32_t16_body<-1>(a, first, stride);
  }
}

}  // namespace

int launch_multi(const MultiArgs& args, int waves_per_block, hipStream_t stream) {
  const int64_t blocks = args.block_start[args.nslots];
  if (blocks <= 0) return 0;
  bool t64 = false;
  for (int i = 0; i < args.nslots; ++i) t64 |= args.slot[i].tile == 64;
  if (t64 && waves_per_block != 4) return -4;   // the tile-64 body needs four wavefronts per workgroup
  // dynamic LDS above the 64 KB default: 76 KB for four wavefronts of N <= 32
  // cells, 79 KB for a tile-64 cell
  constexpr int kMaxLds = kT64LdsBytes > kEoLdsBytes + 4 * kFhatLdsBytes ? kT64LdsBytes
                                                                          : kEoLdsBytes + 4 * kFhatLdsBytes;
  static const bool attr_ok = [] {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(multi_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               kMaxLds) == hipSuccess;
  }();
  if (!attr_ok) return -3;
  const int lds_bytes = t64 ? kMaxLds : kEoLdsBytes + kFhatLdsBytes * waves_per_block;
  hipLaunchKernelGGL(multi_kernel, dim3(static_cast<unsigned>(blocks)), dim3(64 * waves_per_block), lds_bytes, stream,
                     args);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qcoll
