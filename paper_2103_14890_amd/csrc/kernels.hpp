// Device-side argument block shared by the host launcher and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qcoll {

struct KernelArgs {
  const float* f = nullptr;     // [cells][N^d] (updated in place by the step kernels)
  void* q = nullptr;            // [cells][N^d] float, or double with the projection
  int64_t cells = 0;
  int n = 0;                    // grid points per axis (<= the kernel's tile size N)
  const void* econst = nullptr; // per-lane DFT-matrix operands (layout set by the variant)
  const double* filt = nullptr; // FX16: [P][64 lanes][16 modes][re, im], scaled by 2^-filt_exp
  const int* filt_exp = nullptr;
  const double* loss = nullptr; // FX16: [64 lanes][16 modes], scaled by 2^-loss_exp
  int loss_exp = 0;
  const float* filt32 = nullptr;  // FP32: [P][64][16][re, im]
  const float* loss32 = nullptr;  // FP32: [64][16]
  int P = 0;                    // packed gain transforms
  double gram_inv[16] = {};     // inverse Gram matrix of (1, v1, v2, |v|^2), row-major
  double L = 0, dv = 0;
  double dt_eps = 0;            // dt / eps
  int scheme = 0;
  int32_t* status = nullptr;
  int64_t max_blocks = 1 << 20;
};

// Launch the 2D N = 32 kernel. precision: 1 FP32, 4 FX16. out_kind: 0 eval
// (float Q), 1 eval with projection (double Q), 2 stage update of f.
int launch_2d32(const KernelArgs& args, int precision, int out_kind, hipStream_t stream);
int launch_2d16(const KernelArgs& args, int precision, int out_kind, hipStream_t stream);

}  // namespace qcoll
