// Argument block of the dealiased (Galerkin) kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qcoll {

// Dealiased (Galerkin) variant, 2D: trigonometric interpolation of f from the
// n grid to the nf grid (interp [nf][n] FP64) and restriction of the fine-grid
// Q back (restrict_ [n][nf]), with the FP64 projection (gram_inv, 4x4) when
// conserve is set (Q stored as double), else Q as float.
struct GalerkinArgs {
  const float* f = nullptr;       // [cells][n][n]
  float* f_fine = nullptr;        // [cells][nf][nf]
  const double* q_fine = nullptr; // [cells][nf][nf]
  void* q = nullptr;              // [cells][n][n] float, or double with the projection
  int64_t cells = 0;
  int n = 0, nf = 0;
  const double* interp = nullptr;     // [nf][n]
  const double* restrict_ = nullptr;  // [n][nf]
  int conserve = 0;
  double gram_inv[16] = {};       // inverse Gram matrix of (1, v1, v2, |v|^2) on the n grid
  double L = 0, dv = 0;
};
int launch_galerkin_interp(const GalerkinArgs& args, hipStream_t stream);
int launch_galerkin_restrict(const GalerkinArgs& args, hipStream_t stream);

}  // namespace qcoll
