// Argument block of the classical (direct-sum) kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qcoll {

// Classical spectral method (section 3.3, eqs. (CF1)/(ode) summed directly):
// FP64, one workgroup per group of cells. betaT[m][k] = beta((k - m) mod N, m)
// over the full mode grid in FFT order (zero where l or m has a component equal
// to -N/2); tw[j] = exp(-2 pi i j / N).
struct ClassicalArgs {
  const float* f = nullptr;     // [cells][N][N]
  void* q = nullptr;            // [cells][N][N] float, or double with the projection
  int64_t cells = 0;
  int N = 0;
  const double* betaT = nullptr;  // [n][n], n = N^2
  const double* tw = nullptr;     // [N][re, im]
  int conserve = 0;
  double gram_inv[16] = {};
  double L = 0, dv = 0;
};
int launch_classical(const ClassicalArgs& args, hipStream_t stream);

}  // namespace qcoll
