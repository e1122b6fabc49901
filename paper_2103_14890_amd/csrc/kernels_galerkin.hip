// Dealiased (Galerkin) variant of Q_h on 2D grids (section 3.3, eqs. (VAR) and
// (ode) without wrap-around): the operator is evaluated on the grid of
// nf = 3n/2 points per axis with the filters restricted to the active modes of
// the n grid, between a trigonometric interpolation of f (n -> nf) and a
// restriction of Q back to the active n-grid modes (nf -> n). Both are
// separable real matrices (applied along each axis, FP64), one workgroup per
// cell, the cell staged in LDS.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "galerkin_args.hpp"
#include "kernels_common.hpp"

namespace qcoll {
namespace {

// f_fine = I f I^T with I = interp [nf][n].
__global__ __launch_bounds__(256) void galerkin_interp_kernel(GalerkinArgs a) {
  extern __shared__ double sh[];
  const int n = a.n, nf = a.nf;
  double* fs = sh;           // [n][n]
  double* t = sh + n * n;    // [nf][n]: t = I f
  for (int64_t cell = blockIdx.x; cell < a.cells; cell += gridDim.x) {
    const float* fc = a.f + cell * static_cast<int64_t>(n) * n;
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) fs[i] = static_cast<double>(fc[i]);
    __syncthreads();
    for (int i = threadIdx.x; i < nf * n; i += blockDim.x) {
      const int r = i / n, c = i - r * n;
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += a.interp[r * n + k] * fs[k * n + c];
      t[i] = s;
    }
    __syncthreads();
    float* ff = a.f_fine + cell * static_cast<int64_t>(nf) * nf;
    for (int i = threadIdx.x; i < nf * nf; i += blockDim.x) {
      const int r = i / nf, c = i - r * nf;
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += t[r * n + k] * a.interp[c * n + k];
      ff[i] = static_cast<float>(s);
    }
    __syncthreads();
  }
}

// Q = R Q_fine R^T with R = restrict_ [n][nf]; then the FP64 projection onto
// the complement of (1, v, |v|^2) on the n grid when conserve is set.
__global__ __launch_bounds__(256) void galerkin_restrict_kernel(GalerkinArgs a) {
  extern __shared__ double sh[];
  __shared__ double red[4][4];
  const int n = a.n, nf = a.nf;
  double* qs = sh;            // [nf][nf]
  double* t = sh + nf * nf;   // [n][nf]: t = R Q_fine, reused as [n][n] for Q
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t cell = blockIdx.x; cell < a.cells; cell += gridDim.x) {
    const double* qc = a.q_fine + cell * static_cast<int64_t>(nf) * nf;
    for (int i = threadIdx.x; i < nf * nf; i += blockDim.x) qs[i] = qc[i];
    __syncthreads();
    for (int i = threadIdx.x; i < n * nf; i += blockDim.x) {
      const int r = i / nf, c = i - r * nf;
      double s = 0.0;
      for (int k = 0; k < nf; ++k) s += a.restrict_[r * nf + k] * qs[k * nf + c];
      t[i] = s;
    }
    __syncthreads();
    // Q[r][c] = sum_k t[r][k] R[c][k]; each thread keeps its points for the projection
    double m[4] = {0, 0, 0, 0};
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
      const int r = i / n, c = i - r * n;
      double s = 0.0;
      for (int k = 0; k < nf; ++k) s += t[r * nf + k] * a.restrict_[c * nf + k];
      qs[i] = s;             // qs is free again: Q on the n grid
      const double v1 = -a.L + a.dv * r, v2 = -a.L + a.dv * c;
      m[0] += s;
      m[1] += v1 * s;
      m[2] += v2 * s;
      m[3] += (v1 * v1 + v2 * v2) * s;
    }
    const int64_t base = cell * static_cast<int64_t>(n) * n;
    if (!a.conserve) {
      __syncthreads();
      float* Qo = reinterpret_cast<float*>(a.q) + base;
      for (int i = threadIdx.x; i < n * n; i += blockDim.x) Qo[i] = static_cast<float>(qs[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) m[i] = wave_sum(m[i]);
      if (lane == 0)
        for (int i = 0; i < 4; ++i) red[w][i] = m[i];
      __syncthreads();
      double mt[4], lam[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) mt[i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        lam[i] = a.gram_inv[i * 4 + 0] * mt[0] + a.gram_inv[i * 4 + 1] * mt[1] + a.gram_inv[i * 4 + 2] * mt[2] +
                 a.gram_inv[i * 4 + 3] * mt[3];
      double* Qo = reinterpret_cast<double*>(a.q) + base;
      for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
        const int r = i / n, c = i - r * n;
        const double v1 = -a.L + a.dv * r, v2 = -a.L + a.dv * c;
        Qo[i] = qs[i] - (lam[0] + lam[1] * v1 + lam[2] * v2 + lam[3] * (v1 * v1 + v2 * v2));
      }
    }
    __syncthreads();  // qs, t and red are reused by the next cell
  }
}

}  // namespace

int launch_galerkin_interp(const GalerkinArgs& args, hipStream_t stream) {
  if (args.cells <= 0) return 0;
  const unsigned lds = static_cast<unsigned>((args.n * args.n + args.nf * args.n) * sizeof(double));
  int64_t blocks = args.cells < 4096 ? args.cells : 4096;
  hipLaunchKernelGGL(galerkin_interp_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), lds, stream, args);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_galerkin_restrict(const GalerkinArgs& args, hipStream_t stream) {
  if (args.cells <= 0) return 0;
  const unsigned lds = static_cast<unsigned>((args.nf * args.nf + args.n * args.nf) * sizeof(double));
  static const bool attr_ok = [] {  // up to 63^2 + 42 x 63 doubles = 53 KB
    return hipFuncSetAttribute(reinterpret_cast<const void*>(galerkin_restrict_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024) == hipSuccess;
  }();
  if (!attr_ok) return -3;
  int64_t blocks = args.cells < 4096 ? args.cells : 4096;
  hipLaunchKernelGGL(galerkin_restrict_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), lds, stream, args);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qcoll
