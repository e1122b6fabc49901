// Dealiased (Galerkin) variant of Q_h on 2D grids (section 3.3, eqs. (VAR) and
// (ode) without wrap-around): the operator is evaluated on the grid of
// nf = 3n/2 points per axis with the filters restricted to the active modes of
// the n grid, between a trigonometric interpolation of f (n -> nf) and a
// restriction of Q back to the active n-grid modes (nf -> n). Both are
// separable real matrices (applied along each axis, FP64). A workgroup stages
// the matrix and its transpose in LDS once and then loops over cells, each
// cell staged in LDS: every inner product reads one operand as a broadcast and
// the other at consecutive addresses.

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
  double* I = sh;              // [nf][n]
  double* IT = I + nf * n;     // [n][nf]
  double* fs = IT + n * nf;    // [n][n]
  double* t = fs + n * n;      // [nf][n]: t = I f
  for (int i = threadIdx.x; i < nf * n; i += blockDim.x) {
    const int r = i / n, k = i - r * n;
    I[i] = a.interp[i];
    IT[k * nf + r] = a.interp[i];
  }
  for (int64_t cell = blockIdx.x; cell < a.cells; cell += gridDim.x) {
    __syncthreads();  // tables staged; fs and t free again
    const float* fc = a.f + cell * static_cast<int64_t>(n) * n;
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) fs[i] = static_cast<double>(fc[i]);
    __syncthreads();
    // two neighbouring outputs per thread and step (one 16-byte LDS read of the
    // row operand per pair of FMAs; n and nf are even)
    for (int i = threadIdx.x; i < nf * n / 2; i += blockDim.x) {
      const int r = i / (n / 2), c = 2 * (i - r * (n / 2));
      double s0 = 0.0, s1 = 0.0;
      for (int k = 0; k < n; ++k) {
        const double g = I[r * n + k];
        const double2 b = *reinterpret_cast<const double2*>(&fs[k * n + c]);
        s0 += g * b.x;
        s1 += g * b.y;
      }
      t[r * n + c] = s0;
      t[r * n + c + 1] = s1;
    }
    __syncthreads();
    float* ff = a.f_fine + cell * static_cast<int64_t>(nf) * nf;
    for (int i = threadIdx.x; i < nf * nf / 2; i += blockDim.x) {
      const int r = i / (nf / 2), c = 2 * (i - r * (nf / 2));
      double s0 = 0.0, s1 = 0.0;
      for (int k = 0; k < n; ++k) {
        const double g = t[r * n + k];
        const double2 b = *reinterpret_cast<const double2*>(&IT[k * nf + c]);
        s0 += g * b.x;
        s1 += g * b.y;
      }
      ff[r * nf + c] = static_cast<float>(s0);
      ff[r * nf + c + 1] = static_cast<float>(s1);
    }
  }
}

// Q = R Q_fine R^T with R = restrict_ [n][nf]; then the FP64 projection onto
// the complement of (1, v, |v|^2) on the n grid when conserve is set.
__global__ __launch_bounds__(256) void galerkin_restrict_kernel(GalerkinArgs a) {
  extern __shared__ double sh[];
  __shared__ double red[4][4];
  const int n = a.n, nf = a.nf;
  double* R = sh;              // [n][nf]
  double* RT = R + n * nf;     // [nf][n]
  double* qs = RT + nf * n;    // [nf][nf], reused as [n][n] for Q
  double* t = qs + nf * nf;    // [n][nf]: t = R Q_fine
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < n * nf; i += blockDim.x) {
    const int r = i / nf, k = i - r * nf;
    R[i] = a.restrict_[i];
    RT[k * n + r] = a.restrict_[i];
  }
  for (int64_t cell = blockIdx.x; cell < a.cells; cell += gridDim.x) {
    __syncthreads();  // tables staged; qs, t and red free again
    const double* qc = a.q_fine + cell * static_cast<int64_t>(nf) * nf;
    for (int i = threadIdx.x; i < nf * nf; i += blockDim.x) qs[i] = qc[i];
    __syncthreads();
    // two neighbouring outputs per thread and step, as in the interpolation
    for (int i = threadIdx.x; i < n * nf / 2; i += blockDim.x) {
      const int r = i / (nf / 2), c = 2 * (i - r * (nf / 2));
      double s0 = 0.0, s1 = 0.0;
      for (int k = 0; k < nf; ++k) {
        const double g = R[r * nf + k];
        const double2 b = *reinterpret_cast<const double2*>(&qs[k * nf + c]);
        s0 += g * b.x;
        s1 += g * b.y;
      }
      t[r * nf + c] = s0;
      t[r * nf + c + 1] = s1;
    }
    __syncthreads();
    // Q[r][c] = sum_k t[r][k] R[c][k]; each thread keeps its points for the projection
    double m[4] = {0, 0, 0, 0};
    for (int i = threadIdx.x; i < n * n / 2; i += blockDim.x) {
      const int r = i / (n / 2), c = 2 * (i - r * (n / 2));
      double s0 = 0.0, s1 = 0.0;
      for (int k = 0; k < nf; ++k) {
        const double g = t[r * nf + k];
        const double2 b = *reinterpret_cast<const double2*>(&RT[k * n + c]);
        s0 += g * b.x;
        s1 += g * b.y;
      }
      qs[r * n + c] = s0;    // qs is free again: Q on the n grid
      qs[r * n + c + 1] = s1;
      const double v1 = -a.L + a.dv * r, v2 = -a.L + a.dv * c, v2b = v2 + a.dv;
      m[0] += s0;
      m[1] += v1 * s0;
      m[2] += v2 * s0;
      m[3] += (v1 * v1 + v2 * v2) * s0;
      m[0] += s1;
      m[1] += v1 * s1;
      m[2] += v2b * s1;
      m[3] += (v1 * v1 + v2b * v2b) * s1;
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
  }
}

}  // namespace

// Dynamic LDS: the matrix, its transpose and the cell's two staging fields, at
// most 3 x 60 x 40 + 60^2 doubles (86 KB) for the largest device grid (n = 40).
constexpr int kGalerkinMaxLds = 96 * 1024;

int launch_galerkin_interp(const GalerkinArgs& args, hipStream_t stream) {
  if (args.cells <= 0) return 0;
  const size_t lds = (3 * static_cast<size_t>(args.nf) * args.n + static_cast<size_t>(args.n) * args.n) *
                     sizeof(double);
  if (lds > kGalerkinMaxLds) return -1;
  static const bool attr_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(galerkin_interp_kernel),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  kGalerkinMaxLds) == hipSuccess;
  if (!attr_ok) return -3;
  const int64_t blocks = args.cells < 2048 ? args.cells : 2048;
  hipLaunchKernelGGL(galerkin_interp_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256),
                     static_cast<unsigned>(lds), stream, args);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_galerkin_restrict(const GalerkinArgs& args, hipStream_t stream) {
  if (args.cells <= 0) return 0;
  const size_t lds = (3 * static_cast<size_t>(args.nf) * args.n + static_cast<size_t>(args.nf) * args.nf) *
                     sizeof(double);
  if (lds > kGalerkinMaxLds) return -1;
  static const bool attr_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(galerkin_restrict_kernel),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  kGalerkinMaxLds) == hipSuccess;
  if (!attr_ok) return -3;
  const int64_t blocks = args.cells < 2048 ? args.cells : 2048;
  hipLaunchKernelGGL(galerkin_restrict_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256),
                     static_cast<unsigned>(lds), stream, args);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qcoll
