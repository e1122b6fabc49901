// Classical spectral method (section 3.3): Q_hat_k as the direct double sum over
// l + m = k (modulo N, the collocation reading of the fast method) of
// beta(l, m) f_hat_l f_hat_m with a dense table of kernel modes, O(N^4) per cell
// in 2D. FP64 throughout. One workgroup of 256 threads per group of kCb cells:
// the forward DFT of the group into LDS (two passes of N-point sums), the
// double sum (each thread owns output modes k = t, t + 256, ... for every cell
// of the group; the table row betaT[m][.] is read coalesced, f_hat_m is a
// broadcast and f_hat_{k-m} a gather from LDS), the inverse DFT, and the
// optional FP64 moment projection.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "classical_args.hpp"
#include "kernels_common.hpp"

namespace qcoll {
namespace {

constexpr int kCb = 4;          // cells per workgroup
constexpr int kMaxOut = 3;      // output modes per thread (n <= 768)

// 16-byte aligned, so that a lane's complex value is one 128-bit LDS access
// (two 8-byte halves with a 16-byte lane stride conflict in the LDS banks)
struct alignas(16) cplx {
  double re, im;
};

__global__ __launch_bounds__(256) void classical_kernel(ClassicalArgs a) {
  extern __shared__ double2 sh[];   // 16-byte aligned base
  const int N = a.N, n = N * N;
  cplx* fh = reinterpret_cast<cplx*>(sh);          // [kCb][n]
  cplx* tmp = fh + kCb * n;                         // [kCb][n]
  __shared__ double red[4][4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int64_t c0 = static_cast<int64_t>(blockIdx.x) * kCb; c0 < a.cells;
       c0 += static_cast<int64_t>(gridDim.x) * kCb) {
    const int nc = a.cells - c0 < kCb ? static_cast<int>(a.cells - c0) : kCb;
    // forward DFT along the last axis: tmp[c][j1][k2] = sum_j2 f[c][j1][j2] w^(k2 j2)
    for (int i = t; i < kCb * n; i += blockDim.x) {
      const int c = i / n, r = i - c * n, j1 = r / N, k2 = r - j1 * N;
      cplx s = {0.0, 0.0};
      if (c < nc) {
        const float* fr = a.f + (c0 + c) * n + j1 * N;
        for (int j2 = 0; j2 < N; ++j2) {
          const int e = (k2 * j2) % N;
          const double v = static_cast<double>(fr[j2]);
          s.re += v * a.tw[2 * e];
          s.im += v * a.tw[2 * e + 1];
        }
      }
      tmp[i] = s;
    }
    __syncthreads();
    // along the first axis, normalised: fh[c][k1][k2] = N^-2 sum_j1 tmp[c][j1][k2] w^(k1 j1)
    const double inv_n = 1.0 / n;
    for (int i = t; i < kCb * n; i += blockDim.x) {
      const int c = i / n, r = i - c * n, k1 = r / N, k2 = r - k1 * N;
      cplx s = {0.0, 0.0};
      for (int j1 = 0; j1 < N; ++j1) {
        const int e = (k1 * j1) % N;
        const cplx x = tmp[c * n + j1 * N + k2];
        const double wr = a.tw[2 * e], wi = a.tw[2 * e + 1];
        s.re += x.re * wr - x.im * wi;
        s.im += x.re * wi + x.im * wr;
      }
      fh[i] = {s.re * inv_n, s.im * inv_n};
    }
    __syncthreads();
    // the double sum
    cplx acc[kMaxOut][kCb];
    int k1s[kMaxOut], k2s[kMaxOut];
#pragma unroll
    for (int r = 0; r < kMaxOut; ++r) {
      const int k = t + 256 * r;
      k1s[r] = k / N;
      k2s[r] = k - (k / N) * N;
#pragma unroll
      for (int c = 0; c < kCb; ++c) acc[r][c] = {0.0, 0.0};
    }
    for (int m = 0; m < n; ++m) {
      const int m1 = m / N, m2 = m - m1 * N;
      cplx fm[kCb];
#pragma unroll
      for (int c = 0; c < kCb; ++c) fm[c] = fh[c * n + m];
      const double* brow = a.betaT + static_cast<int64_t>(m) * n;
#pragma unroll
      for (int r = 0; r < kMaxOut; ++r) {
        const int k = t + 256 * r;
        if (k < n) {
          int l1 = k1s[r] - m1, l2 = k2s[r] - m2;
          l1 += l1 < 0 ? N : 0;
          l2 += l2 < 0 ? N : 0;
          const int l = l1 * N + l2;
          const double b = brow[k];
#pragma unroll
          for (int c = 0; c < kCb; ++c) {
            const cplx fl = fh[c * n + l];
            const double pr = fl.re * fm[c].re - fl.im * fm[c].im;
            const double pi = fl.re * fm[c].im + fl.im * fm[c].re;
            acc[r][c].re += b * pr;
            acc[r][c].im += b * pi;
          }
        }
      }
    }
    __syncthreads();  // every thread is done with fh: Q_hat goes into tmp
#pragma unroll
    for (int r = 0; r < kMaxOut; ++r) {
      const int k = t + 256 * r;
      if (k < n)
#pragma unroll
        for (int c = 0; c < kCb; ++c) tmp[c * n + k] = acc[r][c];
    }
    __syncthreads();
    // inverse DFT along the first axis: fh[c][j1][k2] = sum_k1 Qh[c][k1][k2] w^(-k1 j1)
    for (int i = t; i < kCb * n; i += blockDim.x) {
      const int c = i / n, r = i - c * n, j1 = r / N, k2 = r - j1 * N;
      cplx s = {0.0, 0.0};
      for (int k1 = 0; k1 < N; ++k1) {
        const int e = (k1 * j1) % N;
        const cplx x = tmp[c * n + k1 * N + k2];
        const double wr = a.tw[2 * e], wi = -a.tw[2 * e + 1];
        s.re += x.re * wr - x.im * wi;
        s.im += x.re * wi + x.im * wr;
      }
      fh[i] = s;
    }
    __syncthreads();
    // along the last axis (real part), moments for the projection
    double* qv = reinterpret_cast<double*>(tmp);   // [kCb][n] real Q
    for (int i = t; i < kCb * n; i += blockDim.x) {
      const int c = i / n, r = i - c * n, j1 = r / N, j2 = r - j1 * N;
      double s = 0.0;
      for (int k2 = 0; k2 < N; ++k2) {
        const int e = (k2 * j2) % N;
        const cplx x = fh[c * n + j1 * N + k2];
        s += x.re * a.tw[2 * e] + x.im * a.tw[2 * e + 1];   // Re(x conj(w^(k2 j2)))
      }
      qv[i] = s;
    }
    __syncthreads();
    for (int c = 0; c < nc; ++c) {
      const int64_t base = (c0 + c) * n;
      if (!a.conserve) {
        float* Qo = reinterpret_cast<float*>(a.q) + base;
        for (int i = t; i < n; i += blockDim.x) Qo[i] = static_cast<float>(qv[c * n + i]);
        continue;
      }
      double mm[4] = {0, 0, 0, 0};
      for (int i = t; i < n; i += blockDim.x) {
        const int j1 = i / N, j2 = i - j1 * N;
        const double v1 = -a.L + a.dv * j1, v2 = -a.L + a.dv * j2, q = qv[c * n + i];
        mm[0] += q;
        mm[1] += v1 * q;
        mm[2] += v2 * q;
        mm[3] += (v1 * v1 + v2 * v2) * q;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) mm[i] = wave_sum(mm[i]);
      if (lane == 0)
        for (int i = 0; i < 4; ++i) red[w][i] = mm[i];
      __syncthreads();
      double lam[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        lam[i] = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          lam[i] += a.gram_inv[i * 4 + j] * (red[0][j] + red[1][j] + red[2][j] + red[3][j]);
      }
      double* Qo = reinterpret_cast<double*>(a.q) + base;
      for (int i = t; i < n; i += blockDim.x) {
        const int j1 = i / N, j2 = i - j1 * N;
        const double v1 = -a.L + a.dv * j1, v2 = -a.L + a.dv * j2;
        Qo[i] = qv[c * n + i] - (lam[0] + lam[1] * v1 + lam[2] * v2 + lam[3] * (v1 * v1 + v2 * v2));
      }
      __syncthreads();  // red is reused by the next cell
    }
    __syncthreads();    // tmp and fh are reused by the next group
  }
}

}  // namespace

int launch_classical(const ClassicalArgs& args, hipStream_t stream) {
  if (args.cells <= 0) return 0;
  const int n = args.N * args.N;
  if (n > 256 * kMaxOut) return -1;
  const unsigned lds = static_cast<unsigned>(2 * kCb * n * sizeof(double) * 2);
  // up to 2 x kCb x 768 complex doubles = 96 KiB (n <= 768)
  static const bool attr_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(classical_kernel),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  static_cast<int>(2 * kCb * 256 * kMaxOut * sizeof(double) * 2)) ==
                              hipSuccess;
  if (!attr_ok) return -3;
  const int64_t groups = (args.cells + kCb - 1) / kCb;
  const int64_t blocks = groups < 4096 ? groups : 4096;
  hipLaunchKernelGGL(classical_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), lds, stream, args);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qcoll
