// Transport on polygonal meshes (section 2.2), two kernels per call:
//  1. reconstruction: for every cell and discrete velocity, the CWENO
//     polynomial of eq. (CWENO:Prec) (optimal polynomial by least squares,
//     one-sided P1 polynomials, central polynomial of eq. (CWENO:P0),
//     nonlinear weights of eq. (eqn.weights)), written out as its average over
//     each face of the cell;
//  2. fluxes: the Rusanov flux of every face (linear in the two face states,
//     so the face integral needs only the face averages) and the update of
//     eq. (finite_vol5).
// One workgroup = 256 consecutive velocities of one cell (four wavefronts); the
// cell and face tables are wave-uniform and come through scalar loads. Blocks
// are dealt to the XCDs in contiguous ranges of cells, so that neighbouring
// cells (numbered along a space-filling curve) share an XCD's L2.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace qcoll {
namespace {

constexpr int kXcds = 8;
constexpr float kEpsW = 1e-14f;   // epsilon of eq. (eqn.weights)
constexpr float kLamCentral = 1e5f;

struct Block {
  int64_t cell;
  int v;
  bool valid;
};

__device__ inline Block map_block(int64_t ncells, int V) {
  const int chunks = (V + 255) / 256;
  const int64_t per_xcd = gridDim.x / kXcds;
  const int64_t b = blockIdx.x;
  const int64_t logical = (b % kXcds) * per_xcd + b / kXcds;
  Block r;
  r.cell = logical / chunks;
  r.v = static_cast<int>(logical - r.cell * chunks) * 256 + static_cast<int>(threadIdx.x);
  r.valid = r.cell < ncells;
  return r;
}

__device__ inline float pow4(float x) {
  const float x2 = x * x;
  return x2 * x2;
}

template <int DEG>
__global__ __launch_bounds__(256) void transport_recon_kernel(TransportArgs a) {
  constexpr int K = DEG == 2 ? 5 : 2;
  constexpr int NS = DEG == 2 ? 11 : 5;
  const Block blk = map_block(a.ncells, a.V);
  if (!blk.valid) return;
  const int V = a.V;
  const int vv = blk.v < V ? blk.v : V - 1;
  const TrCell& C = a.cells[blk.cell];
  const int nf = C.nf;
  const TrFace* F = a.faces + C.slot0;
  const float* f = a.f;
  const float fi = f[blk.cell * V + vv];

  // optimal polynomial (least squares over the central stencil)
  float d[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) d[j] = f[static_cast<int64_t>(C.stencil[j]) * V + vv] - fi;
  float copt[K];
#pragma unroll
  for (int l = 0; l < K; ++l) {
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < NS; ++j) s += C.pinv[l][j] * d[j];
    copt[l] = s;
  }
  // one-sided P1 polynomials
  float dn[kTrMaxFaces];
#pragma unroll
  for (int L = 0; L < kTrMaxFaces; ++L)
    if (L < nf) dn[L] = f[static_cast<int64_t>(F[L].nbr) * V + vv] - fi;
  float c1[kTrMaxFaces], c2[kTrMaxFaces], sig[kTrMaxFaces];
  float sum1 = 0.0f, sum2 = 0.0f;
#pragma unroll
  for (int L = 0; L < kTrMaxFaces; ++L) {
    if (L < nf) {
      const float e0 = dn[L], e1 = (L + 1 == nf) ? dn[0] : dn[(L + 1) % kTrMaxFaces];
      c1[L] = F[L].binv[0] * e0 + F[L].binv[1] * e1;
      c2[L] = F[L].binv[2] * e0 + F[L].binv[3] * e1;
      sig[L] = c1[L] * c1[L] + c2[L] * c2[L];
      sum1 += c1[L];
      sum2 += c2[L];
    }
  }
  // central polynomial of eq. (CWENO:P0) and its oscillation indicator
  const float lamL = 1.0f / (kLamCentral + static_cast<float>(nf));
  const float lam0 = kLamCentral * lamL;
  const float inv0 = 1.0f / lam0;
  float c0[K];
#pragma unroll
  for (int l = 0; l < K; ++l) c0[l] = copt[l] * inv0;
  c0[0] = (copt[0] - lamL * sum1) * inv0;
  c0[1] = (copt[1] - lamL * sum2) * inv0;
  float sig0 = 0.0f;
  {
    int e = 0;
#pragma unroll
    for (int r = 0; r < 5; ++r)
#pragma unroll
      for (int c = r; c < 5; ++c, ++e)
        if (r < K && c < K) sig0 += C.S[e] * c0[r] * c0[c];
  }
  // nonlinear weights lam_s / (sigma_s + eps)^4, normalised; evaluated as
  // lam_s ((sigma_min + eps) / (sigma_s + eps))^4, which has the same ratios
  float smin = sig0;
#pragma unroll
  for (int L = 0; L < kTrMaxFaces; ++L)
    if (L < nf) smin = fminf(smin, sig[L]);
  smin += kEpsW;
  const float w0 = lam0 * pow4(smin / (sig0 + kEpsW));
  float wsum = w0;
  float cw[K];
#pragma unroll
  for (int l = 0; l < K; ++l) cw[l] = w0 * c0[l];
#pragma unroll
  for (int L = 0; L < kTrMaxFaces; ++L) {
    if (L < nf) {
      const float w = lamL * pow4(smin / (sig[L] + kEpsW));
      wsum += w;
      cw[0] += w * c1[L];
      cw[1] += w * c2[L];
    }
  }
  const float inv = 1.0f / wsum;
  // face averages of the reconstruction
  if (blk.v < V) {
#pragma unroll
    for (int L = 0; L < kTrMaxFaces; ++L) {
      if (L < nf) {
        float u = 0.0f;
#pragma unroll
        for (int l = 0; l < K; ++l) u += cw[l] * F[L].phi[l];
        a.fv[static_cast<int64_t>(C.slot0 + L) * V + vv] = fi + u * inv;
      }
    }
  }
}

__global__ __launch_bounds__(256) void transport_flux_kernel(TransportArgs a) {
  const Block blk = map_block(a.ncells, a.V);
  if (!blk.valid) return;
  const int V = a.V;
  const int vv = blk.v < V ? blk.v : V - 1;
  const TrCell& C = a.cells[blk.cell];
  const int nf = C.nf;
  const TrFace* F = a.faces + C.slot0;
  const float vx = static_cast<float>(2 * (vv / a.N) - a.N) * a.vh;
  const float vy = static_cast<float>(2 * (vv % a.N) - a.N) * a.vh;
  float acc = 0.0f;
#pragma unroll
  for (int L = 0; L < kTrMaxFaces; ++L) {
    if (L < nf) {
      const float vn = vx * F[L].nx + vy * F[L].ny;
      // Rusanov with speed |v.n| is the upwind state
      const int64_t row = vn > 0.0f ? static_cast<int64_t>(C.slot0 + L) : static_cast<int64_t>(F[L].twin);
      acc += F[L].coef * vn * a.fv[row * V + vv];
    }
  }
  if (blk.v < V) {
    const int64_t o = blk.cell * V + vv;
    a.out[o] = a.step ? a.f[o] - a.dt * acc : -acc;
  }
}

}  // namespace

int launch_transport(const TransportArgs& args, hipStream_t stream) {
  if (args.ncells <= 0) return 0;
  const int chunks = (args.V + 255) / 256;
  const int64_t blocks = args.ncells * chunks;
  const int64_t grid = (blocks + kXcds - 1) / kXcds * kXcds;
  if (grid > 0x7fffffff) return -1;
  if (args.degree == 2)
    hipLaunchKernelGGL(transport_recon_kernel<2>, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, args);
  else
    hipLaunchKernelGGL(transport_recon_kernel<1>, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, args);
  if (hipGetLastError() != hipSuccess) return -3;
  hipLaunchKernelGGL(transport_flux_kernel, dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, args);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qcoll
