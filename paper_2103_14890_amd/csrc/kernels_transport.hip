// Transport on polygonal meshes (section 2.2), two kernels per call:
//  1. reconstruction: for every cell and discrete velocity, the CWENO
//     polynomial of eq. (CWENO:Prec) (optimal polynomial by least squares,
//     one-sided P1 polynomials, central polynomial of eq. (CWENO:P0),
//     nonlinear weights of eq. (eqn.weights)), written out as its average over
//     each face of the cell;
//  2. fluxes: the Rusanov flux of every face (linear in the two face states,
//     so the face integral needs only the face averages) and the update of
//     eq. (finite_vol5).
// One workgroup = 512 (reconstruction: two per thread, both velocities' row
// gathers issued before either is used) or 1024 (fluxes: four per thread)
// consecutive velocities of one cell (four wavefronts); the cell tables are
// wave-uniform and come through scalar loads. Blocks are dealt to the XCDs in contiguous ranges of cells, so that
// neighbouring cells (numbered along a space-filling curve) share an XCD's L2.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "transport_args.hpp"

namespace qcoll {
namespace {

constexpr int kXcds = 8;
constexpr float kEpsW = 1e-14f;   // epsilon of eq. (eqn.weights)
constexpr float kLamCentral = 1e5f;

struct Block {
  int64_t cell;
  int v;       // first velocity of this thread (then v + 256, v + 512, ...)
  bool valid;
};

// Workgroups are dealt to the XCDs round-robin by the hardware; logical block
// b % 8 * (grid / 8) + b / 8 gives each XCD a contiguous range of cells.
template <int VPT>
__device__ inline Block map_block(int64_t ncells, int V) {
  const int chunks = (V + 256 * VPT - 1) / (256 * VPT);
  const int64_t per_xcd = gridDim.x / kXcds;
  const int64_t b = blockIdx.x;
  const int64_t logical = (b % kXcds) * per_xcd + b / kXcds;
  Block r;
  r.cell = logical / chunks;
  r.v = static_cast<int>(logical - r.cell * chunks) * 256 * VPT + static_cast<int>(threadIdx.x);
  r.valid = r.cell < ncells;
  return r;
}

__device__ inline float pow4(float x) {
  const float x2 = x * x;
  return x2 * x2;
}

__device__ inline float min2(float a, float b) { return a < b ? a : b; }

// Element at a 32-bit byte offset from a wave-uniform row base: the address is
// formed as scalar base + 32-bit vector offset.
__device__ inline const float& at(const float* base, unsigned byte_off) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ inline float& at(float* base, unsigned byte_off) {
  return *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + byte_off);
}

// The face count of a cell is a template parameter (the kernels branch once on
// it): every loop below is then fully unrolled and free of branches, so the
// scalar loads of the cell's tables are issued together, not one per face.

// The row values one velocity's reconstruction reads: its own cell, the
// central stencil and the face neighbours.
template <int DEG, int NF>
struct Gath {
  float fi, d[DEG == 2 ? 11 : 5], dn[NF];
};

template <int DEG, int NF>
__device__ __forceinline__ Gath<DEG, NF> recon_load(const float* __restrict__ f, const TrCell* __restrict__ cells,
                                                    int V, const Block& blk) {
  constexpr int NS = DEG == 2 ? 11 : 5;
  const unsigned vb = 4u * static_cast<unsigned>(blk.v < V ? blk.v : V - 1);
  const TrCell& C = cells[blk.cell];
  Gath<DEG, NF> g;
  g.fi = at(f + blk.cell * V, vb);
#pragma unroll
  for (int j = 0; j < NS; ++j) g.d[j] = at(f + static_cast<int64_t>(C.stencil[j]) * V, vb);
#pragma unroll
  for (int L = 0; L < NF; ++L) g.dn[L] = at(f + static_cast<int64_t>(C.nbr[L]) * V, vb);
  return g;
}

// The reconstruction of one velocity from its gathered values, written out as
// face averages.
template <int DEG, int NF>
__device__ __forceinline__ void recon_cell(const Gath<DEG, NF>& g, const TrCell* __restrict__ cells,
                                           float* __restrict__ fv, int V, const Block& blk) {
  constexpr int K = DEG == 2 ? 5 : 2;
  constexpr int NS = DEG == 2 ? 11 : 5;
  const unsigned vb = 4u * static_cast<unsigned>(blk.v < V ? blk.v : V - 1);  // byte offset in a row
  const TrCell& C = cells[blk.cell];
  const float fi = g.fi;
  float d[NS], dn[NF];
#pragma unroll
  for (int j = 0; j < NS; ++j) d[j] = g.d[j];
#pragma unroll
  for (int L = 0; L < NF; ++L) dn[L] = g.dn[L];
  // optimal polynomial (least squares over the central stencil)
  float copt[K];
#pragma unroll
  for (int l = 0; l < K; ++l) copt[l] = 0.0f;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const float e = d[j] - fi;
#pragma unroll
    for (int l = 0; l < K; ++l) copt[l] += C.pinv[l][j] * e;
  }
  // one-sided P1 polynomials
#pragma unroll
  for (int L = 0; L < NF; ++L) dn[L] -= fi;
  float c1[NF], c2[NF], sig[NF];
  float sum1 = 0.0f, sum2 = 0.0f;
#pragma unroll
  for (int L = 0; L < NF; ++L) {
    const float e0 = dn[L], e1 = dn[(L + 1) % NF];
    c1[L] = C.binv[L][0] * e0 + C.binv[L][1] * e1;
    c2[L] = C.binv[L][2] * e0 + C.binv[L][3] * e1;
    sig[L] = c1[L] * c1[L] + c2[L] * c2[L];
    sum1 += c1[L];
    sum2 += c2[L];
  }
  // central polynomial of eq. (CWENO:P0) and its oscillation indicator
  constexpr float lamL = 1.0f / (kLamCentral + NF);
  constexpr float lam0 = kLamCentral * lamL;
  constexpr float inv0 = 1.0f / lam0;
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
  // (reciprocals to 1 ulp: the weights only enter through their ratios)
  float smin = sig0;
#pragma unroll
  for (int L = 0; L < NF; ++L) smin = min2(smin, sig[L]);
  smin += kEpsW;
  const float w0 = lam0 * pow4(smin * __builtin_amdgcn_rcpf(sig0 + kEpsW));
  float wsum = w0;
  float cw[K];
#pragma unroll
  for (int l = 0; l < K; ++l) cw[l] = w0 * c0[l];
#pragma unroll
  for (int L = 0; L < NF; ++L) {
    const float w = lamL * pow4(smin * __builtin_amdgcn_rcpf(sig[L] + kEpsW));
    wsum += w;
    cw[0] += w * c1[L];
    cw[1] += w * c2[L];
  }
  const float inv = 1.0f / wsum;
#pragma unroll
  for (int l = 0; l < K; ++l) cw[l] *= inv;
  // face averages of the reconstruction (all computed before the first store)
  float u[NF];
#pragma unroll
  for (int L = 0; L < NF; ++L) {
    u[L] = fi;
#pragma unroll
    for (int l = 0; l < K; ++l) u[L] += cw[l] * C.phi[L][l];
  }
  if (blk.v < V) {
#pragma unroll
    for (int L = 0; L < NF; ++L) at(fv + static_cast<int64_t>(C.slot0 + L) * V, vb) = u[L];
  }
}

template <int VPT, int NF>
__device__ __forceinline__ void flux_cell(const float* __restrict__ f, const TrFlux* __restrict__ flux,
                                          const float* __restrict__ fv, float* __restrict__ out,
                                          const TransportArgs& a, const Block& blk) {
  const int V = a.V;
  const TrFlux& X = flux[blk.cell];
  unsigned vb[VPT];
  float vx[VPT], vy[VPT], acc[VPT];
#pragma unroll
  for (int r = 0; r < VPT; ++r) {
    const int v = blk.v + 256 * r;
    const int w = v < V ? v : V - 1;
    vb[r] = 4u * static_cast<unsigned>(w);
    vx[r] = static_cast<float>(2 * (w / a.N) - a.N) * a.vh;
    vy[r] = static_cast<float>(2 * (w % a.N) - a.N) * a.vh;
    acc[r] = 0.0f;
  }
#pragma unroll
  for (int L = 0; L < NF; ++L) {
    const float* own = fv + static_cast<int64_t>(X.slot0 + L) * V;
    const float* other = fv + static_cast<int64_t>(X.twin[L]) * V;
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
      const float vn = vx[r] * X.nx[L] + vy[r] * X.ny[L];
      // Rusanov with speed |v.n| is the upwind state
      acc[r] += X.coef[L] * vn * (vn > 0.0f ? at(own, vb[r]) : at(other, vb[r]));
    }
  }
  const float* fc = f + blk.cell * V;
  float* oc = out + blk.cell * V;
#pragma unroll
  for (int r = 0; r < VPT; ++r)
    if (blk.v + 256 * r < V) at(oc, vb[r]) = a.step ? at(fc, vb[r]) - a.dt * acc[r] : -acc[r];
}

#define QCOLL_TR_SWITCH(NFV, CALL) \
  switch (NFV) {                   \
    case 3: CALL(3); break;        \
    case 4: CALL(4); break;        \
    case 5: CALL(5); break;        \
    case 6: CALL(6); break;        \
    case 7: CALL(7); break;        \
    case 8: CALL(8); break;        \
    case 9: CALL(9); break;        \
    case 10: CALL(10); break;      \
    case 11: CALL(11); break;      \
    default: CALL(12); break;      \
  }

template <int DEG>
__global__ __launch_bounds__(256) void transport_recon_kernel(const float* __restrict__ f,
                                                              const TrCell* __restrict__ cells,
                                                              float* __restrict__ fv, int64_t ncells, int V) {
  const Block blk = map_block<2>(ncells, V);
  if (!blk.valid) return;
  Block b2 = blk;
  b2.v += 256;
#define QCOLL_RECON(n)                                          \
  {                                                             \
    const Gath<DEG, n> g1 = recon_load<DEG, n>(f, cells, V, blk); \
    const Gath<DEG, n> g2 = recon_load<DEG, n>(f, cells, V, b2);  \
    recon_cell<DEG, n>(g1, cells, fv, V, blk);                  \
    recon_cell<DEG, n>(g2, cells, fv, V, b2);                   \
  }
  QCOLL_TR_SWITCH(cells[blk.cell].nf, QCOLL_RECON)
#undef QCOLL_RECON
}

template <int VPT>
__global__ __launch_bounds__(256) void transport_flux_kernel(const float* __restrict__ f,
                                                             const TrFlux* __restrict__ flux,
                                                             const float* __restrict__ fv, float* __restrict__ out,
                                                             TransportArgs a) {
  const Block blk = map_block<VPT>(a.ncells, a.V);
  if (!blk.valid) return;
#define QCOLL_FLUX(n) flux_cell<VPT, n>(f, flux, fv, out, a, blk)
  QCOLL_TR_SWITCH(flux[blk.cell].nf, QCOLL_FLUX)
#undef QCOLL_FLUX
}

}  // namespace

int launch_transport(const TransportArgs& args, hipStream_t stream) {
  if (args.ncells <= 0) return 0;
  auto grid_of = [&](int vpt) {
    const int64_t chunks = (args.V + 256 * vpt - 1) / (256 * vpt);
    return (args.ncells * chunks + kXcds - 1) / kXcds * kXcds;
  };
  const int64_t g1 = grid_of(1);
  if (g1 > 0x7fffffff) return -1;
  const int64_t g2 = grid_of(2);
  if (args.degree == 2)
    hipLaunchKernelGGL(transport_recon_kernel<2>, dim3(static_cast<unsigned>(g2)), dim3(256), 0, stream, args.f,
                       args.cells, args.fv, args.ncells, args.V);
  else
    hipLaunchKernelGGL(transport_recon_kernel<1>, dim3(static_cast<unsigned>(g2)), dim3(256), 0, stream, args.f,
                       args.cells, args.fv, args.ncells, args.V);
  if (hipGetLastError() != hipSuccess) return -3;
  if (args.V >= 1024)
    hipLaunchKernelGGL(transport_flux_kernel<4>, dim3(static_cast<unsigned>(grid_of(4))), dim3(256), 0, stream,
                       args.f, args.flux, args.fv, args.out, args);
  else
    hipLaunchKernelGGL(transport_flux_kernel<1>, dim3(static_cast<unsigned>(g1)), dim3(256), 0, stream, args.f,
                       args.flux, args.fv, args.out, args);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace qcoll
