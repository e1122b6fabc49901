// Tables and argument block of the transport kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qcoll {

// Transport on polygonal meshes: one record per cell for each kernel (FP32,
// read with wave-uniform scalar loads straight from the cell index, so no
// load waits on another table load).
constexpr int kTrMaxFaces = 12;
constexpr int kTrMaxStencil = 11;   // central stencil without the cell itself (degree 2)
constexpr int kTrMaxK = 5;          // non-constant Taylor basis functions (degree 2)
struct TrCell {                                 // reconstruction
  int slot0 = 0, nf = 0, pad0 = 0, pad1 = 0;
  int stencil[kTrMaxStencil + 1] = {};          // central stencil cells
  int nbr[kTrMaxFaces] = {};                    // cell across face L
  float pinv[kTrMaxK][kTrMaxStencil + 1] = {};  // least-squares operator of the optimal polynomial
  float S[16] = {};                             // oscillation form, upper triangle row by row
  float binv[kTrMaxFaces][4] = {};              // one-sided stencil (face L, face L+1): 2x2 inverse
  float phi[kTrMaxFaces][kTrMaxK] = {};         // face averages of the Taylor basis functions
  float pad2[12] = {};
};
struct TrFlux {                                 // fluxes
  int slot0 = 0, nf = 0, pad0 = 0, pad1 = 0;
  int twin[kTrMaxFaces] = {};                   // face L in the neighbour's list
  float nx[kTrMaxFaces] = {}, ny[kTrMaxFaces] = {};  // outward unit normals
  float coef[kTrMaxFaces] = {};                 // |face| / |P_i|
};
struct TransportArgs {
  const TrCell* cells = nullptr;
  const TrFlux* flux = nullptr;
  const float* f = nullptr;     // [cells][V]
  float* fv = nullptr;          // [faces][V] face averages of the reconstruction
  float* out = nullptr;         // [cells][V]
  int64_t ncells = 0;
  int V = 0, N = 0;             // velocities, nodes per axis
  float vh = 0;                 // v = (2 j - N) vh per axis (vh = L / N, exact at v = 0)
  int degree = 2;
  int step = 0;                 // 0: out = R, 1: out = f + dt R
  float dt = 0;
};
int launch_transport(const TransportArgs& args, hipStream_t stream);

}  // namespace qcoll
