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
  const double* filt = nullptr; // FX16 filters scaled by 2^-filt_exp (layout set by the tile family)
  const int* filt_exp = nullptr;
  const double* loss = nullptr; // FX16: [64 lanes][16 modes], scaled by 2^-loss_exp
  int loss_exp = 0;
  const double* tw = nullptr;   // tile-64 kernel: w^(k p), [p in {0,1}][k < 32][re, im]
  const float* filt32 = nullptr;  // FP32: [P][64][16][re, im]
  const float* loss32 = nullptr;  // FP32: [64][16]
  int P = 0;                    // packed gain transforms
  double gram_inv[16] = {};     // inverse Gram matrix of (1, v1, v2, |v|^2), row-major
  double L = 0, dv = 0;
  double dt_eps = 0;            // dt / eps
  int scheme = 0;
  int32_t* status = nullptr;
  int out_kind = 0;             // 0 eval (float Q), 1 eval with projection (double Q), 2 step,
                                // 3 stage of a multi-stage IMEX step, 4 double Q without projection
  // out_kind 3: stage rk_stage (2..S) of scheme rk_scheme (1 ARS(2,2,2), 2
  // BPR(3,4,3)); f holds the stage input F_{l-1}, rk_fn the step's start value
  // f^n (overwritten with the result by the last stage), rk_work the stage
  // slots (F_m, m = 2..S-1, at slot m-2; Q(F_m), m = 1..S-1, at slot S-3+m),
  // rk_stride floats apart. rk_mom: [cells][4] sums over the grid of f^n,
  // v1 f^n, v2 f^n and |v|^2 f^n, written by stage 2 (whose input is f^n) and
  // read by the later stages (2D grids of at most 32 points per axis).
  float* rk_fn = nullptr;
  float* rk_work = nullptr;
  double* rk_mom = nullptr;
  int64_t rk_stride = 0;
  int rk_scheme = 0;
  int rk_stage = 0;
  int tile = 32;                // MFMA tile of the kernel: 16, 32 or 64
  int precision = 4;            // 1 FP32, 4 FX16
  // Transform split (the latency form of batched launches): 1, or the number of
  // workers that share a cell's transforms (32x32 FX16 tiles: 4 wavefronts of
  // one workgroup; tile 64: 2 or 4 workgroups, which leave their partial
  // results in split_ws, [cell][part][wavefront][16][64] doubles, and count
  // their arrivals in split_cnt[cell], zero between launches: the last to
  // arrive adds the parts in a fixed order and runs the epilogue).
  int split = 1;
  double* split_ws = nullptr;
  int* split_cnt = nullptr;
  int waves_per_block = 4;      // launch shape (1, 2 or 4 wavefronts, one cell each)
  int64_t max_blocks = 1 << 20; // grid cap; waves loop over cells beyond it
};

// Batched launch over several plans: slot s owns workgroups
// [block_start[s], block_start[s+1]) of the grid.
constexpr int kMaxSlots = 8;
struct MultiArgs {
  int nslots = 0;
  int64_t block_start[kMaxSlots + 1] = {};
  KernelArgs slot[kMaxSlots];
};

// 3D velocity grids (FP32 MFMA; one workgroup of four wavefronts per cell).
// Slot s of a launch covers the cells [cell_start[s], cell_start[s+1]) of the
// launch's global cell range; every slot has its own plan tables.
struct Slot3 {
  const float* f = nullptr;     // [cells][n^3]
  void* q = nullptr;            // [cells][n^3] float, or double with the projection
  int n = 0;                    // grid points per axis (<= T)
  int T = 32;                   // tile edge: 16 or 32 (zero padding up to T)
  int P = 0;                    // gain transforms; entry P of filt is the loss multiplier
  const float* econst = nullptr;  // FP32: [64 lanes][cos, sin, -sin][T/(64/T) steps]
  int fx16 = 0;                   // 1: FX16 DFT-GEMMs (T = 32) with the table etab16
  const void* etab16 = nullptr;   // FX16: [cos, sin, -sin][K half][lead, hi, lo][64 lanes][8] FP16
  const float* filt = nullptr;    // [P+1][T^3][re, im], modes in FFT order per axis
  double gram_inv[25] = {};     // inverse Gram matrix of (1, v1, v2, v3, |v|^2)
  double L = 0, dv = 0;
  double dt_eps = 0;
  int scheme = 0;
  int32_t* status = nullptr;
  int out_kind = 0;             // 0 eval (float Q), 1 eval with projection (double Q), 2 step,
                                // 3 stage of a multi-stage IMEX step
  // out_kind 3: stage rk_stage (2..S) of scheme rk_scheme (1 ARS(2,2,2), 2
  // BPR(3,4,3)); f holds the stage input F_{l-1}, rk_fn the step's start value
  // f^n (overwritten with the result by the last stage), rk_work the stage
  // slots (F_m, m = 2..S-1, at slot m-2; Q(F_m), m = 1..S-1, at slot S-3+m),
  // rk_stride floats apart.
  float* rk_fn = nullptr;
  float* rk_work = nullptr;
  int64_t rk_stride = 0;
  int rk_scheme = 0;
  int rk_stage = 0;
};
// Gain transforms per group in the 3D kernel, and the scratch a 3D workgroup
// needs on a T^3 tile: the spectrum and k3dGroup work fields (complex FP32)
// and the gain (FP64).
constexpr int k3dGroup = 16;
constexpr int64_t scratch_3d_bytes(int T) { return (8 + 8 * k3dGroup + 8) * static_cast<int64_t>(T) * T * T; }

struct Args3 {
  int nslots = 0;
  int64_t cell_start[kMaxSlots + 1] = {};
  Slot3 slot[kMaxSlots];
  char* scratch = nullptr;      // per workgroup: spectrum, k3dGroup work fields, gain
  int64_t scratch_stride = 0;   // bytes per workgroup (scratch_3d_bytes of the largest T)
  int64_t blocks = 0;           // workgroups (at most the scratch capacity)
};
int launch_3d(const Args3& args, hipStream_t stream);

// Single-plan launches (args.tile selects the 16x16 or 32x32 kernel family).
int launch_2d16(const KernelArgs& args, hipStream_t stream);
int launch_2d32(const KernelArgs& args, hipStream_t stream);
int launch_2d64(const KernelArgs& args, hipStream_t stream);
// One launch over several plans (cells of different grids in one grid).
int launch_multi(const MultiArgs& args, int waves_per_block, hipStream_t stream);

}  // namespace qcoll
