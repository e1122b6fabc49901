// C ABI of libqcoll.so: argument checks, device tables, dispatch.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <utility>
#include <vector>

#include "classical_args.hpp"
#include "galerkin_args.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "qcoll.h"

struct qcoll_plan_s {
  qcoll::HostPlan hp;          // the grid the kernels run on (the fine grid of a Galerkin plan)
  qcoll::HostPlan hp_coarse;   // Galerkin plans: the N grid of f and Q
  bool galerkin = false;
  double* gal_interp = nullptr;    // [Nf][N]
  double* gal_restrict = nullptr;  // [N][Nf]
  bool classical = false;
  std::vector<double> beta;        // classical plans: beta[l][m] (host, FP64)
  double* cl_betaT = nullptr;      // device betaT[m][k] = beta((k - m) mod N, m)
  double* cl_tw = nullptr;         // device exp(-2 pi i j / N)
  int precision = 0;
  unsigned flags = 0;
  int device = -1;
  bool on_device = false;
  // device tables
  void* econst = nullptr;
  double* filt = nullptr;
  int* filt_exp = nullptr;
  double* loss = nullptr;
  int loss_exp = 0;
  float* filt32 = nullptr;
  float* loss32 = nullptr;
  double* tw = nullptr;
  float* filt3 = nullptr;    // 3D: [P+1][T^3] complex FP32
  char* scratch = nullptr;   // 3D: per-workgroup spectrum, work field and gain
  int64_t scratch_stride = 0;
  int64_t scratch_blocks = 0;
  int tile = 32;
  // 2D plans with N <= 16 also hold the tables of the 32x32 tile kernels (zero
  // padded), so that the autotuner can choose the tile family: alt_* is the set
  // of the tile that is not selected, swapped with the fields above by set_tile.
  int alt_tile = 0;
  void* alt_econst = nullptr;
  double* alt_filt = nullptr;
  int* alt_filt_exp = nullptr;
  float* alt_filt32 = nullptr;
  float* alt_loss32 = nullptr;
  int64_t device_bytes = 0;
  int64_t max_blocks = 0;    // grid cap of single-plan launches
  int waves_per_block = 4;   // cells per workgroup
  int cus = 256;
  // transform split (qcoll_plan_set_split) and, for tile-64 plans, the parts'
  // results and arrival counters (grown on demand, split_cap cells)
  int split = 1;
  double* split_ws = nullptr;
  int* split_cnt = nullptr;
  int64_t split_cap = 0;   // cells the buffers hold ...
  int split_alloc = 0;     // ... at this split factor
};

namespace {

constexpr double kPi = 3.14159265358979323846;

// Row order of the contraction index in a 32 x 32 MFMA result tile.
inline int rrow(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// Exponent e with x < 2^e (x > 0).
int exp_above(double x) {
  if (!(x > 0.0)) return 0;
  int e;
  std::frexp(x, &e);
  return e;
}

template <class T>
int upload(const std::vector<T>& host, T** dev, int64_t& bytes) {
  size_t nb = host.size() * sizeof(T);
  if (hipMalloc(reinterpret_cast<void**>(dev), nb) != hipSuccess) return QCOLL_ENOMEM;
  if (hipMemcpy(*dev, host.data(), nb, hipMemcpyHostToDevice) != hipSuccess) return QCOLL_EDEVICE;
  bytes += static_cast<int64_t>(nb);
  return QCOLL_OK;
}

void free_device(qcoll_plan_s* p) {
  hipFree(p->alt_econst);
  hipFree(p->alt_filt);
  hipFree(p->alt_filt_exp);
  hipFree(p->alt_filt32);
  hipFree(p->alt_loss32);
  p->alt_econst = nullptr;
  p->alt_filt = nullptr;
  p->alt_filt_exp = nullptr;
  p->alt_filt32 = p->alt_loss32 = nullptr;
  p->alt_tile = 0;
  hipFree(p->econst);
  hipFree(p->filt);
  hipFree(p->filt_exp);
  hipFree(p->loss);
  hipFree(p->filt32);
  hipFree(p->loss32);
  hipFree(p->tw);
  hipFree(p->filt3);
  hipFree(p->scratch);
  hipFree(p->gal_interp);
  hipFree(p->gal_restrict);
  p->gal_interp = p->gal_restrict = nullptr;
  hipFree(p->split_ws);
  hipFree(p->split_cnt);
  p->split_ws = nullptr;
  p->split_cnt = nullptr;
  p->split_cap = 0;
  p->split_alloc = 0;
  hipFree(p->cl_betaT);
  hipFree(p->cl_tw);
  p->cl_betaT = p->cl_tw = nullptr;
  p->filt3 = nullptr;
  p->scratch = nullptr;
  p->tw = nullptr;
  p->econst = nullptr;
  p->filt = p->loss = nullptr;
  p->filt_exp = nullptr;
  p->filt32 = p->loss32 = nullptr;
}

// Device tables of the 2D N = 32 kernels. Lane l = 32 h + c of a wavefront
// holds, for register v, the mode (k1, k2) = (rrow(v, h), c) of a spectrum and
// the DFT-matrix rows rrow(.., h) of the right-hand operands.
int build_device_2d32(qcoll_plan_s* p) {
  const auto& hp = p->hp;
  const int n = hp.N;  // grid size <= 32; rows and columns >= n of the tile are zero
  const int P = static_cast<int>(hp.packed.size());
  auto emat = [&](int m, int k, int j) -> double {
    if (k >= n || j >= n) return 0.0;
    double ang = 2.0 * kPi * static_cast<double>((k * j) % n) / n;
    return m == 0 ? std::cos(ang) : (m == 1 ? std::sin(ang) : -std::sin(ang));
  };
  auto mode = [&](int r, int c) -> int64_t { return (r < n && c < n) ? static_cast<int64_t>(r) * n + c : -1; };
  if (p->precision == QCOLL_MIX_FX16) {
    // E[k][j] = exp(2 pi i k j / N) scaled by 2^9, split into lead/hi/lo halves:
    // [lane][mat (Er, Ei, -Ei)][K-slice s][part][t], value at row rrow(8s+t, h), column c
    std::vector<_Float16> ec(64 * 3 * 2 * 3 * 8);
    for (int lane = 0; lane < 64; ++lane) {
      int h = lane >> 5, c = lane & 31;
      for (int m = 0; m < 3; ++m)
        for (int s = 0; s < 2; ++s)
          for (int t = 0; t < 8; ++t) {
            double y = 512.0 * emat(m, rrow(8 * s + t, h), c);
            double lead = std::nearbyint(y);
            float r = static_cast<float>(y - lead);
            _Float16 hi = static_cast<_Float16>(r);
            _Float16 lo = static_cast<_Float16>(r - static_cast<float>(hi));
            size_t base = ((((static_cast<size_t>(lane) * 3 + m) * 2 + s) * 3) * 8) + t;
            ec[base + 0 * 8] = static_cast<_Float16>(static_cast<float>(lead));
            ec[base + 1 * 8] = hi;
            ec[base + 2 * 8] = lo;
          }
    }
    _Float16* d = nullptr;
    int rc = upload(ec, &d, p->device_bytes);
    p->econst = d;
    if (rc) return rc;
    // packed gain filters q < P, then the loss multiplier as entry P (imaginary
    // part zero); each entry scaled by 2^-e so that its complex modulus is < 1
    std::vector<double> ft(static_cast<size_t>(P + 1) * 64 * 32);
    std::vector<int> fe(P + 1, 0);
    for (int q = 0; q <= P; ++q) {
      auto val = [&](int64_t k) -> std::complex<double> {
        if (k < 0) return {0.0, 0.0};
        return q < P ? hp.packed[q][k] : std::complex<double>(hp.loss_scaled[k], 0.0);
      };
      double mx = 0.0;
      for (int64_t k = 0; k < static_cast<int64_t>(n) * n; ++k) mx = std::fmax(mx, std::abs(val(k)));
      int e = exp_above(mx);
      fe[q] = e;
      double sc = std::ldexp(1.0, -e);
      // [q][register v][lane][re, im]: one wavefront's load of a register is
      // 1 KB contiguous
      for (int lane = 0; lane < 64; ++lane) {
        int h = lane >> 5, c = lane & 31;
        for (int v = 0; v < 16; ++v) {
          int64_t k = mode(rrow(v, h), c);
          size_t o = ((static_cast<size_t>(q) * 16 + v) * 64 + lane) * 2;
          ft[o] = val(k).real() * sc;
          ft[o + 1] = val(k).imag() * sc;
        }
      }
    }
    if ((rc = upload(ft, &p->filt, p->device_bytes))) return rc;
    if ((rc = upload(fe, &p->filt_exp, p->device_bytes))) return rc;
  } else {
    // FP32 32x32x2 operands: [lane][mat][v] = Mat[rrow(v, h)][c]
    std::vector<float> ec(64 * 48);
    for (int lane = 0; lane < 64; ++lane) {
      int h = lane >> 5, c = lane & 31;
      for (int v = 0; v < 16; ++v) {
        ec[lane * 48 + v] = static_cast<float>(emat(0, rrow(v, h), c));
        ec[lane * 48 + 16 + v] = static_cast<float>(emat(1, rrow(v, h), c));
        ec[lane * 48 + 32 + v] = static_cast<float>(emat(2, rrow(v, h), c));
      }
    }
    float* d = nullptr;
    int rc = upload(ec, &d, p->device_bytes);
    p->econst = d;
    if (rc) return rc;
    std::vector<float> ft(static_cast<size_t>(P) * 64 * 32);
    for (int q = 0; q < P; ++q)
      for (int lane = 0; lane < 64; ++lane)
        for (int v = 0; v < 16; ++v) {
          int64_t k = mode(rrow(v, lane >> 5), lane & 31);
          size_t o = (static_cast<size_t>(q) * 64 + lane) * 32 + 2 * v;
          ft[o] = k < 0 ? 0.0f : static_cast<float>(hp.packed[q][k].real());
          ft[o + 1] = k < 0 ? 0.0f : static_cast<float>(hp.packed[q][k].imag());
        }
    if ((rc = upload(ft, &p->filt32, p->device_bytes))) return rc;
    std::vector<float> lt(64 * 16);
    for (int lane = 0; lane < 64; ++lane)
      for (int v = 0; v < 16; ++v) {
        int64_t k = mode(rrow(v, lane >> 5), lane & 31);
        lt[lane * 16 + v] = k < 0 ? 0.0f : static_cast<float>(hp.loss_scaled[k]);
      }
    if ((rc = upload(lt, &p->loss32, p->device_bytes))) return rc;
  }
  return QCOLL_OK;
}

// Device tables of the 2D N = 16 kernels. Lane l = 16 g + n holds, for
// register v, the mode (k1, k2) = (4 g + v, n). DFT operands per output part
// ([4 real rows | 4 imaginary rows] of the contraction, see kernels_2d16.hip).
int build_device_2d16(qcoll_plan_s* p) {
  const auto& hp = p->hp;
  const int n = hp.N;  // grid size <= 16; rows and columns >= n of the tile are zero
  const int P = static_cast<int>(hp.packed.size());
  auto mode = [&](int r, int c) -> int64_t { return (r < n && c < n) ? static_cast<int64_t>(r) * n + c : -1; };
  // set -> (matrix for the real-part rows, matrix for the imaginary-part rows);
  // 0 Er, 1 Ei, 2 -Ei
  const int sets[4][2] = {{0, 1}, {2, 0}, {0, 2}, {1, 0}};
  auto mat = [&](int m, int k, int j) -> double {
    if (k >= n || j >= n) return 0.0;
    double ang = 2.0 * kPi * static_cast<double>((k * j) % n) / n;
    return m == 0 ? std::cos(ang) : (m == 1 ? std::sin(ang) : -std::sin(ang));
  };
  int rc;
  if (p->precision == QCOLL_MIX_FX16) {
    std::vector<_Float16> ec(64 * 4 * 3 * 8);
    for (int lane = 0; lane < 64; ++lane) {
      int g = lane >> 4, n = lane & 15;
      for (int st = 0; st < 4; ++st)
        for (int t = 0; t < 8; ++t) {
          double y = 512.0 * mat(sets[st][t >> 2], 4 * g + (t & 3), n);
          double lead = std::nearbyint(y);
          float r = static_cast<float>(y - lead);
          _Float16 hi = static_cast<_Float16>(r);
          _Float16 lo = static_cast<_Float16>(r - static_cast<float>(hi));
          size_t base = ((static_cast<size_t>(lane) * 4 + st) * 3) * 8 + t;
          ec[base] = static_cast<_Float16>(static_cast<float>(lead));
          ec[base + 8] = hi;
          ec[base + 16] = lo;
        }
    }
    _Float16* d = nullptr;
    rc = upload(ec, &d, p->device_bytes);
    p->econst = d;
    if (rc) return rc;
    std::vector<double> ft(static_cast<size_t>(P + 1) * 64 * 8);
    std::vector<int> fe(P + 1, 0);
    for (int q = 0; q <= P; ++q) {
      auto val = [&](int64_t k) -> std::complex<double> {
        if (k < 0) return {0.0, 0.0};
        return q < P ? hp.packed[q][k] : std::complex<double>(hp.loss_scaled[k], 0.0);
      };
      double mx = 0.0;
      for (int64_t k = 0; k < static_cast<int64_t>(n) * n; ++k) mx = std::fmax(mx, std::abs(val(k)));
      fe[q] = exp_above(mx);
      double sc = std::ldexp(1.0, -fe[q]);
      for (int lane = 0; lane < 64; ++lane)
        for (int v = 0; v < 4; ++v) {
          int64_t k = mode(4 * (lane >> 4) + v, lane & 15);
          size_t o = (static_cast<size_t>(q) * 64 + lane) * 8 + 2 * v;
          ft[o] = val(k).real() * sc;
          ft[o + 1] = val(k).imag() * sc;
        }
    }
    if ((rc = upload(ft, &p->filt, p->device_bytes))) return rc;
    if ((rc = upload(fe, &p->filt_exp, p->device_bytes))) return rc;
  } else {
    std::vector<float> ec(64 * 32);
    for (int lane = 0; lane < 64; ++lane) {
      int g = lane >> 4, n = lane & 15;
      for (int st = 0; st < 4; ++st)
        for (int part = 0; part < 2; ++part)
          for (int v = 0; v < 4; ++v)
            ec[lane * 32 + st * 8 + part * 4 + v] = static_cast<float>(mat(sets[st][part], 4 * g + v, n));
    }
    float* d = nullptr;
    rc = upload(ec, &d, p->device_bytes);
    p->econst = d;
    if (rc) return rc;
    std::vector<float> ft(static_cast<size_t>(P) * 64 * 8), lt(64 * 4);
    for (int lane = 0; lane < 64; ++lane)
      for (int v = 0; v < 4; ++v) {
        int64_t k = mode(4 * (lane >> 4) + v, lane & 15);
        for (int q = 0; q < P; ++q) {
          size_t o = (static_cast<size_t>(q) * 64 + lane) * 8 + 2 * v;
          ft[o] = k < 0 ? 0.0f : static_cast<float>(hp.packed[q][k].real());
          ft[o + 1] = k < 0 ? 0.0f : static_cast<float>(hp.packed[q][k].imag());
        }
        lt[lane * 4 + v] = k < 0 ? 0.0f : static_cast<float>(hp.loss_scaled[k]);
      }
    if ((rc = upload(ft, &p->filt32, p->device_bytes))) return rc;
    if ((rc = upload(lt, &p->loss32, p->device_bytes))) return rc;
  }
  return QCOLL_OK;
}

// Exchange the selected tile's tables with the alternate set (2D, N <= 16).
void swap_tile_tables(qcoll_plan_s* p) {
  std::swap(p->tile, p->alt_tile);
  std::swap(p->econst, p->alt_econst);
  std::swap(p->filt, p->alt_filt);
  std::swap(p->filt_exp, p->alt_filt_exp);
  std::swap(p->filt32, p->alt_filt32);
  std::swap(p->loss32, p->alt_loss32);
}

int launch(const qcoll::KernelArgs& a, hipStream_t stream) {
  if (a.tile == 64) return qcoll::launch_2d64(a, stream);
  return a.tile == 32 ? qcoll::launch_2d32(a, stream) : qcoll::launch_2d16(a, stream);
}

// Device tables of the tile-64 kernel (grids n = 2 n', n' <= 32): n'-point
// DFT operands in the 32x32-tile order, the filters split into the four mode
// quarters k = k' + n' a (one per wavefront), and the twiddles w^(k p).
int build_device_2d64(qcoll_plan_s* p) {
  const auto& hp = p->hp;
  const int n = hp.N, np = n / 2;
  const int P = static_cast<int>(hp.packed.size());
  // n'-point DFT-matrix value e_m(k, j) (cos, sin, -sin), zero outside n' x n'
  auto emat = [&](int m, int k, int j) -> double {
    if (k >= np || j >= np) return 0.0;
    const double ang = 2.0 * kPi * static_cast<double>((k * j) % np) / np;
    return m == 0 ? std::cos(ang) : (m == 1 ? std::sin(ang) : -std::sin(ang));
  };
  int rc;
  if (p->precision == QCOLL_FP32) {
    // FP32 32x32x2 operands: [lane][mat][v] = E_mat[rrow(v, h)][c]
    std::vector<float> ec(64 * 48);
    for (int lane = 0; lane < 64; ++lane)
      for (int m = 0; m < 3; ++m)
        for (int v = 0; v < 16; ++v)
          ec[lane * 48 + 16 * m + v] = static_cast<float>(emat(m, rrow(v, lane >> 5), lane & 31));
    float* d = nullptr;
    rc = upload(ec, &d, p->device_bytes);
    p->econst = d;
    if (rc) return rc;
  } else {
    // FX16: 2^9 e split into lead/hi/lo, [lane][mat][K-slice s][part][t] at row rrow(8 s + t, h)
    std::vector<_Float16> ec(64 * 3 * 2 * 3 * 8);
    for (int lane = 0; lane < 64; ++lane)
      for (int m = 0; m < 3; ++m)
        for (int s = 0; s < 2; ++s)
          for (int t = 0; t < 8; ++t) {
            const double y = 512.0 * emat(m, rrow(8 * s + t, lane >> 5), lane & 31);
            const double lead = std::nearbyint(y);
            const float r = static_cast<float>(y - lead);
            const _Float16 hi = static_cast<_Float16>(r);
            const _Float16 lo = static_cast<_Float16>(r - static_cast<float>(hi));
            const size_t base = ((((static_cast<size_t>(lane) * 3 + m) * 2 + s) * 3) * 8) + t;
            ec[base] = static_cast<_Float16>(static_cast<float>(lead));
            ec[base + 8] = hi;
            ec[base + 16] = lo;
          }
    _Float16* d = nullptr;
    rc = upload(ec, &d, p->device_bytes);
    p->econst = d;
    if (rc) return rc;
  }
  std::vector<double> ft(static_cast<size_t>(P + 1) * 4 * 64 * 32, 0.0);
  std::vector<int> fe(P + 1, 0);
  for (int q = 0; q <= P; ++q) {
    auto val = [&](int64_t k) -> std::complex<double> {
      return q < P ? hp.packed[q][k] : std::complex<double>(hp.loss_scaled[k], 0.0);
    };
    double mx = 0.0;
    for (int64_t k = 0; k < static_cast<int64_t>(n) * n; ++k) mx = std::fmax(mx, std::abs(val(k)));
    fe[q] = exp_above(mx);
    double sc = std::ldexp(1.0, -fe[q]);
    for (int w = 0; w < 4; ++w)
      for (int lane = 0; lane < 64; ++lane)
        for (int v = 0; v < 16; ++v) {
          int r = rrow(v, lane >> 5), c = lane & 31;
          if (r >= np || c >= np) continue;
          int64_t k = static_cast<int64_t>(r + np * (w >> 1)) * n + (c + np * (w & 1));
          // [q][quarter w][register v][lane][re, im]: 1 KB per wavefront load
          size_t o = (((static_cast<size_t>(q) * 4 + w) * 16 + v) * 64 + lane) * 2;
          ft[o] = val(k).real() * sc;
          ft[o + 1] = val(k).imag() * sc;
        }
  }
  if ((rc = upload(ft, &p->filt, p->device_bytes))) return rc;
  if ((rc = upload(fe, &p->filt_exp, p->device_bytes))) return rc;
  std::vector<double> tw(2 * 32 * 2, 0.0);
  for (int par = 0; par < 2; ++par)
    for (int k = 0; k < 32; ++k) {
      double ang = 2.0 * kPi * static_cast<double>(k * par) / n;
      tw[(par * 32 + k) * 2] = std::cos(ang);
      tw[(par * 32 + k) * 2 + 1] = std::sin(ang);
    }
  return upload(tw, &p->tw, p->device_bytes);
}

// Device tables of the 3D kernel: per-lane DFT-matrix values for the T^3 tile
// (MFMA step s, lane l: x = l % T, j = (64 / T) s + l / T; cos, sin, -sin of
// 2 pi x j / n, zero outside n x n), the packed filters and the loss multiplier
// on the padded mode grid, and the per-workgroup scratch.
int build_device_3d(qcoll_plan_s* p) {
  const auto& hp = p->hp;
  const int n = hp.N, T = p->tile, KS = 64 / T, NS = T / KS;
  const int P = static_cast<int>(hp.packed.size());
  // DFT-matrix value e(x, j) for matrix m (cos, sin, -sin of 2 pi x j / n), zero
  // outside the n x n grid
  auto emat = [&](int m, int x, int j) -> double {
    if (x >= n || j >= n) return 0.0;
    const double ang = 2.0 * kPi * static_cast<double>((x * j) % n) / n;
    return m == 0 ? std::cos(ang) : (m == 1 ? std::sin(ang) : -std::sin(ang));
  };
  int rc;
  if (p->precision == QCOLL_MIX_FX16) {
    // 2^9 e split into an integer lead and the FP16 hi and lo of the remainder,
    // stored at et[base], et[base + 64 * 8], et[base + 2 * 64 * 8]
    auto put = [](std::vector<_Float16>& et, size_t base, double e) {
      const double y = 512.0 * e;
      const double lead = std::nearbyint(y);
      const float r = static_cast<float>(y - lead);
      const _Float16 hi = static_cast<_Float16>(r);
      et[base] = static_cast<_Float16>(static_cast<float>(lead));
      et[base + 64 * 8] = hi;
      et[base + 2 * 64 * 8] = static_cast<_Float16>(r - static_cast<float>(hi));
    };
    std::vector<_Float16> et;
    if (T == 32) {
      // [m][K half i][part][lane][slot]: e_m(x, j), x = lane % 32, j = 2 (8 i + slot) + lane / 32
      et.assign(static_cast<size_t>(3) * 2 * 3 * 64 * 8, static_cast<_Float16>(0.0f));
      for (int m = 0; m < 3; ++m)
        for (int i = 0; i < 2; ++i)
          for (int lane = 0; lane < 64; ++lane)
            for (int sl = 0; sl < 8; ++sl)
              put(et, ((static_cast<size_t>(m) * 2 + i) * 3 * 64 + lane) * 8 + sl,
                  emat(m, lane % 32, 2 * (8 * i + sl) + lane / 32));
    } else {
      // [row r: dr fwd, dr inv, di fwd, di inv][part][lane][slot], x = lane % 16,
      // point 4 (slot % 4) + lane / 16; slots 0-3 multiply the real parts, 4-7
      // the imaginary parts: dr = C xr + S_r xi, di = S_i xr + C xi with
      // S_r = S (forward) or -S (inverse), S_i = -S (forward) or S (inverse)
      const int mats[4][2] = {{0, 1}, {0, 2}, {2, 0}, {1, 0}};   // (matrix of slots 0-3, of slots 4-7)
      et.assign(static_cast<size_t>(4) * 3 * 64 * 8, static_cast<_Float16>(0.0f));
      for (int r = 0; r < 4; ++r)
        for (int lane = 0; lane < 64; ++lane)
          for (int sl = 0; sl < 8; ++sl)
            put(et, (static_cast<size_t>(r) * 3 * 64 + lane) * 8 + sl,
                emat(mats[r][sl / 4], lane % 16, 4 * (sl % 4) + lane / 16));
    }
    _Float16* d = nullptr;
    rc = upload(et, &d, p->device_bytes);
    p->econst = d;
    if (rc) return rc;
  } else {
    std::vector<float> ec(static_cast<size_t>(64) * 3 * NS);
    for (int lane = 0; lane < 64; ++lane) {
      const int x = lane % T, jl = lane / T;
      for (int st = 0; st < NS; ++st)
        for (int m = 0; m < 3; ++m) ec[(lane * 3 + m) * NS + st] = static_cast<float>(emat(m, x, KS * st + jl));
    }
    float* d = nullptr;
    rc = upload(ec, &d, p->device_bytes);
    p->econst = d;
    if (rc) return rc;
  }
  const int64_t T3 = static_cast<int64_t>(T) * T * T;
  std::vector<float> ft(static_cast<size_t>(P + 1) * T3 * 2, 0.0f);
  for (int q = 0; q <= P; ++q)
    for (int k0 = 0; k0 < n; ++k0)
      for (int k1 = 0; k1 < n; ++k1)
        for (int k2 = 0; k2 < n; ++k2) {
          const int64_t k = (static_cast<int64_t>(k0) * n + k1) * n + k2;
          const size_t o = (static_cast<size_t>(q) * T3 + (static_cast<int64_t>(k0) * T + k1) * T + k2) * 2;
          if (q < P) {
            ft[o] = static_cast<float>(hp.packed[q][k].real());
            ft[o + 1] = static_cast<float>(hp.packed[q][k].imag());
          } else {
            ft[o] = static_cast<float>(hp.loss_scaled[k]);
          }
        }
  if ((rc = upload(ft, &p->filt3, p->device_bytes))) return rc;
  // scratch per workgroup: the complex spectrum and one work field per
  // transform of a group (8 T^3 bytes each) and the FP64 gain (8 T^3 bytes);
  // two workgroups per CU for 32^3 tiles
  p->scratch_stride = qcoll::scratch_3d_bytes(T);
  p->scratch_blocks = static_cast<int64_t>(p->cus) * (T == 32 ? 2 : 4);
  const size_t sb = static_cast<size_t>(p->scratch_stride) * p->scratch_blocks;
  if (hipMalloc(reinterpret_cast<void**>(&p->scratch), sb) != hipSuccess) return QCOLL_ENOMEM;
  p->device_bytes += static_cast<int64_t>(sb);
  return QCOLL_OK;
}

qcoll::Slot3 make_slot3(const qcoll_plan_s* p) {
  qcoll::Slot3 a;
  a.n = p->hp.N;
  a.T = p->tile;
  a.P = static_cast<int>(p->hp.packed.size());
  if (p->precision == QCOLL_MIX_FX16) {
    a.fx16 = 1;
    a.etab16 = p->econst;
  } else {
    a.econst = static_cast<const float*>(p->econst);
  }
  a.filt = p->filt3;
  for (int i = 0; i < 25 && i < static_cast<int>(p->hp.gram_inv.size()); ++i) a.gram_inv[i] = p->hp.gram_inv[i];
  a.L = p->hp.L;
  a.dv = 2.0 * p->hp.L / p->hp.N;
  return a;
}

// One 3D launch over the given slots, using the scratch of the plan with the
// largest tile, or the caller's scratch area `ws` of ws_bytes (one workgroup
// per scratch_3d_bytes of it).
int launch3(const qcoll_plan_s* const* plans, const qcoll::Slot3* slots, int nslots, const int64_t* cells,
            hipStream_t stream, char* ws = nullptr, int64_t ws_bytes = 0) {
  qcoll::Args3 A;
  const qcoll_plan_s* big = nullptr;
  int64_t total = 0;
  for (int i = 0; i < nslots; ++i) {
    if (!big || plans[i]->tile > big->tile) big = plans[i];
    A.slot[A.nslots] = slots[i];
    A.cell_start[A.nslots] = total;
    total += cells[i];
    ++A.nslots;
  }
  A.cell_start[A.nslots] = total;
  if (!big || total == 0) return 0;
  A.scratch = big->scratch;
  A.scratch_stride = big->scratch_stride;
  A.blocks = big->scratch_blocks;
  if (ws) {
    A.scratch = ws;
    A.blocks = ws_bytes / big->scratch_stride;
    if (A.blocks < 1) return -1;
  }
  return qcoll::launch_3d(A, stream);
}

qcoll::KernelArgs make_args(const qcoll_plan_s* p) {
  qcoll::KernelArgs a;
  a.econst = p->econst;
  a.filt = p->filt;
  a.filt_exp = p->filt_exp;
  a.loss = p->loss;
  a.loss_exp = p->loss_exp;
  a.filt32 = p->filt32;
  a.loss32 = p->loss32;
  a.P = static_cast<int>(p->hp.packed.size());
  for (int i = 0; i < 16 && i < static_cast<int>(p->hp.gram_inv.size()); ++i) a.gram_inv[i] = p->hp.gram_inv[i];
  a.n = p->hp.N;
  a.L = p->hp.L;
  a.dv = 2.0 * p->hp.L / p->hp.N;
  a.max_blocks = p->max_blocks;
  a.waves_per_block = p->waves_per_block;
  a.tile = p->tile;
  a.tw = p->tw;
  a.precision = p->precision;
  a.split = p->split;
  a.split_ws = p->split_ws;
  a.split_cnt = p->split_cnt;
  return a;
}

// 2D grids up to 32 points per axis run on the 16x16 (N <= 16) or 32x32 tile
// kernels; grids of 34..64 points on the tile-64 kernels (FX16 or FP32).
// Dense kernel-mode table of the classical method: beta[l][m] = B(l, m) - B(m, m)
// with B(l, m) = sum_t W_t alpha_t(l) alpha'_t(m) over the terms of `src` (zero
// wherever l or m is a Nyquist mode, as the filters are). Rows split over host
// threads.
void classical_table(const qcoll::HostPlan& src, std::vector<double>& beta) {
  const int64_t n = static_cast<int64_t>(src.N) * src.N;
  const int T = static_cast<int>(src.W.size());
  beta.assign(n * n, 0.0);
  unsigned nth = std::thread::hardware_concurrency();
  nth = nth < 1 ? 1 : (nth > 16 ? 16 : nth);
  std::vector<std::thread> pool;
  for (unsigned th = 0; th < nth; ++th)
    pool.emplace_back([&, th] {
      std::vector<double> row(n);
      for (int64_t l = th; l < n; l += nth) {
        std::fill(row.begin(), row.end(), 0.0);
        for (int t = 0; t < T; ++t) {
          const double a = src.W[t] * src.alpha[t][l];
          if (a == 0.0) continue;
          const double* ap = src.alphap[t].data();
          for (int64_t m = 0; m < n; ++m) row[m] += a * ap[m];
        }
        // B(m, m) is the loss multiplier; it multiplies f_l for every l, Nyquist
        // modes included (the loss is f times a filtered field)
        for (int64_t m = 0; m < n; ++m) beta[l * n + m] = row[m] - src.loss[m];
      }
    });
  for (auto& th : pool) th.join();
}

bool device_supported(const qcoll::HostPlan& hp, int precision) {
  if (hp.d == 3) return hp.N <= 32 && (precision == QCOLL_FP32 || precision == QCOLL_MIX_FX16);
  if (hp.d != 2) return false;
  return hp.N <= 64;
}

}  // namespace

namespace qcoll {
// Device of a device plan, -1 for a host-only plan (used by the no-allocation
// entry point, which looks up its fixed scratch on that device).
int plan_device(const qcoll_plan_s* p) { return p && p->on_device ? p->device : -1; }
}  // namespace qcoll

extern "C" {

static int plan_create(qcoll_plan_t* out, int d, int n_per_dim, double L, int kernel, double gamma, double b,
                       int M, int K_r, int precision, unsigned flags) {
  if (!out) return QCOLL_EINVAL;
  *out = nullptr;
  if (precision != QCOLL_FP32 && precision != QCOLL_MIX_FX16) return QCOLL_EINVAL;
  if (flags & ~(QCOLL_CONSERVE | QCOLL_R_LITERAL | QCOLL_HOST_ONLY | QCOLL_GALERKIN | QCOLL_CLASSICAL |
                QCOLL_SEPARABLE_MODES))
    return QCOLL_EINVAL;
  if ((flags & QCOLL_SEPARABLE_MODES) && !(flags & QCOLL_CLASSICAL)) return QCOLL_EINVAL;
  if ((flags & QCOLL_CLASSICAL) && (flags & QCOLL_GALERKIN)) return QCOLL_EINVAL;
  qcoll_plan_s* p = new (std::nothrow) qcoll_plan_s;
  if (!p) return QCOLL_ENOMEM;
  p->precision = precision;
  p->flags = flags;
  int rc;
  if (flags & QCOLL_CLASSICAL) {
    p->classical = true;
    rc = qcoll::build_host_plan(p->hp, d, n_per_dim, L, kernel, b, M, K_r, flags, gamma);
    if (!rc && d != 2) rc = QCOLL_EUNSUPPORTED;
    if (!rc && (flags & QCOLL_SEPARABLE_MODES)) {
      classical_table(p->hp, p->beta);
    } else if (!rc) {
      // exact kernel modes: 8 N directions, full-rank radial expansion on 2 N + 16 nodes
      qcoll::HostPlan hx;
      const int nr = 2 * n_per_dim + 16;
      rc = qcoll::build_host_plan(hx, d, n_per_dim, L, kernel, b, 8 * n_per_dim, nr, flags, gamma, nr);
      if (!rc) classical_table(hx, p->beta);
    }
  } else if (flags & QCOLL_GALERKIN) {
    if (n_per_dim % 4) {
      delete p;
      return QCOLL_EINVAL;
    }
    p->galerkin = true;
    rc = qcoll::build_host_plan(p->hp_coarse, d, n_per_dim, L, kernel, b, M, K_r, flags, gamma);
    if (!rc && d != 2) rc = QCOLL_EUNSUPPORTED;
    if (!rc) rc = qcoll::build_host_plan(p->hp, d, 3 * n_per_dim / 2, L, kernel, b, M, K_r, flags, gamma);
    if (!rc) qcoll::restrict_to_coarse_modes(p->hp, n_per_dim);
  } else {
    rc = qcoll::build_host_plan(p->hp, d, n_per_dim, L, kernel, b, M, K_r, flags, gamma);
  }
  if (rc) {
    delete p;
    return rc;
  }
  if (!(flags & QCOLL_HOST_ONLY)) {
    if (p->classical ? (p->hp.N > 24) : !device_supported(p->hp, precision)) {
      delete p;
      return QCOLL_EUNSUPPORTED;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1 || hipGetDevice(&p->device) != hipSuccess) {
      delete p;
      return QCOLL_EDEVICE;
    }
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) cus = prop.multiProcessorCount;
    p->cus = cus;
    p->max_blocks = static_cast<int64_t>(cus) * 8;
    p->tile = p->hp.N > 32 ? 64 : (p->hp.N > 16 ? 32 : 16);
    if (p->classical) {
      const int N = p->hp.N;
      const int64_t n = static_cast<int64_t>(N) * N;
      std::vector<double> bt(n * n), tw(2 * N);
      for (int64_t m = 0; m < n; ++m) {
        const int64_t m1 = m / N, m2 = m % N;
        for (int64_t k = 0; k < n; ++k) {
          const int64_t l = ((k / N - m1 + N) % N) * N + (k % N - m2 + N) % N;
          bt[m * n + k] = p->beta[l * n + m];
        }
      }
      for (int j = 0; j < N; ++j) {
        tw[2 * j] = std::cos(2.0 * kPi * j / N);
        tw[2 * j + 1] = -std::sin(2.0 * kPi * j / N);
      }
      if (!(rc = upload(bt, &p->cl_betaT, p->device_bytes))) rc = upload(tw, &p->cl_tw, p->device_bytes);
    } else if (p->hp.d == 3) {
      rc = build_device_3d(p);
    } else {
      rc = p->tile == 64 ? build_device_2d64(p) : (p->tile == 32 ? build_device_2d32(p) : build_device_2d16(p));
      if (!rc && p->tile == 16) {   // the 32x32 tile family as the alternate set
        swap_tile_tables(p);
        p->tile = 32;
        rc = build_device_2d32(p);
        swap_tile_tables(p);
      }
    }
    if (!rc && p->galerkin) {
      std::vector<double> gi, gr;
      qcoll::galerkin_operators(p->hp_coarse.N, p->hp.N, gi, gr);
      if (!(rc = upload(gi, &p->gal_interp, p->device_bytes))) rc = upload(gr, &p->gal_restrict, p->device_bytes);
    }
    if (rc) {
      free_device(p);
      delete p;
      return rc;
    }
    p->on_device = true;
  }
  *out = p;
  return QCOLL_OK;
}

// Host allocations of the plan builder and the batched calls may throw; no
// exception crosses the C ABI (a failed allocation is QCOLL_ENOMEM).
static int plan_create_nothrow(qcoll_plan_t* out, int d, int n_per_dim, double L, int kernel, double gamma, double b,
                               int M, int K_r, int precision, unsigned flags) {
  try {
    return plan_create(out, d, n_per_dim, L, kernel, gamma, b, M, K_r, precision, flags);
  } catch (const std::bad_alloc&) {
    if (out) *out = nullptr;
    return QCOLL_ENOMEM;
  }
}

int qcoll_plan(qcoll_plan_t* out, int d, int n_per_dim, double L, int kernel, double b, int M,
               int K_r, int precision, unsigned flags) {
  if (kernel == QCOLL_VHS) return QCOLL_EINVAL;   // needs its exponent: qcoll_plan_vhs
  return plan_create_nothrow(out, d, n_per_dim, L, kernel, 1.0, b, M, K_r, precision, flags);
}

int qcoll_plan_vhs(qcoll_plan_t* out, int n_per_dim, double L, double gamma, double b, int M, int K_r,
                   int precision, unsigned flags) {
  if (!(gamma >= -1.0 && gamma <= 1.0)) return QCOLL_EINVAL;
  return plan_create_nothrow(out, 2, n_per_dim, L, QCOLL_VHS, gamma, b, M, K_r, precision, flags);
}

static int multi_launch(const qcoll_plan_t* plans, int nplans, const float* const* f, void* const* Q,
                        const int64_t* cells, bool step, double dt, double eps, int scheme,
                        int32_t* const* status, hipStream_t stream);

static int eval_impl(qcoll_plan_t p, const float* f, void* Q, int64_t cells, char* ws, int64_t ws_bytes,
                     hipStream_t stream) {
  if (!p || cells < 0) return QCOLL_EINVAL;
  if (!p->on_device || p->galerkin) return QCOLL_EUNSUPPORTED;
  if (cells == 0) return QCOLL_OK;
  if (!f || !Q) return QCOLL_EINVAL;
  if (p->classical) {
    qcoll::ClassicalArgs c;
    c.f = f;
    c.q = Q;
    c.cells = cells;
    c.N = p->hp.N;
    c.betaT = p->cl_betaT;
    c.tw = p->cl_tw;
    c.conserve = (p->flags & QCOLL_CONSERVE) ? 1 : 0;
    for (int i = 0; i < 16; ++i) c.gram_inv[i] = p->hp.gram_inv[i];
    c.L = p->hp.L;
    c.dv = 2.0 * p->hp.L / p->hp.N;
    return qcoll::launch_classical(c, stream) ? QCOLL_EDEVICE : QCOLL_OK;
  }
  int64_t n = static_cast<int64_t>(p->hp.N) * p->hp.N * (p->hp.d == 3 ? p->hp.N : 1);
  if (cells > (INT64_MAX / 8) / n) return QCOLL_EINVAL;
  if (p->hp.d == 3) {
    qcoll::Slot3 s3 = make_slot3(p);
    s3.f = f;
    s3.q = Q;
    s3.out_kind = (p->flags & QCOLL_CONSERVE) ? 1 : 0;
    const qcoll_plan_s* pl = p;
    return launch3(&pl, &s3, 1, &cells, stream, ws, ws_bytes) ? QCOLL_EDEVICE : QCOLL_OK;
  }
  if (p->split > 1) {   // the split form runs in the batched kernel
    qcoll_plan_t pl = p;
    return multi_launch(&pl, 1, &f, &Q, &cells, false, 0.0, 0.0, 0, nullptr, stream);
  }
  qcoll::KernelArgs a = make_args(p);
  a.f = f;
  a.q = Q;
  a.cells = cells;
  a.out_kind = (p->flags & QCOLL_CONSERVE) ? 1 : 0;
  return launch(a, stream) ? QCOLL_EDEVICE : QCOLL_OK;
}

int qcoll_eval(qcoll_plan_t p, const float* f, void* Q, int64_t cells, hipStream_t stream) {
  return eval_impl(p, f, Q, cells, nullptr, 0, stream);
}

static int step_impl(qcoll_plan_t p, float* f, int64_t cells, double dt, double eps, int scheme,
                     int32_t* status, char* ws, int64_t ws_bytes, hipStream_t stream) {
  if (!p || cells < 0) return QCOLL_EINVAL;
  if (!(dt > 0.0) || !(eps > 0.0) || !std::isfinite(dt) || !std::isfinite(eps)) return QCOLL_EINVAL;
  if (scheme != QCOLL_EXPLICIT_EULER && scheme != QCOLL_IMEX_EULER_PENALIZED) return QCOLL_EINVAL;
  if (!p->on_device || p->galerkin || p->classical) return QCOLL_EUNSUPPORTED;
  if (cells == 0) return QCOLL_OK;
  if (!f) return QCOLL_EINVAL;
  if (p->hp.d == 3) {
    qcoll::Slot3 s3 = make_slot3(p);
    s3.f = f;
    s3.dt_eps = dt / eps;
    s3.scheme = scheme;
    s3.status = status;
    s3.out_kind = 2;
    const qcoll_plan_s* pl = p;
    return launch3(&pl, &s3, 1, &cells, stream, ws, ws_bytes) ? QCOLL_EDEVICE : QCOLL_OK;
  }
  if (p->split > 1) {   // the split form runs in the batched kernel
    qcoll_plan_t pl = p;
    const float* fc = f;
    return multi_launch(&pl, 1, &fc, nullptr, &cells, true, dt, eps, scheme, &status, stream);
  }
  qcoll::KernelArgs a = make_args(p);
  a.f = f;
  a.cells = cells;
  a.dt_eps = dt / eps;
  a.scheme = scheme;
  a.status = status;
  a.out_kind = 2;
  return launch(a, stream) ? QCOLL_EDEVICE : QCOLL_OK;
}

int qcoll_step(qcoll_plan_t p, float* f, int64_t cells, double dt, double eps, int scheme,
               int32_t* status, hipStream_t stream) {
  return step_impl(p, f, cells, dt, eps, scheme, status, nullptr, 0, stream);
}

int64_t qcoll_scratch_bytes(qcoll_plan_t p) {
  if (!p) return -1;
  return (p->on_device && p->hp.d == 3) ? p->scratch_stride : 0;
}

// A workspace for 3D plans must hold at least one workgroup's scratch and be
// 256-byte aligned (the kernels use 16-byte vector accesses at offsets that are
// multiples of T^3 * 8 from it); 2D plans use none (work may be NULL).
static int check_ws(qcoll_plan_t p, const void* work, int64_t work_bytes) {
  if (!p) return QCOLL_EINVAL;
  if (p->on_device && p->hp.d == 3 &&
      (!work || work_bytes < p->scratch_stride || (reinterpret_cast<uintptr_t>(work) & 255) != 0))
    return QCOLL_EINVAL;
  return QCOLL_OK;
}

int qcoll_eval_ws(qcoll_plan_t p, const float* f, void* Q, int64_t cells, void* work, int64_t work_bytes,
                  hipStream_t stream) {
  if (int rc = check_ws(p, work, work_bytes)) return rc;
  const bool d3 = p->on_device && p->hp.d == 3;
  return eval_impl(p, f, Q, cells, d3 ? static_cast<char*>(work) : nullptr, work_bytes, stream);
}

int qcoll_step_ws(qcoll_plan_t p, float* f, int64_t cells, double dt, double eps, int scheme, int32_t* status,
                  void* work, int64_t work_bytes, hipStream_t stream) {
  if (int rc = check_ws(p, work, work_bytes)) return rc;
  const bool d3 = p->on_device && p->hp.d == 3;
  return step_impl(p, f, cells, dt, eps, scheme, status, d3 ? static_cast<char*>(work) : nullptr, work_bytes,
                   stream);
}

namespace {
int rk_stages(int scheme) { return scheme == QCOLL_IMEX_ARS222 ? 3 : (scheme == QCOLL_IMEX_BPR343 ? 5 : 0); }
}  // namespace

int64_t qcoll_galerkin_work_bytes(qcoll_plan_t p, int64_t cells) {
  if (!p || !p->galerkin || cells < 0) return -1;
  const int64_t nf2 = static_cast<int64_t>(p->hp.N) * p->hp.N;
  return cells * nf2 * static_cast<int64_t>(sizeof(float) + sizeof(double));
}

int qcoll_eval_galerkin(qcoll_plan_t p, const float* f, void* Q, int64_t cells, void* work, int64_t work_bytes,
                        hipStream_t stream) {
  if (!p || cells < 0) return QCOLL_EINVAL;
  if (!p->galerkin || !p->on_device) return QCOLL_EUNSUPPORTED;
  if (cells == 0) return QCOLL_OK;
  if (!f || !Q || !work || work_bytes < qcoll_galerkin_work_bytes(p, cells)) return QCOLL_EINVAL;
  const int n = p->hp_coarse.N, nf = p->hp.N;
  const int64_t nf2 = static_cast<int64_t>(nf) * nf;
  double* q_fine = static_cast<double*>(work);                      // [cells][nf][nf] double
  float* f_fine = reinterpret_cast<float*>(q_fine + cells * nf2);    // [cells][nf][nf] float
  qcoll::GalerkinArgs g;
  g.f = f;
  g.f_fine = f_fine;
  g.q_fine = q_fine;
  g.q = Q;
  g.cells = cells;
  g.n = n;
  g.nf = nf;
  g.interp = p->gal_interp;
  g.restrict_ = p->gal_restrict;
  g.conserve = (p->flags & QCOLL_CONSERVE) ? 1 : 0;
  for (int i = 0; i < 16; ++i) g.gram_inv[i] = p->hp_coarse.gram_inv[i];
  g.L = p->hp_coarse.L;
  g.dv = 2.0 * p->hp_coarse.L / n;
  if (qcoll::launch_galerkin_interp(g, stream)) return QCOLL_EDEVICE;
  qcoll::KernelArgs a = make_args(p);
  a.f = f_fine;
  a.q = q_fine;
  a.cells = cells;
  a.out_kind = 4;
  if (launch(a, stream)) return QCOLL_EDEVICE;
  return qcoll::launch_galerkin_restrict(g, stream) ? QCOLL_EDEVICE : QCOLL_OK;
}

// Work of a multi-stage step: 2S - 3 FP32 stage slots of the batch, then (at
// the next 8-byte boundary of the buffer) four FP64 moments of f^n per cell.
int64_t qcoll_step_rk_work_bytes(qcoll_plan_t p, int scheme, int64_t cells) {
  const int S = rk_stages(scheme);
  if (!p || S == 0 || cells < 0) return -1;
  const int64_t n = static_cast<int64_t>(p->hp.N) * p->hp.N * (p->hp.d == 3 ? p->hp.N : 1);
  return static_cast<int64_t>(2 * S - 3) * cells * n * static_cast<int64_t>(sizeof(float)) + 8 +
         cells * 4 * static_cast<int64_t>(sizeof(double));
}

int qcoll_step_rk(qcoll_plan_t p, float* f, int64_t cells, double dt, double eps, int scheme, float* work,
                  int64_t work_bytes, int32_t* status, hipStream_t stream) {
  if (!p || cells < 0) return QCOLL_EINVAL;
  if (!(dt > 0.0) || !(eps > 0.0) || !std::isfinite(dt) || !std::isfinite(eps)) return QCOLL_EINVAL;
  const int S = rk_stages(scheme);
  if (S == 0) return QCOLL_EINVAL;
  if (!p->on_device || p->galerkin || p->classical) return QCOLL_EUNSUPPORTED;
  if (cells == 0) return QCOLL_OK;
  if (!f || !work || work_bytes < qcoll_step_rk_work_bytes(p, scheme, cells)) return QCOLL_EINVAL;
  const int64_t stride = cells * static_cast<int64_t>(p->hp.N) * p->hp.N * (p->hp.d == 3 ? p->hp.N : 1);
  if (p->hp.d == 3) {
    for (int l = 2; l <= S; ++l) {
      qcoll::Slot3 s3 = make_slot3(p);
      s3.f = l == 2 ? f : work + static_cast<int64_t>(l - 3) * stride;  // stage input F_{l-1}
      s3.dt_eps = dt / eps;
      s3.out_kind = 3;
      s3.rk_fn = f;
      s3.rk_work = work;
      s3.rk_stride = stride;
      s3.rk_scheme = scheme == QCOLL_IMEX_ARS222 ? 1 : 2;
      s3.rk_stage = l;
      s3.status = status;
      const qcoll_plan_s* pl = p;
      if (launch3(&pl, &s3, 1, &cells, stream)) return QCOLL_EDEVICE;
    }
    return QCOLL_OK;
  }
  const uintptr_t mom_at = reinterpret_cast<uintptr_t>(work + static_cast<int64_t>(2 * S - 3) * stride);
  double* mom = reinterpret_cast<double*>((mom_at + 7) & ~static_cast<uintptr_t>(7));
  for (int l = 2; l <= S; ++l) {
    qcoll::KernelArgs a = make_args(p);
    a.f = l == 2 ? f : work + static_cast<int64_t>(l - 3) * stride;  // stage input F_{l-1}
    a.cells = cells;
    a.dt_eps = dt / eps;
    a.out_kind = 3;
    a.rk_fn = f;
    a.rk_work = work;
    a.rk_mom = mom;
    a.rk_stride = stride;
    a.rk_scheme = scheme == QCOLL_IMEX_ARS222 ? 1 : 2;
    a.rk_stage = l;
    a.status = status;
    if (launch(a, stream)) return QCOLL_EDEVICE;
  }
  return QCOLL_OK;
}

// Side streams of a device (default priority, created on first use and kept
// until the process ends) for the independent launches of one batched call.
constexpr int kSideStreams = 3;
constexpr int kMaxDevices = 64;

static hipStream_t side_stream(int dev, int k) {
  static std::mutex mu;
  static hipStream_t pool[kMaxDevices][kSideStreams] = {};
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!pool[dev][k]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess) pool[dev][k] = s;
    if (cur != dev) hipSetDevice(cur);
  }
  return pool[dev][k];
}

// Fork/join events of a device (created on first use, kept until the process
// ends) and the lock that serialises their use: [0] marks the caller's stream
// at the fork, [1 + k] side stream k at the join.
struct ForkJoin {
  std::mutex mu;
  hipEvent_t ev[1 + kSideStreams] = {};
};

static ForkJoin* fork_join(int dev) {
  static ForkJoin pool[kMaxDevices];
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  return &pool[dev];
}

// One launch of a batched 2D call: a slot table of up to kMaxSlots plans (N <= 32
// tiles, a wavefront per cell; tile-64 plans, a workgroup per cell).
struct MultiJob {
  qcoll::MultiArgs m;
};

// Run the launches of a batched call (more than one only when the call holds
// more plans than a slot table). They write disjoint outputs, so when there are
// several and the batch is small (`concurrent`: too few cells to fill the GPU
// with one launch at a time, as in a serving tick) they run concurrently: the
// first on the caller's stream, the others on side streams that wait for the
// caller's stream and are waited for by it (so the call is still ordered on the
// caller's stream as a whole). Large batches run one launch after another, and
// so does a call while the stream is being captured into a graph.
static int run_jobs(const std::vector<MultiJob>& jobs, int wpb, int dev, bool concurrent, hipStream_t stream) {
  auto run = [&](const MultiJob& j, hipStream_t s) {
    return qcoll::launch_multi(j.m, wpb, s);
  };
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const bool fork = concurrent && jobs.size() > 1 && hipStreamIsCapturing(stream, &cs) == hipSuccess &&
                    cs == hipStreamCaptureStatusNone;
  hipStream_t side[kSideStreams] = {};
  int nside = 0;
  if (fork) {
    for (; nside < kSideStreams && nside + 1 < static_cast<int>(jobs.size()); ++nside) {
      side[nside] = side_stream(dev, nside);
      if (!side[nside]) break;
    }
  }
  ForkJoin* fj = nside > 0 ? fork_join(dev) : nullptr;
  std::unique_lock<std::mutex> lock;
  if (fj) {
    lock = std::unique_lock<std::mutex>(fj->mu);
    int cur = -1;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    if (have_cur && cur != dev) hipSetDevice(dev);   // events belong to the plans' device
    for (int k = 0; k <= nside && fj; ++k)
      if (!fj->ev[k] && hipEventCreateWithFlags(&fj->ev[k], hipEventDisableTiming) != hipSuccess) {
        fj->ev[k] = nullptr;
        fj = nullptr;   // no events: run the jobs one after another
      }
    if (have_cur && cur != dev) hipSetDevice(cur);
  }
  if (!fj) {
    for (const MultiJob& j : jobs)
      if (run(j, stream)) return QCOLL_EDEVICE;
    return QCOLL_OK;
  }
  // a wait takes the event's most recent record at the time of the call, so
  // the events can be recorded again by the next call once its waits are queued
  int rc = hipEventRecord(fj->ev[0], stream) == hipSuccess ? QCOLL_OK : QCOLL_EDEVICE;
  for (int k = 0; k < nside && rc == QCOLL_OK; ++k)
    if (hipStreamWaitEvent(side[k], fj->ev[0], 0) != hipSuccess) rc = QCOLL_EDEVICE;
  // job 0 and every (nside + 1)-th job after it on the caller's stream, the others round-robin
  for (size_t i = 0; i < jobs.size() && rc == QCOLL_OK; ++i) {
    const int lane = static_cast<int>(i % (nside + 1));
    if (run(jobs[i], lane == 0 ? stream : side[lane - 1])) rc = QCOLL_EDEVICE;
  }
  for (int k = 0; k < nside; ++k)  // join (also after an error, so no side work is left unordered)
    if (hipEventRecord(fj->ev[1 + k], side[k]) != hipSuccess || hipStreamWaitEvent(stream, fj->ev[1 + k], 0) != hipSuccess)
      rc = QCOLL_EDEVICE;
  return rc;
}

// Room in a tile-64 plan's split buffers for `cells` cells (grown on demand: the
// parts' results and the arrival counters, zeroed here; the kernels leave them
// zero). Growing waits for the stream (the old buffers may be in use) and is
// refused while the stream is being captured into a graph.
static int ensure_split_ws(qcoll_plan_s* p, int64_t cells, hipStream_t stream) {
  if (p->split <= 1 || p->tile != 64 || (cells <= p->split_cap && p->split <= p->split_alloc)) return QCOLL_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return QCOLL_EDEVICE;
  if (cs != hipStreamCaptureStatusNone) return QCOLL_EINVAL;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return QCOLL_EDEVICE;
  if (cur != p->device && hipSetDevice(p->device) != hipSuccess) return QCOLL_EDEVICE;
  int rc = QCOLL_OK;
  if (hipStreamSynchronize(stream) != hipSuccess) rc = QCOLL_EDEVICE;
  if (rc == QCOLL_OK) {
    hipFree(p->split_ws);
    hipFree(p->split_cnt);
    p->split_ws = nullptr;
    p->split_cnt = nullptr;
    p->split_cap = 0;
    const int64_t cap = std::max<int64_t>(cells, 64);
    const size_t ws_bytes = static_cast<size_t>(cap) * p->split * 4 * 1024 * sizeof(double);
    if (hipMalloc(reinterpret_cast<void**>(&p->split_ws), ws_bytes) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&p->split_cnt), cap * sizeof(int)) != hipSuccess) {
      hipFree(p->split_ws);
      p->split_ws = nullptr;
      p->split_cnt = nullptr;
      rc = QCOLL_ENOMEM;
    } else if (hipMemsetAsync(p->split_cnt, 0, cap * sizeof(int), stream) != hipSuccess) {   // not captured (above)
      rc = QCOLL_EDEVICE;
    } else {
      p->split_cap = cap;
      p->split_alloc = p->split;
    }
  }
  if (cur != p->device) hipSetDevice(cur);
  return rc;
}

// Shared by qcoll_eval_multi and qcoll_step_multi: validate the slot list and
// build the batched launch (one workgroup per waves_per_block cells of a slot).
static int multi_launch(const qcoll_plan_t* plans, int nplans, const float* const* f, void* const* Q,
                        const int64_t* cells, bool step, double dt, double eps, int scheme,
                        int32_t* const* status, hipStream_t stream) {
  if (!plans || nplans < 0 || nplans > 64 || !f || !cells) return QCOLL_EINVAL;
  if (!step && !Q) return QCOLL_EINVAL;
  if (step && (!(dt > 0.0) || !(eps > 0.0) || !std::isfinite(dt) || !std::isfinite(eps))) return QCOLL_EINVAL;
  if (step && scheme != QCOLL_EXPLICIT_EULER && scheme != QCOLL_IMEX_EULER_PENALIZED) return QCOLL_EINVAL;
  qcoll::MultiArgs m;
  int wpb = 4, dev = -1;
  int64_t blocks = 0;
  for (int i = 0; i < nplans; ++i) {
    const qcoll_plan_s* p = plans[i];
    if (!p || cells[i] < 0) return QCOLL_EINVAL;
    if (!p->on_device || p->galerkin || p->classical) return QCOLL_EUNSUPPORTED;
    if (dev >= 0 && p->device != dev) return QCOLL_EINVAL;
    dev = p->device;
    if (cells[i] > 0 && (!f[i] || (!step && !Q[i]))) return QCOLL_EINVAL;
    if (p->hp.d != plans[0]->hp.d) return QCOLL_EUNSUPPORTED;  // 2D and 3D plans do not mix
  }
  if (nplans > 0 && plans[0]->hp.d == 3) {
    const qcoll_plan_s* pl[qcoll::kMaxSlots];
    qcoll::Slot3 sl[qcoll::kMaxSlots];
    int64_t cs[qcoll::kMaxSlots];
    int ns = 0;
    for (int i = 0; i < nplans; ++i) {
      if (cells[i] == 0) continue;
      if (ns == qcoll::kMaxSlots) {  // slot table full: launch it and start the next
        if (launch3(pl, sl, ns, cs, stream)) return QCOLL_EDEVICE;
        ns = 0;
      }
      pl[ns] = plans[i];
      sl[ns] = make_slot3(plans[i]);
      sl[ns].f = f[i];
      if (step) {
        sl[ns].dt_eps = dt / eps;
        sl[ns].scheme = scheme;
        sl[ns].status = status ? status[i] : nullptr;
        sl[ns].out_kind = 2;
      } else {
        sl[ns].q = Q[i];
        sl[ns].out_kind = (plans[i]->flags & QCOLL_CONSERVE) ? 1 : 0;
      }
      cs[ns] = cells[i];
      ++ns;
    }
    if (ns == 0) return QCOLL_OK;
    return launch3(pl, sl, ns, cs, stream) ? QCOLL_EDEVICE : QCOLL_OK;
  }
  // tile-64 plans in the split form: every slot of a plan takes its own range of
  // the plan's split buffers (a plan may fill several slots of one launch)
  std::vector<std::pair<qcoll_plan_s*, int64_t>> split_use;
  for (int i = 0; i < nplans; ++i) {
    qcoll_plan_s* p = plans[i];
    if (p->split <= 1 || p->tile != 64 || cells[i] == 0) continue;
    auto it = std::find_if(split_use.begin(), split_use.end(), [p](const auto& u) { return u.first == p; });
    if (it == split_use.end()) split_use.emplace_back(p, cells[i]);
    else it->second += cells[i];
  }
  for (auto& u : split_use) {
    if (int rc = ensure_split_ws(u.first, u.second, stream)) return rc;
    u.second = 0;   // from here on: the next free cell of the plan's buffers
  }
  std::vector<MultiJob> jobs;
  for (int i = 0; i < nplans; ++i) {
    if (cells[i] == 0) continue;
    qcoll_plan_s* p = plans[i];
    qcoll::KernelArgs a = make_args(p);
    if (p->split > 1 && p->tile == 64) {
      auto it = std::find_if(split_use.begin(), split_use.end(), [p](const auto& u) { return u.first == p; });
      a.split_ws = p->split_ws + it->second * p->split * 4 * 1024;
      a.split_cnt = p->split_cnt + it->second;
      it->second += cells[i];
    }
    a.f = f[i];
    a.cells = cells[i];
    if (step) {
      a.dt_eps = dt / eps;
      a.scheme = scheme;
      a.status = status ? status[i] : nullptr;
      a.out_kind = 2;
    } else {
      a.q = Q[i];
      a.out_kind = (p->flags & QCOLL_CONSERVE) ? 1 : 0;
    }
    if (m.nslots == qcoll::kMaxSlots) {  // slot table full: queue it and start the next
      m.block_start[m.nslots] = blocks;
      jobs.emplace_back();
      jobs.back().m = m;
      m = qcoll::MultiArgs();
      blocks = 0;
    }
    m.slot[m.nslots] = a;
    m.block_start[m.nslots] = blocks;
    // tile 64: one workgroup per cell, or per part of a cell in the split form;
    // N <= 32: one wavefront per cell, or one workgroup per cell in the split form
    blocks += p->tile == 64 ? cells[i] * p->split : (p->split > 1 ? cells[i] : (cells[i] + wpb - 1) / wpb);
    ++m.nslots;
  }
  m.block_start[m.nslots] = blocks;
  if (m.nslots > 0) {
    jobs.emplace_back();
    jobs.back().m = m;
  }
  if (jobs.empty()) return QCOLL_OK;
  int64_t total = 0;
  for (int i = 0; i < nplans; ++i) total += cells[i];
  const int cus = plans[0]->cus;
  return run_jobs(jobs, wpb, dev, total <= 4 * static_cast<int64_t>(cus), stream);
}

int qcoll_eval_multi(const qcoll_plan_t* plans, int nplans, const float* const* f, void* const* Q,
                     const int64_t* cells, hipStream_t stream) {
  try {
    return multi_launch(plans, nplans, f, Q, cells, false, 0.0, 0.0, 0, nullptr, stream);
  } catch (const std::bad_alloc&) {
    return QCOLL_ENOMEM;
  }
}

int qcoll_step_multi(const qcoll_plan_t* plans, int nplans, float* const* f, const int64_t* cells, double dt,
                     double eps, int scheme, int32_t* const* status, hipStream_t stream) {
  try {
    return multi_launch(plans, nplans, const_cast<const float* const*>(f), nullptr, cells, true, dt, eps, scheme,
                        status, stream);
  } catch (const std::bad_alloc&) {
    return QCOLL_ENOMEM;
  }
}

static bool split_ok(const qcoll_plan_s* p, int split);

// Eight wavefronts per workgroup select the ping-pong variant of the FX16
// 32x32 kernel (two wavefronts per SIMD in alternating matrix/vector phases).
static bool pingpong_ok(const qcoll_plan_s* p) {
  return p->on_device && p->hp.d == 2 && p->tile == 32 && p->precision == QCOLL_MIX_FX16 && !p->classical;
}

int qcoll_plan_set_launch(qcoll_plan_t p, int waves_per_block, int64_t max_blocks) {
  if (!p) return QCOLL_EINVAL;
  if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4 &&
      !(waves_per_block == 8 && pingpong_ok(p)))
    return QCOLL_EINVAL;
  if (max_blocks < 1) return QCOLL_EINVAL;
  p->waves_per_block = waves_per_block;
  p->max_blocks = max_blocks;
  return QCOLL_OK;
}

int qcoll_plan_get_launch(qcoll_plan_t p, int* waves_per_block, int64_t* max_blocks) {
  if (!p) return QCOLL_EINVAL;
  if (waves_per_block) *waves_per_block = p->waves_per_block;
  if (max_blocks) *max_blocks = p->max_blocks;
  return QCOLL_OK;
}

int qcoll_plan_set_tile(qcoll_plan_t p, int tile) {
  if (!p) return QCOLL_EINVAL;
  if (tile == p->tile) return QCOLL_OK;
  if (!p->on_device || tile != p->alt_tile || p->alt_tile == 0) return QCOLL_EINVAL;
  swap_tile_tables(p);
  if (p->waves_per_block == 8 && !pingpong_ok(p)) p->waves_per_block = 4;
  if (!split_ok(p, p->split)) p->split = 1;
  return QCOLL_OK;
}

// Split factors a plan's kernels support: 4 (a workgroup of four wavefronts per
// cell) for FX16 32x32 tiles; 2, 4, 8 or 16 workgroups per cell for tile-64 plans.
static bool split_ok(const qcoll_plan_s* p, int split) {
  if (split == 1) return true;
  if (!p->on_device || p->hp.d != 2 || p->classical || p->galerkin) return false;
  if (p->tile == 32) return split == 4 && p->precision == QCOLL_MIX_FX16;
  if (p->tile == 64) return split == 2 || split == 4 || split == 8 || split == 16;
  return false;
}

int qcoll_plan_set_split(qcoll_plan_t p, int split) {
  if (!p || !split_ok(p, split)) return QCOLL_EINVAL;
  p->split = split;
  return QCOLL_OK;
}

int qcoll_plan_get_split(qcoll_plan_t p, int* split) {
  if (!p || !split) return QCOLL_EINVAL;
  *split = p->split;
  return QCOLL_OK;
}

int qcoll_plan_get_tile(qcoll_plan_t p, int* tile, int* alternate) {
  if (!p) return QCOLL_EINVAL;
  if (tile) *tile = p->tile;
  if (alternate) *alternate = p->alt_tile;
  return QCOLL_OK;
}

// Time every launch shape on the caller's data with HIP events and keep the
// fastest in the plan: tile family (2D plans with N <= 16: 16x16 or zero-padded
// 32x32 MFMA tiles) x cells per workgroup (1, 2, 4; 8 = the ping-pong variant
// of the FX16 32x32 kernel) x grid cap (1, 2, 8 workgroups per CU, or one per
// cell group). Synchronises the stream. Q receives the result of the last
// timed launch.
int qcoll_plan_autotune(qcoll_plan_t p, const float* f, void* Q, int64_t cells, int reps, hipStream_t stream) {
  if (!p || !f || !Q || cells < 1 || reps < 1) return QCOLL_EINVAL;
  if (!p->on_device || p->hp.d == 3 || p->galerkin || p->classical) return QCOLL_EUNSUPPORTED;  // one fixed launch shape
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return QCOLL_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return QCOLL_EDEVICE;
  }
  const int tiles[2] = {p->tile, p->alt_tile};
  const int wpbs[4] = {1, 2, 4, 8};
  const int64_t caps[4] = {1, 2, 8, 1 << 30};  // multiples of the CU count; last = one wave per cell
  float best = 1e30f;
  int best_t = p->tile, best_w = p->waves_per_block;
  int64_t best_b = p->max_blocks;
  int rc = QCOLL_OK;
  for (int ti = 0; ti < 2 && rc == QCOLL_OK; ++ti) {
    if (tiles[ti] == 0) continue;
    if (p->tile != tiles[ti]) swap_tile_tables(p);
    for (int w : wpbs) {
      if (w == 8 && !pingpong_ok(p)) continue;
      for (int64_t c : caps) {
        qcoll::KernelArgs a = make_args(p);
        a.f = f;
        a.q = Q;
        a.cells = cells;
        a.out_kind = (p->flags & QCOLL_CONSERVE) ? 1 : 0;
        a.waves_per_block = w;
        a.max_blocks = c >= (1 << 30) ? (int64_t{1} << 40) : c * p->cus * (w >= 4 ? 1 : 4 / w);
        if (launch(a, stream)) { rc = QCOLL_EDEVICE; break; }  // warm-up
        hipEventRecord(e0, stream);
        for (int r = 0; r < reps; ++r) launch(a, stream);
        hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess) { rc = QCOLL_EDEVICE; break; }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
          best = ms;
          best_t = p->tile;
          best_w = w;
          best_b = a.max_blocks;
        }
      }
      if (rc != QCOLL_OK) break;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (p->tile != best_t) swap_tile_tables(p);
  if (rc == QCOLL_OK) {
    p->waves_per_block = best_w;
    p->max_blocks = best_b;
  } else if (p->waves_per_block == 8 && !pingpong_ok(p)) {
    p->waves_per_block = 4;
  }
  return rc;
}

int qcoll_plan_info(qcoll_plan_t p, int* transforms, int* K_r, double* R, int64_t* device_bytes) {
  if (!p) return QCOLL_EINVAL;
  if (transforms) *transforms = static_cast<int>(p->hp.packed.size()) + 1;
  if (K_r) *K_r = p->hp.K_r;
  if (R) *R = p->hp.R;
  if (device_bytes)   // tables, plus the split buffers when allocated
    *device_bytes = p->device_bytes + p->split_cap * (static_cast<int64_t>(p->split_alloc) * 4 * 1024 * 8 + 4);
  return QCOLL_OK;
}

int qcoll_plan_table(qcoll_plan_t p, int which, int index, double* out, int64_t n) {
  if (!p || !out || n < 0) return QCOLL_EINVAL;
  const auto& hp = p->hp;
  const std::vector<double>* src = nullptr;
  switch (which) {
    case 0:
    case 1:
      if (index < 0 || index >= static_cast<int>(hp.alpha.size())) return QCOLL_EINVAL;
      src = which == 0 ? &hp.alpha[index] : &hp.alphap[index];
      break;
    case 2: src = &hp.W; break;
    case 3: src = &hp.loss; break;
    case 4: src = &hp.lambda; break;
    case 5: src = p->galerkin ? &p->hp_coarse.gram_inv : &hp.gram_inv; break;
    case 6: {
      if (!p->classical) return QCOLL_EINVAL;
      const int64_t nn = static_cast<int64_t>(hp.N) * hp.N;
      if (index < 0 || index >= nn) return QCOLL_EINVAL;
      if (n < nn) return QCOLL_EINVAL;
      for (int64_t l = 0; l < nn; ++l) out[l] = p->beta[l * nn + index];
      return static_cast<int>(nn);
    }
    default: return QCOLL_EINVAL;
  }
  if (static_cast<int64_t>(src->size()) > n) return QCOLL_EINVAL;
  std::memcpy(out, src->data(), src->size() * sizeof(double));
  return static_cast<int>(src->size());
}

void qcoll_plan_destroy(qcoll_plan_t p) {
  if (!p) return;
  if (p->on_device) free_device(p);
  delete p;
}

const char* qcoll_strerror(int code) {
  switch (code) {
    case QCOLL_OK: return "ok";
    case QCOLL_EINVAL: return "invalid argument";
    case QCOLL_ENOMEM: return "out of memory";
    case QCOLL_EDEVICE: return "HIP device error";
    case QCOLL_EUNSUPPORTED: return "unsupported configuration";
    case QCOLL_ETOOLARGE: return "work larger than the fixed scratch of the no-allocation entry point";
    default: return "unknown error";
  }
}

}  // extern "C"
