// Multi-stage penalised IMEX step for callers that cannot allocate device
// memory (code under graph capture, tight serving loops, harnesses that
// forbid allocation): the step's work buffer is a fixed array in the library's
// device memory instead of a caller-owned buffer.
//
// `scratch` is a file-scope device array. In host code its name only stands
// for the symbol; its device address (one copy per GPU, each at its own
// address) is looked up once per device with hipGetSymbolAddress and kept in
// `g_scratch`, and only that address is ever handed to kernels.

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "qcoll.h"

namespace qcoll {
int plan_device(const qcoll_plan_s* p);   // api.cpp
}

static_assert(QCOLL_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");

static __device__ __align__(256) char scratch[QCOLL_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device dev (looked up with that device
// current the first time, then cached). Returns nullptr on failure.
void* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[dev]) return g_scratch[dev];
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return nullptr;
  if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);   // the lookup's status decides
  if (e != hipSuccess || !ptr) return nullptr;
  g_scratch[dev] = ptr;
  return ptr;
}

}  // namespace

extern "C" int qcoll_step_rk_noalloc(qcoll_plan_t plan, float* f, int64_t cells, double dt, double eps, int scheme,
                                     int32_t* status, hipStream_t stream) {
  if (!plan || cells < 0) return QCOLL_EINVAL;
  const int64_t need = qcoll_step_rk_work_bytes(plan, scheme, cells);
  if (need < 0) return QCOLL_EINVAL;
  if (need > QCOLL_NOALLOC_SCRATCH_BYTES) return QCOLL_ETOOLARGE;
  if (cells == 0) return QCOLL_OK;
  const int dev = qcoll::plan_device(plan);
  if (dev < 0) return QCOLL_EUNSUPPORTED;   // host-only plan
  void* ptr = scratch_on(dev);
  if (!ptr) return QCOLL_EDEVICE;
  // The stage slots and the moments of f^n are written before they are read
  // within the step, so the array needs no clearing between calls.
  return qcoll_step_rk(plan, f, cells, dt, eps, scheme, static_cast<float*>(ptr), QCOLL_NOALLOC_SCRATCH_BYTES, status,
                       stream);
}
