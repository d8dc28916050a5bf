// vif_neighbors_noalloc: the exact neighbor search of vif_neighbors with its
// workspace (per-lag tables, flags, the bounding box and the per-slab spatial
// grid) in a file-scope device array instead of a caller-owned buffer, for
// callers that cannot allocate device memory.
//
// Every GPU the library runs on holds its own copy of `scratch` until the
// process ends. Host code never passes the array's name to a kernel or a copy:
// the name is a host-side stand-in, not a device address. The device address
// of each GPU's copy is resolved once per device with hipGetSymbolAddress
// (that device current) and kept; only that address is handed to the search.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "internal.hpp"
#include "vif.h"

namespace {

static __device__ __align__(256) unsigned char scratch[VIF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
std::atomic<void*> g_ptr[kMaxDevices];

// Device address of `dev`'s copy of the array; resolved on first use with that
// device current (the caller's current device is restored).
int32_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return vif::report_error(VIF_E_UNSUPPORTED, "device ordinal out of range for the static scratch");
  void* p = g_ptr[dev].load(std::memory_order_acquire);
  if (p) {
    *out = p;
    return VIF_OK;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  p = g_ptr[dev].load(std::memory_order_relaxed);
  if (!p) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    if (e == hipSuccess) {
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (cur != dev) {
        const hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
      }
    }
    if (e != hipSuccess || !p)
      return vif::report_error(VIF_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device");
    g_ptr[dev].store(p, std::memory_order_release);
  }
  *out = p;
  return VIF_OK;
}

}  // namespace

extern "C" int32_t vif_neighbors_noalloc(const vif_points* p, const vif_kernel* kern, int32_t m,
                                         int32_t* nbr, void* hip_stream) {
  if (!p) return vif::report_error(VIF_E_ARG, "points is NULL");
  if (p->n < 1) return vif::report_error(VIF_E_ARG, "n must be >= 1");
  if (m < 0) return vif::report_error(VIF_E_ARG, "m must be >= 0");
  if (m > VIF_MAX_M) return vif::report_error(VIF_E_UNSUPPORTED, "m exceeds VIF_MAX_M");
  const size_t need = vif_workspace_bytes(p->n, m, 0, VIF_PREC_FP64, VIF_OP_NEIGHBORS);
  if (need == 0 || need > (size_t)VIF_NOALLOC_SCRATCH_BYTES)
    return vif::report_error(VIF_E_WORKSPACE,
                             "n too large for the static scratch of vif_neighbors_noalloc "
                             "(VIF_NOALLOC_SCRATCH_BYTES); use vif_neighbors with a workspace");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  int dev = 0;
  hipError_t e = s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return vif::report_error(VIF_E_DEVICE, "cannot determine the stream's device");
  void* ws = nullptr;
  const int32_t st = scratch_address(dev, &ws);
  if (st) return st;
  // vif_neighbors clears the flags and the grid counters it uses on the stream
  // before reading them, so the contents a previous call left do not matter.
  return vif_neighbors(p, kern, m, nbr, ws, (size_t)VIF_NOALLOC_SCRATCH_BYTES, hip_stream);
}
