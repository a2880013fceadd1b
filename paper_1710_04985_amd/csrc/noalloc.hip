// sptrsv_solve_noalloc: the self-scheduled (or level-scheduled) solve of
// sptrsv_solve for callers that cannot allocate device memory (code under
// HIP graph capture, serving loops, harnesses that forbid hipMalloc).  The
// solve's only per-call device buffer, the position-ordered solution that
// the kernels publish and poll, comes from the file-scope array `scratch`
// below instead of the handle's own buffer.
//
// `scratch` is a __device__ variable: each GPU the library runs on holds its
// own copy, at its own address, for the life of the process.  In host code
// its name is only a stand-in; the device address is looked up once per
// device with hipGetSymbolAddress (with that device current) and cached,
// and only that address is passed to kernels.  Every call on one GPU shares
// the array; the solve refills it with the readiness sentinel first, so the
// previous call's contents never matter, but calls that overlap in time on
// one GPU (different handles on unordered streams) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "api_internal.hpp"
#include "sptrsv.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // SPTRSV_NOALLOC_SCRATCH_BYTES

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (looked up on first use).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return SPTRSV_ERR_NOT_SUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SPTRSV_ERR_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return SPTRSV_OK;
}

}  // namespace

static_assert(kScratchBytes == SPTRSV_NOALLOC_SCRATCH_BYTES, "header and source disagree");

extern "C" int sptrsv_solve_noalloc(sptrsv_handle_t h, const void* b, void* x,
                                    hipStream_t stream) {
  if (!h) return SPTRSV_ERR_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SPTRSV_ERR_HIP;
  if (dev != sptrsv::handle_device(h)) return SPTRSV_ERR_INVALID_ARG;
  void* p = nullptr;
  if (const int st = scratch_address(dev, &p)) return st;
  return sptrsv::solve_external_scratch(h, b, x, p, static_cast<int64_t>(kScratchBytes), stream);
}
