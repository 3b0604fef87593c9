// The allocation-free entry point: mpts_integrate_dev on a workspace that is
// a file-scope device array of this library instead of caller memory, for
// callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// The array is `scratch` below.  Each GPU the library runs on holds its own
// copy until the process ends.  In host code the name `scratch` is only a
// host-side stand-in: the device address of the current GPU's copy comes
// from hipGetSymbolAddress, taken once per device (with that device
// current) and kept in g_scratch_ptr; every use below goes through that
// pointer.  The call allocates nothing: it only launches kernels and issues
// stream-ordered copies of its small descriptors.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mpts.h"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[MPTS_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (nullptr and the
// HIP error on failure).
void *scratch_ptr(hipError_t *err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

namespace mpts {

// The current device's scratch address (first use on a device sets it up).
int noalloc_scratch(void **ptr) {
  hipError_t e = hipSuccess;
  void *p = scratch_ptr(&e);
  if (!p) return MPTS_EHIP;
  *ptr = p;
  return MPTS_OK;
}

// Defined with the contexts (mpts_host.cpp): MPTS_OK when an integration of
// nsteps steps fits `limit` bytes of workspace, else MPTS_ENOSPC with the
// context's error text set.
int integrate_fits(mpts_ctx *ctx, int64_t nsteps, size_t limit);

}  // namespace mpts

extern "C" int mpts_integrate_dev_noalloc(mpts_ctx *ctx, const void *x0_dev, int64_t nsteps,
                                          void *xout_dev, void *ckpt_dev, void *stream) {
  if (!ctx || !x0_dev || !xout_dev || nsteps < 0) return MPTS_EINVAL;
  int st = mpts::integrate_fits(ctx, nsteps, (size_t)MPTS_NOALLOC_SCRATCH_BYTES);
  if (st != MPTS_OK) return st;
  void *ws = nullptr;
  st = mpts::noalloc_scratch(&ws);
  if (st != MPTS_OK) return st;
  return mpts_integrate_dev(ctx, x0_dev, nsteps, xout_dev, ckpt_dev, ws,
                            (size_t)MPTS_NOALLOC_SCRATCH_BYTES, stream);
}
