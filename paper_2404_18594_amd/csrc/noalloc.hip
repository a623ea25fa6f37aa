// cdtwa_step_rk4_noalloc: cdtwa_step_rk4 for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).
//
// The workspace of the RK4 steps (status word and mean-field exchange words
// of the fused paths; K1, K2, K3 and the field buffers of the per-stage
// paths) comes from the file-scope device array `scratch` instead of a
// caller buffer.  Each device holds its own copy of the array, at its own
// address, from the first use of the library on that device until the
// process ends.  In host code the name `scratch` is only a host-side stand-in
// for the symbol, never a device address: the device address is looked up
// once per device with hipGetSymbolAddress (with that device current) and
// cached, and only the cached pointer is handed to the kernels.
//
// Nothing here allocates: no hipMalloc, hipFree or allocating library call.
// Every call on one device shares that device's array, so calls that overlap
// on one device (two streams, or two host threads) race on it; the array
// keeps the contents of the last call, and every kernel that needs a cleared
// part clears it itself (the fused paths zero their exchange words with a
// fill kernel at the start of every call).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/cdtwa.h"

namespace cdtwa {
cdtwa_status set_error(cdtwa_status st, const std::string& msg);
size_t step_workspace_bytes(cdtwa_plan P);
cdtwa_status step_rk4_checked(cdtwa_plan P, void* rho, void* ws, double dt, int32_t n_steps, hipStream_t s);
}  // namespace cdtwa

namespace {

static __device__ __align__(256) unsigned char scratch[CDTWA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

// Device address of this device's copy of `scratch` (looked up on the first
// call with that device current).
cdtwa_status scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return cdtwa::set_error(CDTWA_EHIP, std::string("step_rk4_noalloc: hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return cdtwa::set_error(CDTWA_EUNSUPPORTED, "step_rk4_noalloc: device index beyond 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return cdtwa::set_error(CDTWA_EHIP,
                              std::string("step_rk4_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return CDTWA_OK;
}

}  // namespace

extern "C" cdtwa_status cdtwa_step_rk4_noalloc(cdtwa_plan plan, void* rho, double dt, int32_t n_steps,
                                               void* stream) {
  if (!plan || !rho) return cdtwa::set_error(CDTWA_EINVAL, "step_rk4_noalloc: NULL argument");
  if (!(std::isfinite(dt) && dt > 0))
    return cdtwa::set_error(CDTWA_EINVAL, "step_rk4_noalloc: dt must be finite and positive");
  if (n_steps < 0) return cdtwa::set_error(CDTWA_EINVAL, "step_rk4_noalloc: negative n_steps");
  const size_t need = cdtwa::step_workspace_bytes(plan);
  if (need > (size_t)CDTWA_NOALLOC_SCRATCH_BYTES)
    return cdtwa::set_error(CDTWA_EINVAL, "step_rk4_noalloc: the plan needs " + std::to_string(need) +
                                              " bytes of workspace, more than the " +
                                              std::to_string((size_t)CDTWA_NOALLOC_SCRATCH_BYTES) +
                                              " of the static scratch buffer; use cdtwa_step_rk4");
  void* ws = nullptr;
  const cdtwa_status st = scratch_ptr(&ws);
  if (st != CDTWA_OK) return st;
  if (n_steps == 0) return CDTWA_OK;
  return cdtwa::step_rk4_checked(plan, rho, ws, dt, n_steps, (hipStream_t)stream);
}
