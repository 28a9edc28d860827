// State readout for callers that cannot allocate device memory (code under graph capture, serving loops, harnesses
// that forbid hipMalloc): cn_mech_state_noalloc.
//
// cn_mech_state gathers the requested state of every instance into a device buffer it allocates for the call, then
// copies that buffer to the caller. This variant runs the same gather kernel into `scratch`, a buffer of fixed size
// that lives as long as the process on every device the library runs on. The device address of a device's copy is
// looked up once per device, with that device current, and kept; host code never passes the array's name itself.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "cn.h"

namespace cn {
int set_error(int code, const char *msg);
int model_device(const cn_model *m);
int mech_state_check(const cn_model *m, int32_t type, int32_t which, const double *out, int64_t n);
int mech_state_run(const cn_model *m, int32_t type, int32_t which, double *out, int64_t n, double *dbuf);
}  // namespace cn

namespace {

static __device__ __align__(256) double scratch[CN_NOALLOC_STATE_MAX];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch[MAX_DEVICES] = {};  // device address of `scratch` on each device, once looked up

// the device address of `scratch` on device `dev` (looked up on the first call for that device)
int scratch_on(int dev, void **out) {
  if (dev < 0 || dev >= MAX_DEVICES) return cn::set_error(CN_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void *p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return cn::set_error(CN_E_DEVICE, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return CN_OK;
}

}  // namespace

extern "C" int cn_mech_state_noalloc(const cn_model *m, int32_t type, int32_t which, double *out, int64_t n) {
  const int rc = cn::mech_state_check(m, type, which, out, n);
  if (rc != CN_OK) return rc;
  if (n > (int64_t)CN_NOALLOC_STATE_MAX)
    return cn::set_error(CN_E_CAPACITY, ("cn_mech_state_noalloc reads at most " + std::to_string(CN_NOALLOC_STATE_MAX) +
                                         " instances (asked for " + std::to_string(n) + "); use cn_mech_state")
                                            .c_str());
  void *p = nullptr;
  const int r = scratch_on(cn::model_device(m), &p);
  if (r != CN_OK) return r;
  return cn::mech_state_run(m, type, which, out, n, static_cast<double *>(p));
}
