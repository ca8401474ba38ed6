// godec_solve_static: godec_solve for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  Its workspace is the file-scope device array `scratch`
// below instead of a caller's buffer.
//
// `scratch` names a host-side stand-in in host code, not a device address:
// the device address of each GPU's copy is taken once per device with
// hipGetSymbolAddress (the device current at the first call) and only that
// address is handed to the kernels.  Every call on a GPU shares the array
// and finds the previous call's contents in it; godec_init sets up every
// buffer it reads before reading it (the same rule as for a caller's
// uninitialised workspace), so nothing relies on a zeroed array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/godec.h"
#include "host_common.h"

using namespace godec_host;

namespace {

__device__ __align__(256) unsigned char scratch[GODEC_STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device: address of its `scratch`

// Device address of the current device's scratch (looked up on the first
// call on that device).
godec_status scratch_of_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0) return fail(GODEC_E_DEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[(size_t)dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GODEC_E_DEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[(size_t)dev] = p;
  }
  *out = g_scratch_ptr[(size_t)dev];
  return GODEC_OK;
}

}  // namespace

extern "C" godec_status godec_solve_static(const void* X_dev, godec_dtype dtype, int64_t m,
                                           int64_t n, int64_t ldx, int32_t r, int64_t k,
                                           int32_t q, uint64_t seed, int32_t iters,
                                           const godec_opts* opts, void* UL_dev, void* VL_dev,
                                           int64_t* S_idx_dev, void* S_val_dev,
                                           godec_info* info) {
  // the per-iteration draws of redraw_a1 are staged in pinned host memory,
  // which this entry point does not allocate
  if (opts && opts->size == sizeof(godec_opts) && opts->redraw_a1)
    return fail(GODEC_E_UNSUPPORTED, "godec_solve_static does not support redraw_a1");
  // size check first: host arithmetic only
  size_t need = 0;
  godec_status s = godec_workspace_size(m, n, r, k, q, dtype, opts, &need);
  if (s != GODEC_OK) return s;
  if (need > (size_t)GODEC_STATIC_SCRATCH_BYTES)
    return fail(GODEC_E_UNSUPPORTED,
                "problem needs " + std::to_string(need) +
                    " bytes of workspace; godec_solve_static's scratch holds " +
                    std::to_string((unsigned long long)GODEC_STATIC_SCRATCH_BYTES) +
                    " (use godec_solve with a caller workspace)");
  void* base = nullptr;
  s = scratch_of_current_device(&base);
  if (s != GODEC_OK) return s;
  return godec_solve(X_dev, dtype, m, n, ldx, r, k, q, seed, iters, base,
                     (size_t)GODEC_STATIC_SCRATCH_BYTES, opts, UL_dev, VL_dev, S_idx_dev,
                     S_val_dev, info);
}
