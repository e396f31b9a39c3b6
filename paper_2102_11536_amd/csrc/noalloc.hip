// ga_apply_Pinv_noalloc: the FP64 preconditioner apply for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).  Its
// two intermediate vectors live in `scratch`, a file-scope device array of fixed
// size that every GPU the library runs on holds from module load until the process
// ends.  Host code never passes the array's name to a kernel (on the host it is
// only a stand-in): the device address is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_dev.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ga_internal.h"

namespace {

// two intermediate vectors of nrhs * n_free doubles each: nrhs * n_free <= GA_NOALLOC_MAX_ENTRIES
constexpr size_t kScratchDoubles = 2 * (size_t)GA_NOALLOC_MAX_ENTRIES;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
double* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

// the device address of `scratch` on the current device (looked up on the first
// call on that device, with that device current)
int scratch_on_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    ga::set_error("ga_apply_Pinv_noalloc: no usable current device");
    return GA_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      ga::set_error(std::string("ga_apply_Pinv_noalloc: hipGetSymbolAddress failed: ") +
                    hipGetErrorString(e));
      return GA_EDEVICE;
    }
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return GA_OK;
}

}  // namespace

extern "C" int ga_apply_Pinv_noalloc(ga_patch* pt, int nrhs, const double* r, double* z,
                                     void* stream) {
  if (!pt || !r || !z) { ga::set_error("null argument"); return GA_EINVAL; }
  if (nrhs < 1) { ga::set_error("nrhs must be >= 1"); return GA_EINVAL; }
  const size_t tot = (size_t)nrhs * (size_t)pt->n_free;
  if (tot > (size_t)GA_NOALLOC_MAX_ENTRIES) {
    ga::set_error("ga_apply_Pinv_noalloc: nrhs * n_free exceeds GA_NOALLOC_MAX_ENTRIES");
    return GA_EINVAL;
  }
  double* base = nullptr;
  const int rc = scratch_on_current_device(&base);
  if (rc) return rc;
  // every pass writes its whole output before the next one reads it: nothing in
  // the scratch needs clearing
  return ga::pinv_apply_scratch(pt, nrhs, r, z, base, base + tot, ga::S(stream));
}
