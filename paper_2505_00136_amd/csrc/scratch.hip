// File-scope device scratch of the allocation-free prediction entry point.
//
// `scratch` holds the per-chunk partial sums of the fused K_{Zs,Z} alpha product.  Each
// GPU the library runs on holds its own copy until the process ends.  In host code the
// array's name is not a device address: set-up looks the address up once per device with
// hipGetSymbolAddress (that device current) and every launch takes that pointer.
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace gpr {

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

hipError_t scratch_setup(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    double* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  if (out) *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace gpr
