// k_scratch.hip -- the fixed device scratch of npt_render_noalloc: one
// static array in every GPU's copy of the code object, held until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is a stand-in, not a device address): it looks the address up once
// per device with hipGetSymbolAddress and uses that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "npt.h"
#include "npt_kernels.h"

namespace npt {

static __device__ __align__(256) unsigned char scratch[NPT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_ptr(int device, void** ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace npt
