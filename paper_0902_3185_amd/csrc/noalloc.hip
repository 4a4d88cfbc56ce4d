// Fixed device scratch for the entry point that allocates nothing
// (dmrg_hpsi_noalloc): a file-scope device array, one copy per GPU, whose
// device address is looked up once per device when a context is created.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace dmrg {

// kScratchFloats floats on every device the library runs on, held until the
// process ends.  Host code never uses the array's name as an address: only
// the pointer that hipGetSymbolAddress returned for the device.
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return hipSuccess;
  int prev = -1;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return e;
  if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (prev != device) (void)hipSetDevice(prev);
  if (e != hipSuccess) return e;
  if (p == nullptr) return hipErrorInvalidSymbol;
  g_ptr[device] = p;
  return hipSuccess;
}

float* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return static_cast<float*>(g_ptr[device]);
}

}  // namespace dmrg
