// A fixed device work area for batches created without a caller work buffer, for callers
// that cannot allocate device memory (code under graph capture, serving loops).  The area is
// a file-scope device array; its device address is taken once per device, with that device
// current, and only that address is handed to kernels.  One batch at a time may use the area
// of a device: a second request while it is held fails.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mpsb.h"
#include "kernels.h"

namespace mpsb {

__device__ __align__(256) char scratch[MPSB_STATIC_WORK_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {nullptr};
bool g_held[MAX_DEVICES] = {false};
}  // namespace

hipError_t static_work_acquire(void** ptr, int* device, bool* busy) {
  std::lock_guard<std::mutex> lock(g_mu);
  *busy = false;
  int d = 0;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) return e;
  if (d < 0 || d >= MAX_DEVICES) return hipErrorInvalidDevice;
  if (!g_ptr[d]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[d] = p;
  }
  if (g_held[d]) {
    *busy = true;
    return hipSuccess;
  }
  g_held[d] = true;
  *ptr = g_ptr[d];
  *device = d;
  return hipSuccess;
}

void static_work_release(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (device >= 0 && device < MAX_DEVICES) g_held[device] = false;
}

}  // namespace mpsb
