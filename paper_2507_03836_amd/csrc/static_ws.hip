// Library-owned scratch for the entry points that allocate nothing
// (fhash_fused_train_static): a file-scope device array, one copy per GPU,
// resolved to its device address once per device.
//
// The array's name is a host-side stand-in in host code; only the address
// returned by hipGetSymbolAddress (taken with the device current) may be
// passed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace fh {

namespace {

// Decoder-gradient partials of one fused training launch: at most 256
// workgroups (2048 waves of the backward modes) x the largest decoder the
// fused kernels are built for (32 inputs, 3 hidden layers of 64: 10,497
// parameters), rounded up to 10,560 floats per partial.
constexpr size_t kStaticPartialFloats = 10560;
constexpr size_t kStaticPartials = 256;
constexpr size_t kStaticFloats = kStaticPartials * kStaticPartialFloats;

__device__ __align__(256) float scratch[kStaticFloats];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

size_t static_scratch_bytes() { return kStaticFloats * sizeof(float); }

// Device address of the current device's copy of the scratch array (set up
// on the first call for that device, with it current).
hipError_t static_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return hipSuccess;
}

}  // namespace fh
