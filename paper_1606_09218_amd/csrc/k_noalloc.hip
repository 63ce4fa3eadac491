// Device scratch of the entry points that allocate nothing: one file-scope
// array per GPU, its address looked up once per device.
//
// A __device__ array named in host code is only a host-side stand-in for the
// symbol, not a device address; every host use goes through the pointer that
// hipGetSymbolAddress returns for the current device (each device holds its
// own copy of the array at its own address).
#include "rs_internal.h"

namespace rs {

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex& g_scratch_mu = *new std::mutex;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Called with `device` current (from rs_ctx_create); idempotent.
void noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices)
    throw Error{RS_E_UNSUPPORTED, "device index above the scratch table"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  RS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw Error{RS_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch array"};
  g_scratch_ptr[device] = (double*)ptr;
}

double* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices || !g_scratch_ptr[device])
    throw Error{RS_E_DEVICE, "scratch array of this device not set up (no context created on it)"};
  return g_scratch_ptr[device];
}

}  // namespace rs
