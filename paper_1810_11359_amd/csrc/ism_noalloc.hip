// ism_simulate_noalloc: ism_simulate whose workspace is a fixed device array
// of the library instead of caller memory, for callers that cannot allocate.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ism.h"

namespace {

// The workspace of every ism_simulate_noalloc call on a device. Each device
// the library runs on holds its own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[ISM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};  // device address of scratch, per device (null until first use)

// Device address of the current device's scratch array, looked up once per
// device with that device current; null on failure.
void *scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" int ism_simulate_noalloc(const ism_room *room, const float *src, int n_src, const float *rcv, int n_rcv,
                                    int precision, float *out, void *stream) {
  size_t need = 0;
  const int st = ism_workspace_size(room, n_src, n_rcv, precision, &need);
  if (st != ISM_OK) return st;
  if (need > (size_t)ISM_NOALLOC_SCRATCH_BYTES) return ISM_E_TOO_LARGE;
  if (!src || !rcv || !out) return ISM_E_INVALID_ARG;
  void *ws = scratch_ptr();
  if (!ws) return ISM_E_DEVICE;
  // every byte the kernels read from the workspace is written earlier in the
  // same call, so nothing needs clearing between calls
  return ism_simulate(room, src, n_src, rcv, n_rcv, precision, out, ws, (size_t)ISM_NOALLOC_SCRATCH_BYTES, stream);
}
