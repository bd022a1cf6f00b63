// Allocation-free variant of mpv_pyramid (declared in include/mpv.h): the workspace is a
// fixed device array of this translation unit, one copy per GPU, whose address is obtained
// once per device and kept for the life of the process.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mpv.h"

namespace {

// The array itself. In host code its name stands for a host-side shadow, not for device
// memory: kernels and copies get the per-device address from hipGetSymbolAddress instead.
__device__ __align__(256) uint8_t scratch[MPV_PYRAMID_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices];  // per-device address of `scratch`, null until set up
std::mutex g_mu;

// Address of this device's copy of the array; the device must be current.
mpv_status device_scratch(int dev, void** ptr) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MPV_ERR_DEVICE;
    g_scratch[dev] = p;
  }
  *ptr = g_scratch[dev];
  return MPV_OK;
}

}  // namespace

extern "C" mpv_status mpv_pyramid_noalloc(const mpv_pyramid_params* p, const mpv_image* left,
                                          const mpv_image* right, const mpv_pyramid_out* out,
                                          hipStream_t stream) {
  if (!p || !left || !right || !out) return MPV_ERR_INVALID_ARG;
  const size_t need = mpv_pyramid_workspace_bytes(p, left->width, left->height);
  // invalid parameters or shapes: mpv_pyramid reports them before it looks at a workspace
  if (need == 0) return mpv_pyramid(p, left, right, out, nullptr, 0, stream);
  if (need > MPV_PYRAMID_NOALLOC_MAX_BYTES) return MPV_ERR_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MPV_ERR_DEVICE;
  void* ws = nullptr;
  const mpv_status st = device_scratch(dev, &ws);
  if (st != MPV_OK) return st;
  return mpv_pyramid(p, left, right, out, ws, MPV_PYRAMID_NOALLOC_MAX_BYTES, stream);
}
