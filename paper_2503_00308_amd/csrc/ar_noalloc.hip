// Allocation-free variant of ar_render_bounds for callers that cannot allocate memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Every device buffer of the render is carved from one file-scope device array
// (`scratch`, kScratchBytes) by the workspace's arena mode; host staging (one pose box's
// forms, the statistics counters) is a file-scope host array.  The call itself makes no
// hipMalloc / hipFree / hipHostMalloc / hipEventCreate and no allocating torch call; the
// kernels are those of ar_render_bounds, so the result is bit for bit the same.
//
// Per device, once, with that device current: hipGetSymbolAddress gives the device
// address of `scratch` on that device (each GPU holds its own copy of the array); host
// code only ever passes that address, never the array's name, to kernels and copies.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>

#include "ar_host.h"

namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;   // 256 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceState {
  std::mutex mu;                 // serialises calls on one device (they share `scratch`)
  bool ready = false;
  unsigned char *ptr = nullptr;  // device address of `scratch` on this device
  ar::PoseForms pose_host;       // host staging of the pose forms
  unsigned long long counters_host[16];
  ar::Workspace ws;              // arena-mode workspace (rebuilt on every call)
};

DeviceState g_dev[kMaxDevices];

}  // namespace

extern "C" int ar_render_bounds_noalloc(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *box,
                                        const ar_options *opts, float *lo_rgb, float *hi_rgb, void *hip_stream,
                                        ar_stats *stats) {
  using ar::fail;
  if (!scene) return fail(AR_E_INVALID, "scene is NULL");
  int rc = ar::validate_box(box);
  if (rc) return rc;
  ar::Params prm{};
  rc = ar::make_params(scene, intr, opts, prm);
  if (rc) return rc;
  rc = ar::check_outputs(lo_rgb, hi_rgb);
  if (rc) return rc;
  bool rot = false;
  int P = 0;
  rc = ar::render_vars(scene, box, &rot, &P);
  if (rc) return rc;
  if (rot)
    return fail(AR_E_UNSUPPORTED,
                "ar_render_bounds_noalloc takes translation boxes of plain scenes only (rotation boxes and "
                "scene variables stage host tables)");
  // the per-item buffers alone must fit before anything is launched
  const size_t per_item = 8 * (size_t)ar::rec_stride(P) + 4 * 64 + 16 * (ar::kMaxP + 1);
  if ((size_t)scene->dev.n * per_item > kScratchBytes)
    return fail(AR_E_UNSUPPORTED, "%d Gaussians need more than the %zu-byte scratch of ar_render_bounds_noalloc",
                scene->dev.n, kScratchBytes);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(AR_E_DEVICE, "no current HIP device (or device index above %d)", kMaxDevices - 1);
  DeviceState &d = g_dev[dev];
  std::lock_guard<std::mutex> lock(d.mu);
  if (!d.ready) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(AR_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    d.ptr = static_cast<unsigned char *>(p);
    d.ready = true;
  }
  // a fresh arena workspace: every buffer is carved again from the start of `scratch`
  d.ws = ar::Workspace{};
  d.ws.arena = d.ptr;
  d.ws.arena_cap = kScratchBytes;
  d.ws.pose_host = &d.pose_host;
  d.ws.host_counters = d.counters_host;
  if (stats) memset(stats, 0, sizeof(*stats));
  rc = ar::render_cells(scene, d.ws, prm, box, 1, P, false, lo_rgb, hi_rgb, (hipStream_t)hip_stream, stats);
  // a failed render may leave launches in flight on the stream: drain them before the
  // next call may reuse the scratch
  if (rc) (void)hipStreamSynchronize((hipStream_t)hip_stream);
  if (rc && d.ws.arena_overflow)
    return fail(AR_E_UNSUPPORTED, "the render needs more than the %zu-byte scratch of ar_render_bounds_noalloc",
                kScratchBytes);
  return rc;
}
