// Host-side internals shared by the C ABI (ar_api.hip) and the query server
// (ar_server.hip).
#pragma once

#include <string>

#include "ar_internal.h"

// A resident scene: device copies of the Gaussians and the workspace of the calls made
// directly on it (ar_render_bounds / ar_render_batch).
struct ar_scene {
  ar::SceneDev dev{};
  ar::Workspace ws{};
  float *base = nullptr;  // one allocation holding the scene arrays
};

namespace ar {

extern thread_local std::string g_error;
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIP_TRY(expr)                                                                                  \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ == hipErrorOutOfMemory) return ::ar::fail(AR_E_OOM, "%s: out of device memory", #expr);    \
    if (e_ != hipSuccess) return ::ar::fail(AR_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int pose_vars(const ar_pose_box *b, bool *rotates);
// pose plus scene variables of a render (AR_OK, or AR_E_UNSUPPORTED above 6 in all)
int render_vars(const ar_scene *sc, const ar_pose_box *b, bool *rotates, int *P);
int validate_box(const ar_pose_box *b);
int make_params(const ar_scene *sc, const ar_intrinsics *in, const ar_options *op, Params &prm);
int check_outputs(const float *lo, const float *hi);
// estimated device bytes of a launch of ncells cells at the list density d (of an earlier
// launch on the scene; zeros: a first guess)
size_t query_bytes(const ar_scene *sc, const Params &prm, int P, bool rotates, int ncells, const Density &d);
// cells per launch of a batch (memory-bounded)
int batch_cells(const ar_scene *sc, const Workspace &ws, const Params &prm, int P, bool rotates,
                const ar_options *opts);
// ncells pose boxes with the same pose variables into images [cell][H][W][3] on stream s,
// using workspace ws; waits for the stream before returning.  cell_scenes (may be null:
// every cell renders sc) gives each cell's scene; scenes other than sc must be plain
// (no scene variables), as sc
int render_cells(const ar_scene *sc, Workspace &ws, const Params &prm, const ar_pose_box *boxes, int ncells, int P,
                 bool rotates, float *lo, float *hi, hipStream_t s, ar_stats *st,
                 const ar_scene *const *cell_scenes = nullptr);
// staging images of the workspace: two blocks of `floats` floats at ws.out_stage
int ensure_out_stage(Workspace &ws, size_t floats);
// buffers of a planned launch; the launch itself (no host synchronisation, no
// allocation: capturable in a HIP graph), pose forms read from poses_dev
int ensure_planned(Workspace &ws, const ar_scene *sc, const Params &prm, int ncells, int P, bool rotates,
                   const PlanCaps &caps);
int render_cells_planned(const ar_scene *sc, Workspace &ws, const Params &prm, const PoseForms *poses_dev,
                         int ncells, int P, bool rotates, float *lo, float *hi, hipStream_t s, const PlanCaps &caps);

}  // namespace ar
