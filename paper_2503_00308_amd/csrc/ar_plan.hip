// Planned batched renders: the whole launch sequence of a batch of pose cells captured
// once in a HIP graph and replayed (include/ar.h, ar_plan_*).
//
// A plan renders its cells once through the ordinary batched path to learn the sizes of
// each launch of cells (list entries, segments, Ind runs), takes capacities with
// headroom, sizes a workspace of its own, runs the capturable launch sequence once
// (render_cells_planned: every count on the device, no host synchronisation, no
// allocation) and captures it, for every launch of cells, together with the copy of the
// cells' pose forms in and of the statistics out.  A replay checks the overflow counter
// of every launch: cells that outgrow the capacities are rendered on the ordinary path
// and the plan is made again from their sizes.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ar_host.h"
#include "ar_limits.h"

using ar::fail;

struct ar_plan {
  const ar_scene *scene = nullptr;
  ar_intrinsics intr{};
  ar_options opts{};
  ar::Params prm{};
  int P = 0;
  bool rotates = false;
  int ncells = 0, per_launch = 0, nlaunch = 0;
  std::vector<ar_pose_box> cells;
  ar::PoseForms *pose_host = nullptr;          // pinned, [ncells]
  ar::PoseForms *pose_dev = nullptr;           // [ncells]
  unsigned long long *stats_host = nullptr;    // pinned, [nlaunch][16] counters of each launch
  float *lo = nullptr, *hi = nullptr;          // the caller's images [ncells][H][W][3]
  ar::Workspace ws;
  ar::PlanCaps caps;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;            // the plan's own stream, captured (the null stream cannot be)
  hipEvent_t ev[2] = {nullptr, nullptr};
};

namespace ar {

static void plan_release_graph(ar_plan *p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

static size_t img_floats(const ar_intrinsics &in) { return (size_t)in.width * in.height * 3; }

// A planned rotation launch holds the running sums of all its list entries at once (1 KB
// each); cells per launch are cut until they fit this.
constexpr double kPlanPrefixBytes = 16.0 * 1024 * 1024 * 1024;

// Sizes of every launch of cells from an ordinary render of them (the images are written
// too), and capacities with a quarter of headroom.
static int plan_size_once(ar_plan *p, hipStream_t s);
static int plan_size(ar_plan *p, hipStream_t s) {
  for (int attempt = 0;; ++attempt) {
    int rc = plan_size_once(p, s);
    if (rc) return rc;
    const double bytes = (double)p->caps.entries * 1024.0;
    if (!p->rotates || bytes <= kPlanPrefixBytes || p->per_launch == 1 || attempt >= 4) return AR_OK;
    p->per_launch = std::max(1, (int)(p->per_launch * 0.9 * kPlanPrefixBytes / bytes));
    p->nlaunch = (p->ncells + p->per_launch - 1) / p->per_launch;
    unsigned long long *h = nullptr;
    HIP_TRY(hipHostMalloc((void **)&h, (size_t)p->nlaunch * 16 * sizeof(unsigned long long), hipHostMallocDefault));
    if (p->stats_host) (void)hipHostFree(p->stats_host);
    p->stats_host = h;
  }
}

static int plan_size_once(ar_plan *p, hipStream_t s) {
  ar_scene *sc = const_cast<ar_scene *>(p->scene);
  Workspace &ws = sc->ws;
  uint64_t entries = 0, segments = 0, runs = 0;
  int L = 0;
  bool compact = false, absolute = false;
  const size_t img = img_floats(p->intr);
  for (int k = 0; k < p->nlaunch; ++k) {
    const int c0 = k * p->per_launch, m = std::min(p->per_launch, p->ncells - c0);
    ar_stats st{};
    int rc = render_cells(p->scene, ws, p->prm, p->cells.data() + c0, m, p->P, p->rotates, p->lo + c0 * img,
                          p->hi + c0 * img, s, &st);
    if (rc) return rc;
    const LaunchSizes &z = ws.last;
    if (p->rotates && z.groups > 1)
      return fail(AR_E_UNSUPPORTED, "a planned launch holds one list group: %llu list entries in %d cells "
                  "(use fewer cells per launch)", (unsigned long long)z.entries, m);
    entries = std::max(entries, z.entries);
    segments = std::max(segments, z.segments);
    runs = std::max(runs, z.runs);
    if (k == 0) L = z.L;
    compact = compact || z.compact;
    absolute = absolute || z.absolute;
  }
  const uint64_t e = entries + entries / 4 + 4096, sg = segments + segments / 4 + 1024, r = runs + runs / 4 + 4096;
  const uint64_t emax = p->rotates ? kMaxGroupEntries : kMaxEntries;
  if (e > emax || sg > 0xFFFFFFF0ull || r > kMaxGroupRuns)
    return fail(AR_E_UNSUPPORTED, "a planned launch outgrows the 32-bit counts (%llu entries, %llu runs); use "
                "fewer cells per launch", (unsigned long long)entries, (unsigned long long)runs);
  p->caps.entries = (uint32_t)e;
  p->caps.runs = (uint32_t)r;
  p->caps.L = p->prm.chunk > 0 ? p->prm.chunk : L;
  // segments: every list of L-position segments fits entries / L + lists (times the 8x8
  // blocks per tile), so with the entries within their room the segments cannot outgrow
  // theirs
  const uint64_t nlists = (uint64_t)p->per_launch * p->prm.ntx * p->prm.nty;
  const uint64_t sg_bound = (e / (uint64_t)std::max(p->caps.L, 1) + nlists + 1) * (uint64_t)tile_subs(p->prm);
  if (std::max(sg, sg_bound) > 0xFFFFFFF0ull)
    return fail(AR_E_UNSUPPORTED, "a planned launch outgrows the 32-bit segment count; use fewer cells per launch");
  p->caps.segments = (uint32_t)std::max(sg, sg_bound);
  p->caps.compact = compact;
  p->caps.absolute = absolute;
  return AR_OK;
}

// The launch sequence of every launch of cells, on stream s (captured or not).
static int plan_issue(ar_plan *p, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(p->pose_dev, p->pose_host, (size_t)p->ncells * sizeof(PoseForms), hipMemcpyHostToDevice, s));
  const size_t img = img_floats(p->intr);
  for (int k = 0; k < p->nlaunch; ++k) {
    const int c0 = k * p->per_launch, m = std::min(p->per_launch, p->ncells - c0);
    int rc = render_cells_planned(p->scene, p->ws, p->prm, p->pose_dev + c0, m, p->P, p->rotates, p->lo + c0 * img,
                                  p->hi + c0 * img, s, p->caps);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(p->stats_host + 16 * (size_t)k, p->ws.counters, 16 * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
  }
  return AR_OK;
}

static bool plan_overflowed(const ar_plan *p) {
  for (int k = 0; k < p->nlaunch; ++k)
    if (p->stats_host[16 * (size_t)k + kOverflow]) return true;
  return false;
}

// Sizes, buffers, one uncaptured run of the sequence (which also sizes the scratch of the
// sorts and scans), then the capture.
static int plan_build(ar_plan *p, hipStream_t s) {
  plan_release_graph(p);
  int rc = plan_size(p, s);
  if (rc) return rc;
  rc = ensure_planned(p->ws, p->scene, p->prm, p->per_launch, p->P, p->rotates, p->caps);
  if (rc) return rc;
  rc = plan_issue(p, s);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  if (plan_overflowed(p)) return fail(AR_E_DEVICE, "planned launch overflowed its own sizing run");
  HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  rc = plan_issue(p, p->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(AR_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
  p->graph = g;
  HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  return AR_OK;
}

static void fill_stats(const ar_plan *p, ar_stats *st) {
  memset(st, 0, sizeof(*st));
  for (int k = 0; k < p->nlaunch; ++k) {
    const unsigned long long *c = p->stats_host + 16 * (size_t)k;
    st->pairs += (int64_t)c[0];
    st->ind_tests += (int64_t)c[1];
    st->n_fallback += (int32_t)c[2];
    st->n_wild += (int32_t)c[3];
    st->n_dropped += (int32_t)c[4];
    st->max_window = std::max(st->max_window, (int32_t)c[5]);
    st->cycles_a += (int64_t)c[6];
    st->cycles_b += (int64_t)c[7];
    st->tile_pairs += (int64_t)c[8];
    st->runs += (int64_t)c[9];
    st->ind_borderline += (int64_t)c[ar::kIndBorder];
  }
  st->P = p->P;
  st->segment_length = p->caps.L;
}

static int set_cells(ar_plan *p, const ar_pose_box *cells) {
  for (int i = 0; i < p->ncells; ++i) {
    int rc = validate_box(&cells[i]);
    if (rc) return rc;
    bool rot = false;
    int P = 0;
    rc = render_vars(p->scene, &cells[i], &rot, &P);
    if (rc) return rc;
    if (P != p->P || rot != p->rotates)
      return fail(AR_E_INVALID, "cell %d has other pose variables than the plan's cells", i);
  }
  for (int i = 0; i < p->ncells; ++i) {
    if (pose_forms_host(cells[i], p->P, p->pose_host[i])) return fail(AR_E_INVALID, "unsupported pose variables");
    if (p->prm.ind_quick == 2) ind_quick_off(p->pose_host[i]);
  }
  p->cells.assign(cells, cells + p->ncells);
  return AR_OK;
}

}  // namespace ar

extern "C" {

void ar_plan_destroy(ar_plan *p) {
  if (!p) return;
  ar::plan_release_graph(p);
  ar::release_workspace(p->ws);
  if (p->pose_host) (void)hipHostFree(p->pose_host);
  if (p->stats_host) (void)hipHostFree(p->stats_host);
  if (p->pose_dev) (void)hipFree(p->pose_dev);
  for (hipEvent_t e : p->ev)
    if (e) (void)hipEventDestroy(e);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
}

int ar_plan_create(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *cells, int32_t ncells,
                   const ar_options *opts, float *lo_rgb, float *hi_rgb, void *hip_stream, ar_plan **out) {
  if (!out) return fail(AR_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!scene) return fail(AR_E_INVALID, "scene is NULL");
  if (!cells || ncells < 1) return fail(AR_E_INVALID, "a plan needs at least one cell");
  for (int i = 0; i < ncells; ++i) {
    int rc = ar::validate_box(&cells[i]);
    if (rc) return rc;
  }
  ar_plan *p = new ar_plan();
  int rc = ar::make_params(scene, intr, opts, p->prm);
  if (!rc) rc = ar::check_outputs(lo_rgb, hi_rgb);
  if (!rc) rc = ar::render_vars(scene, &cells[0], &p->rotates, &p->P);
  if (rc) {
    delete p;
    return rc;
  }
  p->scene = scene;
  p->intr = *intr;
  if (opts) p->opts = *opts;
  p->ncells = ncells;
  p->lo = lo_rgb;
  p->hi = hi_rgb;
  p->ws.no_events = true;
  hipStream_t s = (hipStream_t)hip_stream;
  p->per_launch = std::min<int>(ncells, ar::batch_cells(scene, const_cast<ar_scene *>(scene)->ws, p->prm, p->P,
                                                         p->rotates, opts));
  p->nlaunch = (ncells + p->per_launch - 1) / p->per_launch;
  hipError_t e = hipHostMalloc((void **)&p->pose_host, (size_t)ncells * sizeof(ar::PoseForms), hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&p->stats_host, (size_t)p->nlaunch * 16 * sizeof(unsigned long long),
                      hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void **)&p->pose_dev, (size_t)ncells * sizeof(ar::PoseForms));
  if (e == hipSuccess) e = hipEventCreate(&p->ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&p->ev[1]);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    ar_plan_destroy(p);
    return fail(e == hipErrorOutOfMemory ? AR_E_OOM : AR_E_DEVICE, "plan allocation failed: %s",
                hipGetErrorString(e));
  }
  rc = ar::set_cells(p, cells);
  if (!rc) rc = ar::plan_build(p, s);
  if (rc) {
    (void)hipStreamSynchronize(s);
    ar_plan_destroy(p);
    return rc;
  }
  *out = p;
  return AR_OK;
}

int ar_plan_set_cells(ar_plan *plan, const ar_pose_box *cells) {
  if (!plan || !cells) return fail(AR_E_INVALID, "plan or cells is NULL");
  return ar::set_cells(plan, cells);
}

int ar_plan_launch(ar_plan *plan, void *hip_stream, ar_stats *stats, int32_t *replanned) {
  if (!plan) return fail(AR_E_INVALID, "plan is NULL");
  if (replanned) *replanned = 0;
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(hipEventRecord(plan->ev[0], s));
  HIP_TRY(hipGraphLaunch(plan->exec, s));
  HIP_TRY(hipEventRecord(plan->ev[1], s));
  HIP_TRY(hipStreamSynchronize(s));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, plan->ev[0], plan->ev[1]));
  if (ar::plan_overflowed(plan)) {
    // the cells outgrew the plan: render them on the ordinary path (plan_size does) and
    // capture again with their sizes
    if (replanned) *replanned = 1;
    int rc = ar::plan_build(plan, s);
    if (rc) return rc;
    if (stats) {
      ar::fill_stats(plan, stats);
      stats->total_ms = 0.0;
    }
    return AR_OK;
  }
  if (stats) {
    ar::fill_stats(plan, stats);
    stats->total_ms = ms;
  }
  return AR_OK;
}

}  // extern "C"
