// Host side of the C ABI (include/ar.h): validation, device workspace and the launch
// sequence of one abstract render.
//
// Sequence for one pose box (AbstractSplat over all pixels, Sec. 3.3):
//   pose forms (host) -> per-Gaussian records (FP64 mid-radius forms) -> depth order
//   (radix sort of the upper depth bound) -> tile lists (count, scan, emit, stable
//   sort by tile) -> per-pixel BlendInd loop (translation boxes: segments of the tile
//   lists and a front-to-back merge; rotation boxes: Ind runs and a two-phase loop)
//   -> lower / upper images.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <string>
#include <vector>

#include "ar_host.h"
#include "ar_limits.h"

using ar::fail;

namespace ar {

thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

void release_workspace(Workspace &ws) {
  for (auto &kv : ws.sizes) (void)hipFree(kv.first);
  if (ws.host_counters) (void)hipHostFree(ws.host_counters);
  if (ws.host_ranges) (void)hipHostFree(ws.host_ranges);
  if (ws.host_seg) (void)hipHostFree(ws.host_seg);
  if (ws.pose_host) (void)hipHostFree(ws.pose_host);
  if (ws.tab_host) (void)hipHostFree(ws.tab_host);
  if (ws.tab_off_host) (void)hipHostFree(ws.tab_off_host);
  for (int i = 0; i < 4; ++i)
    if (ws.ev[i]) (void)hipEventDestroy(ws.ev[i]);
  ws = Workspace{};
}

}  // namespace ar

namespace ar {

static bool finite_box(const ar_pose_box *b) {
  for (int i = 0; i < 9; ++i)
    if (!isfinite(b->R0[i])) return false;
  for (int i = 0; i < 3; ++i)
    if (!isfinite(b->t0[i]) || !isfinite(b->pivot[i])) return false;
  for (int i = 0; i < 6; ++i)
    if (!isfinite(b->lo[i]) || !isfinite(b->hi[i])) return false;
  return true;
}

// number of pose variables; *rotates: the depth order may change inside the box
int pose_vars(const ar_pose_box *b, bool *rotates) {
  if (b->model == AR_POSE_ORBIT) {
    *rotates = b->hi[0] > b->lo[0];
    return *rotates ? 1 : 0;
  }
  int P = 0;
  for (int a = 0; a < 6; ++a) P += b->hi[a] > b->lo[a];
  *rotates = (b->hi[3] > b->lo[3]) || (b->hi[4] > b->lo[4]) || (b->hi[5] > b->lo[5]);
  return P;
}

// Pose variables of the box plus the scene's variables (Sec. 4.6), which follow them in
// the forms; *rotates: the general (depth-order) path is needed, for a rotation or for
// scene variables (a moved mean can change the depth order under any box).
int render_vars(const ar_scene *sc, const ar_pose_box *b, bool *rotates, int *P) {
  const int pp = pose_vars(b, rotates);
  *P = pp + sc->dev.nvar;
  if (sc->dev.nvar > 0) *rotates = true;
  if (*P > kMaxP)
    return fail(AR_E_UNSUPPORTED, "%d pose and %d scene variables: at most %d in all", pp, sc->dev.nvar, kMaxP);
  return AR_OK;
}

int validate_box(const ar_pose_box *b) {
  if (!b) return fail(AR_E_INVALID, "pose box is NULL");
  if (b->model != AR_POSE_CAMERA6 && b->model != AR_POSE_ORBIT)
    return fail(AR_E_INVALID, "unknown pose model %d", b->model);
  if (!finite_box(b)) return fail(AR_E_INVALID, "pose box has a non-finite entry");
  const int na = b->model == AR_POSE_ORBIT ? 1 : 6;
  for (int a = 0; a < na; ++a) {
    if (b->lo[a] > b->hi[a]) return fail(AR_E_INVALID, "pose box axis %d has lo > hi", a);
    const bool angle = b->model == AR_POSE_ORBIT || a >= 3;
    if (angle && 0.5 * (b->hi[a] - b->lo[a]) > 0.5)
      return fail(AR_E_INVALID, "angle half-width above 0.5 rad on axis %d", a);
  }
  return AR_OK;
}

int make_params(const ar_scene *sc, const ar_intrinsics *in, const ar_options *op, Params &prm) {
  if (!in) return fail(AR_E_INVALID, "intrinsics are NULL");
  if (in->width < 1 || in->height < 1 || in->width > 16384 || in->height > 16384)
    return fail(AR_E_INVALID, "image size %dx%d outside [1, 16384]", in->width, in->height);
  if (!(isfinite(in->fx) && isfinite(in->fy) && isfinite(in->cx) && isfinite(in->cy)) || !(in->fx > 0) ||
      !(in->fy > 0))
    return fail(AR_E_INVALID, "intrinsics must be finite with fx, fy > 0");
  ar_options o{};
  if (op) o = *op;
  if (o.tile != 0 && o.tile != kTile && o.tile != kTileMax)
    return fail(AR_E_UNSUPPORTED, "tile %d: only %d and %d are built", o.tile, kTile, kTileMax);
  if (o.ind_window < 0 || o.ind_window > 2) return fail(AR_E_INVALID, "ind_window %d outside [0, 2]", o.ind_window);
  if (o.prefix_entries < 0) return fail(AR_E_INVALID, "prefix_entries %d is negative", o.prefix_entries);
  if (o.cells_per_launch < 0 || o.cells_per_launch > 256)
    return fail(AR_E_INVALID, "cells_per_launch %d outside [0, 256]", o.cells_per_launch);
  if (o.chunk != 0 && (o.chunk < 8 || o.chunk > 4096)) return fail(AR_E_INVALID, "chunk %d outside [8, 4096]", o.chunk);
  if (o.taylor_k < 0 || o.taylor_k > 16) return fail(AR_E_INVALID, "taylor_k %d outside [1, 16]", o.taylor_k);
  if (!(o.cull_budget >= 0.0) || !isfinite(o.cull_budget) || o.cull_budget >= 1.0)
    return fail(AR_E_INVALID, "cull_budget must be in [0, 1)");
  if (!(o.z_near >= 0.0) || !isfinite(o.z_near)) return fail(AR_E_INVALID, "z_near must be finite and >= 0");
  if (!isfinite(o.t_min) || o.t_min >= 1.0) return fail(AR_E_INVALID, "t_min must be finite and < 1");
  for (int32_t v : {o.abs_sums, o.ind_copy, o.ind_masks})
    if (v < 0 || v > 2) return fail(AR_E_INVALID, "layout switch %d outside [0, 2]", v);
  if (o.group_entries < 0) return fail(AR_E_INVALID, "group_entries %d is negative", o.group_entries);
  if (o.inverse < 0 || o.inverse > 2) return fail(AR_E_INVALID, "inverse %d outside [0, 2]", o.inverse);
  if (o.group_runs < 0) return fail(AR_E_INVALID, "group_runs %d is negative", o.group_runs);
  if (o.ind_quick < 0 || o.ind_quick > 2) return fail(AR_E_INVALID, "ind_quick %d outside [0, 2]", o.ind_quick);
  prm.width = in->width;
  prm.height = in->height;
  prm.fx = in->fx;
  prm.fy = in->fy;
  prm.cx = in->cx;
  prm.cy = in->cy;
  prm.taylor_k = o.taylor_k ? o.taylor_k : 8;
  prm.z_near = o.z_near > 0 ? o.z_near : 0.01;
  const double budget = o.cull_budget > 0 ? o.cull_budget : 1e-7;
  prm.cull_budget = budget;
  prm.eps_cull = budget / (double)sc->dev.n;
  prm.E = budget * (1.0 + 0x1p-10);
  prm.t_min = o.t_min == 0.0 ? 1e-7 : o.t_min;  // negative disables the early stop
  prm.tile = o.tile ? o.tile : kTile;
  prm.ntx = (in->width + prm.tile - 1) / prm.tile;
  prm.nty = (in->height + prm.tile - 1) / prm.tile;
  prm.ind_window = o.ind_window;
  prm.chunk = o.chunk;  // 0: chosen per call from the number of (tile, Gaussian) pairs
  prm.prefix_entries = o.prefix_entries;
  prm.abs_sums = o.abs_sums;
  prm.ind_copy = o.ind_copy;
  prm.ind_masks = o.ind_masks;
  prm.group_entries = o.group_entries;
  prm.inverse = o.inverse;
  prm.ind_quick = o.ind_quick;
  prm.group_runs = o.group_runs;
  return AR_OK;
}

// Workspace buffers for n_total = cells * n Gaussian items with P pose variables and
// nlists = cells * ntiles tile lists.
static int ensure_ws(Workspace &ws, size_t n_total, size_t nlists, int P, int ncells) {
  if (n_total > ws.cap_n || !ws.key) {
    const size_t c = n_total + 64;
    HIP_TRY(grow(ws, ws.key, c));
    HIP_TRY(grow(ws, ws.key_sort, c));
    HIP_TRY(grow(ws, ws.key_alt, c));
    HIP_TRY(grow(ws, ws.perm, c));
    HIP_TRY(grow(ws, ws.perm_alt, c));
    HIP_TRY(grow(ws, ws.cell_key, c));
    HIP_TRY(grow(ws, ws.cell_key_alt, c));
    HIP_TRY(grow(ws, ws.rect, 4 * c));
    HIP_TRY(grow(ws, ws.dform, 2 * (kMaxP + 1) * c));
    HIP_TRY(grow(ws, ws.count, c + 1));
    HIP_TRY(grow(ws, ws.dint, 2 * c));
    ws.cap_n = n_total;
  }
  const size_t rec_doubles = n_total * (size_t)rec_stride(P);
  if (rec_doubles > ws.cap_rec || !ws.rec) {
    const size_t c = rec_doubles + 64 * (size_t)rec_stride(kMaxP);
    HIP_TRY(grow(ws, ws.rec, c));
    ws.cap_rec = c;
  }
  if (nlists > ws.cap_tiles || !ws.tile_range) {
    HIP_TRY(grow(ws, ws.tile_range, 2 * nlists + 2));
    HIP_TRY(grow(ws, ws.lbox, kListBox * nlists + 2 * kListBox));
    ws.cap_tiles = nlists;
  }
  if ((size_t)ncells > ws.cap_cells || !ws.pose_dev) {
    if (ws.arena) {
      // arena mode: pose_host is the caller's host storage for one pose box
      if (ncells != 1 || !ws.pose_host) return fail(AR_E_UNSUPPORTED, "arena workspace holds one pose box");
    } else if (ws.pose_host) {
      HIP_TRY(hipHostFree(ws.pose_host));
      ws.pose_host = nullptr;
    }
    HIP_TRY(grow(ws, ws.pose_dev, (size_t)ncells));
    if (!ws.arena)
      HIP_TRY(hipHostMalloc((void **)&ws.pose_host, (size_t)ncells * sizeof(PoseForms), hipHostMallocDefault));
    ws.cap_cells = (size_t)ncells;
  }
  if (!ws.counters) {
    HIP_TRY(grow(ws, ws.counters, 16));
    if (!ws.arena) {
      HIP_TRY(hipHostMalloc((void **)&ws.host_counters, 16 * sizeof(unsigned long long), hipHostMallocDefault));
      if (!ws.no_events)
        for (int i = 0; i < 4; ++i) HIP_TRY(hipEventCreate(&ws.ev[i]));
    }
  }
  return AR_OK;
}

// Rotation path: list entries whose per-pixel prefix sums are held at once (the pixel
// loop runs over chunks of tile lists with at most this many entries, or one list).
constexpr size_t kPrefixEntries = (size_t)1 << 21;   // 2M entries, 2.1 GB
constexpr size_t kRotChunkSegs = (size_t)1 << 16;    // segments per launch of the rotation pixel loop
constexpr double kMaskBytes = 8.0 * 1024 * 1024 * 1024;   // largest store of Ind masks kept between passes
constexpr double kCompactWindow = 32.0;              // mean Ind window from which the tests read the compact copy
constexpr double kAbsoluteRuns = 8.0;                // runs per list position from which the sums are made absolute
constexpr int kRotSegment = 64;                      // list positions per segment (rotation path)
constexpr int kClassifyCells = 1024;                 // pose cells per launch of the classification
constexpr int kMaxRefineDepth = 24;                  // bisections of a cell in the adaptive refinement
constexpr uint64_t kGroupEntries = 1ull << 27;       // list entries per group of the Ind passes (rotation path)

// buffers of the general path: run counts, windows and mask offsets for a list group of
// npairs entries
static int ensure_general(Workspace &ws, size_t npairs) {
  if (2 * npairs + 1 > ws.cap_run_cnt || !ws.run_cnt) {
    const size_t need = 2 * npairs + 1 + npairs / 2 + 1024;
    HIP_TRY(grow(ws, ws.run_cnt, need));
    ws.cap_run_cnt = need;
  }
  if (npairs + 1 > ws.cap_win || !ws.win) {
    const size_t need = npairs + npairs / 4 + 1024;
    HIP_TRY(grow(ws, ws.win, 2 * need));
    HIP_TRY(grow(ws, ws.woff, need + 1));
    ws.cap_win = need;
  }
  return AR_OK;
}

// per-pixel prefix sums: `rows` rows of 64 doubles in each of three planes, the running
// sums of log(1 - a_lo) and of log(1 - a_hi), then the transmittance bounds (a float pair
// per pixel); a launch of the pixel loop takes one row per list entry and one zero row per
// list
static int ensure_prefix(Workspace &ws, size_t rows) {
  if (rows <= ws.cap_pre && ws.pre) return AR_OK;
  const size_t need = rows + rows / 8 + 64;
  HIP_TRY(grow(ws, ws.pre, need * kTilePix * 3));
  ws.cap_pre = need;
  return AR_OK;
}

static int ensure_runs(Workspace &ws, size_t nruns) {
  if (nruns <= ws.cap_runs && ws.runs) return AR_OK;
  const size_t need = nruns + nruns / 4 + 1024;
  HIP_TRY(grow(ws, ws.runs, 2 * need));
  ws.cap_runs = need;
  return AR_OK;
}

// rotation path: pinned segment table (offsets of nlists lists, then segment -> list)
// and its device copy
static int ensure_rot_segments(Workspace &ws, size_t nlists, size_t nseg) {
  const size_t host_need = nlists + 1 + nseg;
  if (host_need > ws.cap_host_seg || !ws.host_seg) {
    if (ws.host_seg) HIP_TRY(hipHostFree(ws.host_seg));
    ws.host_seg = nullptr;
    const size_t need = host_need + host_need / 4 + 1024;
    HIP_TRY(hipHostMalloc((void **)&ws.host_seg, need * sizeof(uint32_t), hipHostMallocDefault));
    ws.cap_host_seg = need;
  }
  if (nlists + 2 > ws.cap_seg_off || !ws.seg_off) {
    HIP_TRY(grow(ws, ws.seg_off, nlists + 2));
    ws.cap_seg_off = nlists + 2;
  }
  if (nseg > ws.cap_seg || !ws.seg_tile) {
    const size_t need = nseg + nseg / 4 + 1024;
    HIP_TRY(grow(ws, ws.seg_tile, need));
    ws.cap_seg = need;
  }
  return AR_OK;
}

// rotation path: list totals of log(1 - a_lo) for nl lists of one launch
static int ensure_listlo(Workspace &ws, size_t nl) {
  if (nl <= ws.cap_listlo && ws.listlo) return AR_OK;
  const size_t need = nl + nl / 4 + 64;
  HIP_TRY(grow(ws, ws.listlo, need * kTilePix));
  ws.cap_listlo = need;
  return AR_OK;
}

// rotation path: segment totals and partial colour sums for nseg segments of one launch
static int ensure_rot_parts(Workspace &ws, size_t nseg, int P) {
  if (nseg > ws.cap_segsum || !ws.segsum) {
    const size_t need = nseg + nseg / 4 + 256;
    HIP_TRY(grow(ws, ws.segsum, need * kTilePix * 2));
    ws.cap_segsum = need;
  }
  const size_t doubles = nseg * (size_t)part_fields(P) * kTilePix;
  if (doubles > ws.cap_part || !ws.part) {
    const size_t need = doubles + doubles / 4 + 4096;
    HIP_TRY(grow(ws, ws.part, need));
    ws.cap_part = need;
  }
  return AR_OK;
}

// Segment length of the rotation pixel loop: fixed (not tied to the size of the call),
// so a cell gives the same bounds alone and in a batch.
static int rot_segment_length(const Params &prm) { return prm.chunk > 0 ? prm.chunk : kRotSegment; }

// translation path: segment table and partial results for up to nseg segments
static int ensure_segments(Workspace &ws, size_t ntiles, size_t nseg, int P) {
  if (ntiles + 2 > ws.cap_seg_off || !ws.seg_off) {
    HIP_TRY(grow(ws, ws.seg_off, ntiles + 2));
    ws.cap_seg_off = ntiles + 2;
  }
  if (nseg > ws.cap_seg || !ws.seg_tile) {
    const size_t need = nseg + nseg / 4 + 1024;
    HIP_TRY(grow(ws, ws.seg_tile, need));
    ws.cap_seg = need;
  }
  const size_t doubles = nseg * (size_t)part_fields(P) * kTilePix;
  if (doubles > ws.cap_part || !ws.part) {
    const size_t need = doubles + doubles / 4 + 4096;
    HIP_TRY(grow(ws, ws.part, need));
    ws.cap_part = need;
  }
  return AR_OK;
}

// Segment length of the translation pixel loop: about two rounds of the waves the
// device holds at once (each nonempty list adds half a segment on average), so the last
// round is nearly full and each wave's share is long enough to amortise its loads; at
// least 32 list positions.  On the 10k-Gaussian 128x128 workload (three waves per SIMD,
// 3072 resident) this gives L = 112, measured 0.91 ms against 0.98 ms at L = 88 and
// 1.06 ms at L = 128.
static int segment_length(const Params &prm, size_t npairs, size_t nlists, int P) {
  if (prm.chunk > 0) return prm.chunk;
  const double C = (double)seg_resident_waves(P);
  const double target = std::max(2.0 * C - 0.5 * (double)nlists, C);
  size_t L = (size_t)ceil((double)npairs / target);
  L = (L + 7) / 8 * 8;
  return (int)std::min<size_t>(std::max<size_t>(L, 32), 4096);
}

static int ensure_pairs(Workspace &ws, size_t npairs) {
  if (npairs <= ws.cap_pairs && ws.pair_key) return AR_OK;
  const size_t need = std::max(npairs + npairs / 4, (size_t)4096);
  HIP_TRY(grow(ws, ws.pair_key, need));
  HIP_TRY(grow(ws, ws.pair_key_alt, need));
  HIP_TRY(grow(ws, ws.pair_val, need));
  HIP_TRY(grow(ws, ws.pair_val_alt, need));
  ws.cap_pairs = need;
  return AR_OK;
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
  const int i = threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void k_zero_u32(uint32_t *p, int n) {
  const int i = threadIdx.x;
  if (i < n) p[i] = 0u;
}

static int bits_for(uint32_t v) {
  int b = 0;
  while (b < 32 && (1ull << b) <= (unsigned long long)v) ++b;
  return b;
}

// Estimated device bytes of a launch of ncells cells: the buffers the launch sequence
// grows (records and per-item arrays, list entries, list boxes, segment partials; on the
// rotation path the windows, run counts, runs, stored masks, the compact copy, prefix
// sums and segment totals of one list group), with their headroom, at the list density d.
size_t query_bytes(const ar_scene *sc, const Params &prm, int P, bool rotates, int ncells, const Density &d) {
  const double items = (double)sc->dev.n * ncells;
  const double lists = (double)prm.ntx * prm.nty * ncells;
  const double pairs = items * (d.pairs_per_item > 0.0 ? d.pairs_per_item : 32.0);
  // per item: record, 3 depth keys, 4 permutation / cell arrays, rectangle, depth forms,
  // count, depth pair
  const double per_item = 8.0 * rec_stride(P) + 24.0 + 16.0 + 16.0 + 16.0 * (kMaxP + 1) + 4.0 + 16.0;
  // list entries (4 arrays of 4 B, 1.25x), radix histograms and scan sums (about 1 B per entry)
  double b = items * per_item + pairs * (20.0 + 1.0) + lists * (8.0 + 8.0 * kListBox) + (double)(16 << 20);
  if (rotates) {
    const double gcap = prm.group_entries > 0 ? (double)prm.group_entries : (double)kGroupEntries;
    const double g = std::min(pairs, gcap);
    b += g * (10.0 + 10.0 + 5.0);                                    // run counts, windows, mask offsets
    b += 1.25 * g * 8.0 * (d.runs_per_entry > 0.0 ? d.runs_per_entry : 16.0);   // runs
    b += std::min(1.25 * g * 8.0 * d.mask_words_per_entry, kMaskBytes);         // stored masks
    if (d.compact || prm.ind_copy == 1) b += 1.25 * g * (16.0 * (P + 1) + 16.0);   // compact copy
    const double pre = prm.prefix_entries > 0 ? (double)prm.prefix_entries : (double)kPrefixEntries;
    b += 1.125 * std::min(pairs + lists, pre) * 64.0 * 24.0;        // prefix sums and transmittances
    const double segs = pairs / kRotSegment + lists;
    b += 1.25 * segs * 4.0 + 1.25 * std::min(segs, (double)kRotChunkSegs) * (8.0 * part_fields(P) * 64.0 + 16.0 * 64.0);
  } else {
    const double segs = tile_subs(prm) * std::min(8192.0 + lists, pairs / 32.0 + lists);
    b += 1.25 * segs * (8.0 * part_fields(P) * 64.0 + 4.0);
  }
  return (size_t)b;
}

// Union of m cell images (each n floats) into out: minimum of the lower images, maximum of
// the upper ones; with first, out is overwritten, else included.
__global__ void k_union(const float *__restrict__ lo_c, const float *__restrict__ hi_c, int m, size_t n, bool first,
                        float *__restrict__ lo, float *__restrict__ hi) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float l = first ? INFINITY : lo[i], h = first ? -INFINITY : hi[i];
  for (int c = 0; c < m; ++c) {
    l = fminf(l, lo_c[(size_t)c * n + i]);
    h = fmaxf(h, hi_c[(size_t)c * n + i]);
  }
  lo[i] = l;
  hi[i] = h;
}

void add_stats(ar_stats &a, const ar_stats &b) {
  a.pairs += b.pairs;
  a.tile_pairs += b.tile_pairs;
  a.n_fallback += b.n_fallback;
  a.n_wild += b.n_wild;
  a.n_dropped += b.n_dropped;
  a.P = std::max(a.P, b.P);
  a.max_window = std::max(a.max_window, b.max_window);
  a.segment_length = std::max(a.segment_length, b.segment_length);
  a.raster_ms += b.raster_ms;
  a.total_ms += b.total_ms;
  a.runs += b.runs;
  a.cycles_a += b.cycles_a;
  a.cycles_b += b.cycles_b;
  a.ind_tests += b.ind_tests;
  a.ind_borderline += b.ind_borderline;
}

// Cells per launch of a batch: the option if given, else as many as fit a quarter of
// the free device memory (at most 64 GiB) at the list density of the last launch (32
// list entries per Gaussian before the first), at most 256.
int batch_cells(const ar_scene *sc, const Workspace &ws, const Params &prm, int P, bool rotates,
                const ar_options *opts) {
  if (opts && opts->cells_per_launch > 0) return opts->cells_per_launch;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = (size_t)16 << 30;
  const double budget = std::min(0.25 * (double)free_b, 64.0 * 1024 * 1024 * 1024);
  const double per_cell = (double)query_bytes(sc, prm, P, rotates, 1, ws.density);
  return (int)std::max(1.0, std::min(256.0, floor(budget / per_cell)));
}

// Rotation path after the tile lists are built: per list group, the Ind windows, tests
// and runs (k_runs, three passes), then the two-phase pixel loop over chunks of the
// group's lists.  A group is a run of consecutive whole lists with at most
// prm.group_entries entries (default kGroupEntries), so the 32-bit scans of a group's
// mask words and run counts cover a bounded number of entries; the group's run total is
// summed in 64 bits and a group with more runs than uint32 offsets hold is rejected.
// One group (no extra synchronisation) when all entries fit.
static int render_rotation(const ar_scene *sc, Workspace &ws, const Params &prm, int P, uint32_t npairs,
                           size_t nlists, int ntiles, float *lo, float *hi, hipStream_t s, ar_stats *st) {
  const uint64_t gcap = prm.group_entries > 0 ? (uint64_t)prm.group_entries : kGroupEntries;
  const bool split = (uint64_t)npairs > gcap;
  if (2 * nlists + 2 > ws.cap_host_ranges || !ws.host_ranges) {
    if (ws.host_ranges) HIP_TRY(hipHostFree(ws.host_ranges));
    ws.host_ranges = nullptr;
    const size_t need = 2 * nlists + 2;
    HIP_TRY(hipHostMalloc((void **)&ws.host_ranges, need * sizeof(uint32_t), hipHostMallocDefault));
    ws.cap_host_ranges = need;
  }
  const uint32_t *R = ws.host_ranges;
  HIP_TRY(launch_list_box(ws, ws.pair_val, ws.pose_dev, (int)nlists, ntiles, sc->dev, s));
  // boxes of the kChunk-position chunks, with which the windows pass trims the Ind windows
  DevCounts wdc;
  if (prm.ind_window != 2) {
    const size_t nchunks = ((size_t)npairs + kChunk - 1) / kChunk;
    if (nchunks * 8 > ws.cap_cbox || !ws.cbox) {
      HIP_TRY(grow(ws, ws.cbox, nchunks * 8 + 64));
      ws.cap_cbox = nchunks * 8 + 64;
    }
    HIP_TRY(launch_chunk_boxes(ws, ws.pair_val, sc->dev, ntiles, npairs, ws.cbox, s));
    wdc.cbox = ws.cbox;
  }
  std::vector<size_t> groups;
  bool have_ranges = false;
  if (split) {
    // the list ranges first: they define the groups
    HIP_TRY(hipMemcpyAsync(ws.host_ranges, ws.tile_range, 2 * nlists * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    have_ranges = true;
    if (!plan_groups(R, nlists, gcap, groups))
      return fail(AR_E_UNSUPPORTED, "a tile list holds more than %llu entries", (unsigned long long)kMaxGroupEntries);
  } else {
    groups = {0, nlists};
  }
  // first and end list position of group g (lists are contiguous and in order; an empty
  // list has the range [0, 0))
  auto span = [&](size_t g, uint32_t &pa, uint32_t &pb) {
    if (!have_ranges) {
      pa = 0;
      pb = npairs;
      return;
    }
    pa = pb = 0;
    bool any = false;
    for (size_t l = groups[g]; l < groups[g + 1]; ++l) {
      if (R[2 * l + 1] > R[2 * l]) {
        if (!any) pa = R[2 * l];
        pb = R[2 * l + 1];
        any = true;
      }
    }
  };
  size_t gmax = 0;
  for (size_t g = 0; g + 1 < groups.size(); ++g) {
    uint32_t pa, pb;
    span(g, pa, pb);
    gmax = std::max<size_t>(gmax, pb - pa);
  }
  int rc = ensure_general(ws, gmax);
  if (rc) return rc;
  const int L = rot_segment_length(prm);
  if (st) st->segment_length = std::max(st->segment_length, L);
  // segment table of all lists (segments of L positions, the last one ragged) and the
  // prefix-sum buffer; built once the list ranges are on the host
  const size_t want = prm.prefix_entries > 0 ? (size_t)prm.prefix_entries : kPrefixEntries;
  size_t cap = 0;
  uint32_t *so = nullptr;
  bool tables = false;
  auto build_tables = [&]() -> int {
    size_t nseg_total = 0, longest = 0;
    for (size_t l = 0; l < nlists; ++l) {
      const size_t nl = R[2 * l + 1] - R[2 * l];
      longest = std::max(longest, nl);
      nseg_total += (nl + (size_t)L - 1) / (size_t)L;
    }
    int r = ensure_prefix(ws, std::min<size_t>(npairs + nlists, std::max(want, longest + 1)));
    if (r) return r;
    r = ensure_rot_segments(ws, nlists, nseg_total);
    if (r) return r;
    so = ws.host_seg;
    ws.last.segments = nseg_total;
    ws.last.L = L;
    uint32_t *stl = ws.host_seg + (nlists + 1);
    so[0] = 0;
    for (size_t l = 0, k = 0; l < nlists; ++l) {
      const uint32_t ns = (R[2 * l + 1] - R[2 * l] + (uint32_t)L - 1) / (uint32_t)L;
      for (uint32_t j = 0; j < ns; ++j) stl[k++] = (uint32_t)l;
      so[l + 1] = so[l] + ns;
    }
    HIP_TRY(hipMemcpyAsync(ws.seg_off, so, (nlists + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    if (nseg_total)
      HIP_TRY(hipMemcpyAsync(ws.seg_tile, stl, nseg_total * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    cap = std::max(std::min<size_t>(ws.cap_pre, want), longest);
    tables = true;
    return AR_OK;
  };
  if (have_ranges) {
    rc = build_tables();
    if (rc) return rc;
  }
  unsigned long long tests_before = 0;   // window statistic counters[1] is cumulative over groups
  bool first_pixel_chunk = true;
  for (size_t g = 0; g + 1 < groups.size(); ++g) {
    const size_t la = groups[g], lb = groups[g + 1];
    uint32_t pa, pb;
    span(g, pa, pb);
    const int ng = (int)(pb - pa);
    // Ind windows, and the mask words of the long ones
    HIP_TRY(launch_runs(P, ws, ws.pair_val, ws.pose_dev, ntiles, sc->dev, pa, ng, prm.ind_window, kRunsWindows,
                        nullptr, false, s, wdc));
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, ws.woff + ng, 1);
    HIP_TRY(hipGetLastError());
    HIP_TRY(exclusive_scan_u32(ws.woff, ng + 1, ws, s));
    HIP_TRY(hipMemcpyAsync(ws.host_counters, ws.woff + ng, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ws.host_counters + 1, ws.counters + 5, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipMemcpyAsync(ws.host_counters + 2, ws.counters + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipStreamSynchronize(s));
    // masks of the long windows are kept for the emitting pass when their (32-bit) offsets
    // cannot have wrapped and they fit kMaskBytes; otherwise that pass tests them again
    const size_t words = *(const uint32_t *)ws.host_counters;
    const double words_max = (double)ng * 2.0 * (double)((ws.host_counters[1] + 63) / 64);
    const unsigned long long tests = ws.host_counters[2] - tests_before;
    tests_before = ws.host_counters[2];
    unsigned long long *masks = nullptr;
    if (!prm.ind_only && prm.ind_masks != 2 && words > 0 && words_max < 4294967295.0 &&
        (double)words * 8.0 <= kMaskBytes) {
      if (words > ws.cap_masks || !ws.masks) {
        const size_t need = words + words / 4 + 1024;
        HIP_TRY(grow(ws, ws.masks, need));
        ws.cap_masks = need;
      }
      masks = ws.masks;
    }
    // long windows on average: the Ind tests read a copy laid out by list position
    const bool compact = prm.ind_copy == 1 || (prm.ind_copy == 0 && (double)tests >= kCompactWindow * (double)ng);
    if (compact && ng > 0) {
      const size_t forms = (size_t)ng * (size_t)(2 * (P + 1));
      if (forms > ws.cap_compact || !ws.cform) {
        const size_t w2 = forms + forms / 4 + 1024;
        HIP_TRY(grow(ws, ws.cform, w2));
        ws.cap_compact = w2;
      }
      if ((size_t)ng > ws.cap_cmean || !ws.cmean) {
        const size_t w2 = (size_t)ng + (size_t)ng / 4 + 256;
        HIP_TRY(grow(ws, ws.cmean, 4 * w2));
        ws.cap_cmean = w2;
      }
      HIP_TRY(launch_ind_gather(P, ws, ws.pair_val, sc->dev, ntiles, pa, ng, s));
    }
    DevCounts dcount;
    dcount.ind_und = prm.ind_und;
    HIP_TRY(launch_runs(P, ws, ws.pair_val, ws.pose_dev, ntiles, sc->dev, pa, ng, prm.ind_window, kRunsCount, masks,
                        compact, s, dcount));
    if (prm.ind_only) continue;   // the undecided pairs were all that was asked for
    // run counts: their 64-bit total beside the 32-bit scan into offsets
    const size_t ncnt = 2 * (size_t)ng;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, ws.run_cnt + ncnt, 1);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, ws.counters + 9, 1);
    HIP_TRY(hipGetLastError());
    HIP_TRY(sum_u32_u64(ws.run_cnt, ncnt, ws.counters + 9, s));
    HIP_TRY(exclusive_scan_u32(ws.run_cnt, (int)(ncnt + 1), ws, s));
    HIP_TRY(hipMemcpyAsync(ws.host_counters + 9, ws.counters + 9, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           s));
    if (!have_ranges)
      HIP_TRY(hipMemcpyAsync(ws.host_ranges, ws.tile_range, 2 * nlists * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint64_t nruns64 = ws.host_counters[9];
    if (!have_ranges) {
      have_ranges = true;
      rc = build_tables();
      if (rc) return rc;
    }
    const uint64_t run_cap = prm.group_runs > 0 ? (uint64_t)prm.group_runs : kMaxGroupRuns;
    if (nruns64 > run_cap) {
      const char *why = "more Ind runs in one list group than its offsets hold";
      // too many runs for the group's uint32 offsets: the lists from this group on are
      // grouped again with a cap scaled to fit (the group's work so far is discarded; the
      // groups before it are complete), unless the group is a single list
      const size_t nl_rest = nlists - la;
      std::vector<size_t> rest;
      const uint64_t cap2 = (uint64_t)((double)std::max(ng, 1) * 0.9 * (double)run_cap / (double)nruns64);
      if (lb - la <= 1 || cap2 < 1 || !plan_groups(R + 2 * la, nl_rest, cap2, rest))
        return fail(AR_E_UNSUPPORTED, "%s: %llu runs in the %d entries of one tile list", why,
                    (unsigned long long)nruns64, ng);
      groups.resize(g);
      for (size_t b : rest) groups.push_back(la + b);
      --g;
      continue;
    }
    const size_t nruns = (size_t)nruns64;
    if (st) st->runs += (int64_t)nruns;
    ws.last.runs += nruns;
    ws.last.groups += 1;
    ws.last.compact = ws.last.compact || compact;
    if (ng > 0) {
      Density &dn = ws.density;
      dn.runs_per_entry = std::max(dn.runs_per_entry, (double)nruns / ng);
      dn.mask_words_per_entry = std::max(dn.mask_words_per_entry, masks ? (double)words / ng : 0.0);
      dn.compact = dn.compact || compact;
    }
    rc = ensure_runs(ws, nruns);
    if (rc) return rc;
    // chunks of consecutive lists of the group with at most cap entries and kRotChunkSegs
    // segments (or one longer list), whose rows (entries plus one zero row per list up to
    // the last non-empty one) fit the prefix planes; leading empty lists that would not
    // fit with the next list form a chunk of their own
    const bool absolute =
        prm.abs_sums == 1 || (prm.abs_sums == 0 && (double)nruns >= kAbsoluteRuns * (double)std::max(ng, 1));
    ws.last.absolute = ws.last.absolute || absolute;
    std::vector<RotChunk> chunks;
    size_t max_segs = 0;
    for (size_t l = la; l < lb;) {
      size_t l1 = l;
      uint32_t pos0 = 0;
      bool have = false;
      while (l1 < lb) {
        const uint32_t b = R[2 * l1], e = R[2 * l1 + 1];
        const size_t rows = (size_t)(l1 - l) + 1;   // zero rows up to this list
        if (e > b) {
          if (!have) {
            if (l1 > l && (size_t)(e - b) + rows > ws.cap_pre) break;
            pos0 = b;
            have = true;
          } else if ((size_t)(e - pos0) > cap || (size_t)(e - pos0) + rows > ws.cap_pre ||
                     so[l1 + 1] - so[l] > kRotChunkSegs) {
            break;
          }
        }
        ++l1;
      }
      RotChunk c;
      c.list0 = (int)l;
      c.nl = (int)(l1 - l);
      c.seg0 = (int)so[l];
      c.nseg = (int)(so[l1] - so[l]);
      c.L = L;
      c.pos0 = pos0;
      c.gbase = pa;
      // with many runs per list position the blend reads each run end once from absolute
      // sums; with few, adding the offsets in the blend is cheaper than a pass over them
      c.absolute = absolute;
      chunks.push_back(c);
      max_segs = std::max(max_segs, (size_t)c.nseg);
      l = l1;
    }
    rc = ensure_rot_parts(ws, max_segs, P);
    if (rc) return rc;
    size_t max_nl = 0;
    for (const RotChunk &c : chunks) max_nl = std::max(max_nl, (size_t)c.nl);
    rc = ensure_listlo(ws, max_nl);
    if (rc) return rc;
    HIP_TRY(launch_runs(P, ws, ws.pair_val, ws.pose_dev, ntiles, sc->dev, pa, ng, prm.ind_window, kRunsEmit, masks,
                        compact, s));
    if (first_pixel_chunk && ws.ev[1]) HIP_TRY(hipEventRecord(ws.ev[1], s));
    first_pixel_chunk = false;
    for (const RotChunk &c : chunks) HIP_TRY(launch_raster_general(P, ws, ws.pair_val, c, prm, lo, hi, s));
  }
  if (ws.ev[2]) HIP_TRY(hipEventRecord(ws.ev[2], s));
  return AR_OK;
}

// Abstract renders of ncells pose boxes (same P, all rotating or all not) with one
// launch per stage: item cell * n + g, list cell * ntiles + tile, images [cell][H][W][3].
// The host waits twice per call (the number of list entries, and on the rotation path
// the number of Ind runs) and once at the end.
// The table of a launch whose cells render different scenes: pinned staging and device
// copy for up to ncells cells.
static int ensure_tab(Workspace &ws, int ncells) {
  if ((size_t)ncells <= ws.cap_tab && ws.tab_dev) return AR_OK;
  if (ws.arena) return fail(AR_E_UNSUPPORTED, "arena workspace renders one scene");
  if (ws.tab_host) HIP_TRY(hipHostFree(ws.tab_host));
  if (ws.tab_off_host) HIP_TRY(hipHostFree(ws.tab_off_host));
  ws.tab_host = nullptr;
  ws.tab_off_host = nullptr;
  HIP_TRY(grow(ws, ws.tab_dev, (size_t)ncells));
  HIP_TRY(grow(ws, ws.tab_off_dev, (size_t)ncells + 1));
  HIP_TRY(hipHostMalloc((void **)&ws.tab_host, (size_t)ncells * sizeof(CellScene), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void **)&ws.tab_off_host, ((size_t)ncells + 1) * sizeof(uint32_t), hipHostMallocDefault));
  ws.cap_tab = (size_t)ncells;
  return AR_OK;
}

// Clears the workspace's launch table when the launch ends (the table is in use only
// for the launch that set it).
struct TabScope {
  Workspace &ws;
  ~TabScope() {
    ws.tab = nullptr;
    ws.tab_off = nullptr;
    ws.tab_cells = 0;
  }
};

int render_cells(const ar_scene *sc, Workspace &ws, const Params &prm_in, const ar_pose_box *boxes, int ncells, int P,
                 bool rotates, float *lo, float *hi, hipStream_t s, ar_stats *st, const ar_scene *const *cell_scenes) {
  Params prm = prm_in;
  prm.nominal_order = rotates ? 1 : 0;   // rotation path: lists in order of the nominal depth
  prm.pose_vars = P - sc->dev.nvar;      // scene variables follow the pose variables
  if (sc->dev.moving) prm.ind_window = 2;   // moved means: every pair of a list is tested
  prm.eps_cull = prm.cull_budget / (double)sc->dev.n;   // this launch's scene (batches of several scenes)
  const int n = sc->dev.n;
  const int ntiles = prm.ntx * prm.nty;
  // cells of different scenes: items of cell c at [first_c, first_c + n_c), first_c the
  // sum of the scenes' sizes before it
  bool mixed = false;
  size_t n_total = (size_t)ncells * n;
  if (cell_scenes) {
    size_t sum = 0;
    for (int c = 0; c < ncells; ++c) {
      mixed = mixed || cell_scenes[c] != sc;
      sum += (size_t)cell_scenes[c]->dev.n;
    }
    if (mixed) n_total = sum;
  }
  const size_t nlists = (size_t)ncells * ntiles;
  if (!rotates && P > 3) return fail(AR_E_INVALID, "more than 3 translation variables");
  if (rotates && prm.tile != kTile) return fail(AR_E_UNSUPPORTED, "tile %d: rotation boxes use %d", prm.tile, kTile);
  if (launch_limit(n_total, 0) || nlists >= kScanMax)
    return fail(AR_E_UNSUPPORTED, "too many cells in one launch (%zu items, %zu tile lists)", n_total, nlists);
  int rc = ensure_ws(ws, n_total, nlists, P, ncells);
  if (rc) return rc;
  TabScope tab_scope{ws};
  if (mixed) {
    rc = ensure_tab(ws, ncells);
    if (rc) return rc;
    size_t off = 0;
    for (int c = 0; c < ncells; ++c) {
      const SceneDev &d = cell_scenes[c]->dev;
      ws.tab_host[c].sc = d;
      ws.tab_host[c].off = off;
      ws.tab_host[c].eps_cull = prm.cull_budget / (double)d.n;   // as a render of that scene alone
      ws.tab_off_host[c] = (uint32_t)off;
      off += (size_t)d.n;
    }
    ws.tab_off_host[ncells] = (uint32_t)off;
    HIP_TRY(hipMemcpyAsync(ws.tab_dev, ws.tab_host, (size_t)ncells * sizeof(CellScene), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ws.tab_off_dev, ws.tab_off_host, ((size_t)ncells + 1) * sizeof(uint32_t),
                           hipMemcpyHostToDevice, s));
    ws.tab = ws.tab_dev;
    ws.tab_off = ws.tab_off_dev;
    ws.tab_cells = ncells;
  }
  const bool timed = ws.ev[0] != nullptr;   // no events in arena mode
  if (timed) HIP_TRY(hipEventRecord(ws.ev[0], s));
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, ws.counters, 16);
  HIP_TRY(hipGetLastError());
  // pose forms on the host; by value for a single translation box, else in device memory
  for (int c = 0; c < ncells; ++c) {
    if (pose_forms_host(boxes[c], P, ws.pose_host[c])) return fail(AR_E_INVALID, "unsupported pose variables %d", P);
    if (prm.ind_quick == 2) ind_quick_off(ws.pose_host[c]);
  }
  const bool by_value = ncells == 1 && !rotates;
  if (!by_value)
    HIP_TRY(hipMemcpyAsync(ws.pose_dev, ws.pose_host, (size_t)ncells * sizeof(PoseForms), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_project(P, sc->dev, ws.pose_host[0], by_value ? nullptr : ws.pose_dev, ncells, prm, ws, s));
  // depth order per cell: the upper depth bound as an orderable 64-bit key, values =
  // global item; then a stable pass by cell
  bool alt = false;
  HIP_TRY(radix_sort_u64(ws.key_sort, ws.key_alt, ws.perm, ws.perm_alt, (int)n_total, 0, 64, ws, s, &alt));
  if (alt) {
    std::swap(ws.key_sort, ws.key_alt);
    std::swap(ws.perm, ws.perm_alt);
  }
  if (ncells > 1) {
    HIP_TRY(launch_cell_keys(ws.perm, (int)n_total, n, ws.cell_key, s, ws.tab_off, ws.tab_cells));
    HIP_TRY(radix_sort_u32(ws.cell_key, ws.cell_key_alt, ws.perm, ws.perm_alt, (int)n_total, 0,
                           ((bits_for((uint32_t)(ncells - 1)) + 7) / 8) * 8, ws, s, &alt));
    if (alt) {
      std::swap(ws.cell_key, ws.cell_key_alt);
      std::swap(ws.perm, ws.perm_alt);
    }
  }
  // tile lists in depth order; the number of entries is summed in 64 bits beside the
  // 32-bit scan, so a total that would wrap is rejected instead of used
  HIP_TRY(launch_count_tiles(P, ws, (int)n_total, n, prm, s));
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, ws.count + n_total, 1);
  HIP_TRY(hipGetLastError());
  HIP_TRY(sum_u32_u64(ws.count, n_total, ws.counters + 8, s));
  HIP_TRY(exclusive_scan_u32(ws.count, (int)n_total + 1, ws, s));
  HIP_TRY(hipMemcpyAsync(ws.host_counters + 8, ws.counters + 8, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const uint64_t npairs64 = ws.host_counters[8];
  if (const char *why = launch_limit(n_total, npairs64))
    return fail(AR_E_UNSUPPORTED, "%s: %llu entries of %zu items (use fewer cells per launch or a smaller image)", why,
                (unsigned long long)npairs64, n_total);
  const uint32_t npairs = (uint32_t)npairs64;
  ws.density = Density{};
  ws.density.pairs_per_item = (double)npairs / (double)std::max<size_t>(n_total, 1);
  rc = ensure_pairs(ws, npairs);
  if (rc) return rc;
  HIP_TRY(launch_emit_tiles(P, ws, (int)n_total, n, prm, s));
  const int lbits = bits_for((uint32_t)(nlists - 1));
  HIP_TRY(radix_sort_u32(ws.pair_key, ws.pair_key_alt, ws.pair_val, ws.pair_val_alt, (int)npairs, 0,
                         ((lbits + 7) / 8) * 8, ws, s, &alt));
  if (alt) {
    std::swap(ws.pair_key, ws.pair_key_alt);
    std::swap(ws.pair_val, ws.pair_val_alt);
  }
  HIP_TRY(launch_tile_ranges(ws.pair_key, (int)npairs, ws.tile_range, (int)nlists, s));
  ws.last = LaunchSizes{};
  ws.last.entries = npairs;
  if (!rotates) {
    // every 8x8 block of a tile walks the tile's list
    const size_t nsub = (size_t)tile_subs(prm);
    const int L = segment_length(prm, npairs * nsub, nlists * nsub, P);
    if (st) st->segment_length = std::max(st->segment_length, L);
    const size_t nseg_max = ((npairs + (size_t)L - 1) / (size_t)L + nlists) * nsub;
    ws.last.L = L;
    ws.last.segments = nseg_max;
    ws.last.groups = 1;
    rc = ensure_segments(ws, nlists, nseg_max, P);
    if (rc) return rc;
    HIP_TRY(launch_segments(ws, (int)nlists, L, s, tile_subs(prm)));
    HIP_TRY(exclusive_scan_u32(ws.seg_off, (int)nlists + 1, ws, s));
    HIP_TRY(launch_segment_map(ws, (int)nlists, s));
    HIP_TRY(launch_raster_translation(P, ws, ws.pair_val, (int)nlists, prm, L, (int)nseg_max, lo, hi, s));
  } else {
    rc = render_rotation(sc, ws, prm, P, npairs, nlists, ntiles, lo, hi, s, st);
    if (rc) return rc;
  }
  if (timed) HIP_TRY(hipEventRecord(ws.ev[3], s));
  HIP_TRY(hipMemcpyAsync(ws.host_counters, ws.counters, (kIndBorder + 1) * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  float ms_raster = 0.0f, ms_total = 0.0f;
  if (timed) {
    if (!prm.ind_only) HIP_TRY(hipEventElapsedTime(&ms_raster, ws.ev[1], ws.ev[2]));
    HIP_TRY(hipEventElapsedTime(&ms_total, ws.ev[0], ws.ev[3]));
  }
  if (st) {
    st->pairs += (int64_t)ws.host_counters[0];
    st->tile_pairs += (int64_t)npairs;
    st->n_fallback += (int32_t)ws.host_counters[2];
    st->n_wild += (int32_t)ws.host_counters[3];
    st->n_dropped += (int32_t)ws.host_counters[4];
    st->P = P;
    st->raster_ms += ms_raster;
    st->total_ms += ms_total;
    st->max_window = std::max(st->max_window, (int32_t)ws.host_counters[5]);
    st->cycles_a += (int64_t)ws.host_counters[6];
    st->cycles_b += (int64_t)ws.host_counters[7];
    st->ind_tests += (int64_t)ws.host_counters[1];
    st->ind_borderline += (int64_t)ws.host_counters[kIndBorder];
  }
  return AR_OK;
}

__global__ void k_fill_u32_n(uint32_t *p, size_t n, uint32_t v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static hipError_t fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32_n, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// *eff = *total when it fits cap, else 0 (an overflowed launch then has no list entries)
__global__ void k_fit_count(const uint32_t *__restrict__ total, uint32_t cap, uint32_t *__restrict__ eff) {
  if (threadIdx.x == 0) eff[0] = total[0] <= cap ? total[0] : 0u;
}

// p[0 .. n) = 0 when the overflow counter is set (no runs are read then)
__global__ void k_zero_if_overflow(uint32_t *__restrict__ p, size_t n, const unsigned long long *__restrict__ ovf) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && ovf[0]) p[i] = 0u;
}

// Workspace buffers of a planned launch of ncells cells with the capacities caps.
int ensure_planned(Workspace &ws, const ar_scene *sc, const Params &prm, int ncells, int P, bool rotates,
                   const PlanCaps &caps) {
  const size_t n_total = (size_t)ncells * sc->dev.n;
  const size_t nlists = (size_t)ncells * prm.ntx * prm.nty;
  int rc = ensure_ws(ws, n_total, nlists, P, ncells);
  if (rc) return rc;
  rc = ensure_pairs(ws, caps.entries);
  if (rc) return rc;
  if (nlists + 2 > ws.cap_seg_off || !ws.seg_off) {
    HIP_TRY(grow(ws, ws.seg_off, nlists + 2));
    ws.cap_seg_off = nlists + 2;
  }
  if (caps.segments > ws.cap_seg || !ws.seg_tile) {
    HIP_TRY(grow(ws, ws.seg_tile, caps.segments));
    ws.cap_seg = caps.segments;
  }
  if (!rotates) return ensure_segments(ws, nlists, caps.segments, P);
  rc = ensure_general(ws, caps.entries);
  if (rc) return rc;
  rc = ensure_runs(ws, caps.runs);
  if (rc) return rc;
  rc = ensure_prefix(ws, (size_t)caps.entries + nlists);
  if (rc) return rc;
  rc = ensure_rot_parts(ws, caps.segments, P);
  if (rc) return rc;
  rc = ensure_listlo(ws, nlists);
  if (rc) return rc;
  if (caps.compact) {
    const size_t forms = (size_t)caps.entries * (size_t)(2 * (P + 1));
    if (forms > ws.cap_compact || !ws.cform) {
      HIP_TRY(grow(ws, ws.cform, forms));
      ws.cap_compact = forms;
    }
    if ((size_t)caps.entries > ws.cap_cmean || !ws.cmean) {
      HIP_TRY(grow(ws, ws.cmean, 4 * (size_t)caps.entries));
      ws.cap_cmean = caps.entries;
    }
  }
  return AR_OK;
}

// A launch of ncells pose cells (same P, all rotating or all not) with no host
// synchronisation and no allocation, so that it can be captured in a HIP graph: every
// count stays on the device and the kernels run over the capacities caps (the buffers
// were sized by ensure_planned).  Pose forms are read from poses_dev[ncells].  List
// entries past the count are keyed past the last list (sorted to the end, in no list),
// segments past the count map to an empty list; a count above its capacity skips the
// writes that would exceed it and sets the overflow counter, which the caller reads
// after the launch (the images are then not valid).  The rotation path runs as one list
// group with the Ind masks not stored.
int render_cells_planned(const ar_scene *sc, Workspace &ws, const Params &prm_in, const PoseForms *poses_dev,
                         int ncells, int P, bool rotates, float *lo, float *hi, hipStream_t s, const PlanCaps &caps) {
  Params prm = prm_in;
  prm.nominal_order = rotates ? 1 : 0;
  prm.pose_vars = P - sc->dev.nvar;
  if (sc->dev.moving) prm.ind_window = 2;
  if (rotates && prm.tile != kTile) return fail(AR_E_UNSUPPORTED, "tile %d: rotation boxes use %d", prm.tile, kTile);
  const int n = sc->dev.n;
  const int ntiles = prm.ntx * prm.nty;
  const size_t n_total = (size_t)ncells * n;
  const size_t nlists = (size_t)ncells * ntiles;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, ws.counters, 16);
  HIP_TRY(hipGetLastError());
  PoseForms unused{};
  HIP_TRY(launch_project(P, sc->dev, unused, poses_dev, ncells, prm, ws, s));
  bool alt = false;
  HIP_TRY(radix_sort_u64(ws.key_sort, ws.key_alt, ws.perm, ws.perm_alt, (int)n_total, 0, 64, ws, s, &alt));
  if (alt) {
    std::swap(ws.key_sort, ws.key_alt);
    std::swap(ws.perm, ws.perm_alt);
  }
  if (ncells > 1) {
    HIP_TRY(launch_cell_keys(ws.perm, (int)n_total, n, ws.cell_key, s));
    HIP_TRY(radix_sort_u32(ws.cell_key, ws.cell_key_alt, ws.perm, ws.perm_alt, (int)n_total, 0,
                           ((bits_for((uint32_t)(ncells - 1)) + 7) / 8) * 8, ws, s, &alt));
    if (alt) {
      std::swap(ws.cell_key, ws.cell_key_alt);
      std::swap(ws.perm, ws.perm_alt);
    }
  }
  HIP_TRY(launch_count_tiles(P, ws, (int)n_total, n, prm, s));
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, ws.count + n_total, 1);
  HIP_TRY(hipGetLastError());
  HIP_TRY(sum_u32_u64(ws.count, n_total, ws.counters + 8, s));
  HIP_TRY(exclusive_scan_u32(ws.count, (int)n_total + 1, ws, s));
  // the scanned total, and its value when it fits the capacity (else 0, so that an
  // overflowed launch has no entries: every key is padding and every list empty)
  const uint32_t cap = caps.entries;
  uint32_t *entries = ws.count + n_total + 1;
  hipLaunchKernelGGL(k_fit_count, dim3(1), dim3(64), 0, s, ws.count + n_total, cap, entries);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_emit_tiles(P, ws, (int)n_total, n, prm, s, cap));
  HIP_TRY(launch_fill_tail(ws.pair_key, entries, cap, 0xFFFFFFFFu, s));
  const int lbits = bits_for((uint32_t)(nlists - 1));
  HIP_TRY(radix_sort_u32(ws.pair_key, ws.pair_key_alt, ws.pair_val, ws.pair_val_alt, (int)cap, 0,
                         ((lbits + 7) / 8) * 8, ws, s, &alt));
  if (alt) {
    std::swap(ws.pair_key, ws.pair_key_alt);
    std::swap(ws.pair_val, ws.pair_val_alt);
  }
  HIP_TRY(launch_tile_ranges(ws.pair_key, (int)cap, ws.tile_range, (int)nlists, s));
  const int L = caps.L;
  HIP_TRY(launch_segments(ws, (int)nlists, L, s, tile_subs(prm)));
  HIP_TRY(exclusive_scan_u32(ws.seg_off, (int)nlists + 1, ws, s));
  if (!rotates) {
    HIP_TRY(launch_segment_map(ws, (int)nlists, s, caps.segments));
    HIP_TRY(launch_raster_translation(P, ws, ws.pair_val, (int)nlists, prm, L, (int)caps.segments, lo, hi, s));
    return AR_OK;
  }
  HIP_TRY(launch_list_box(ws, ws.pair_val, poses_dev, (int)nlists, ntiles, sc->dev, s));
  DevCounts dc;
  dc.entries = entries;
  dc.runs_cap = caps.runs;
  HIP_TRY(launch_runs(P, ws, ws.pair_val, poses_dev, ntiles, sc->dev, 0, (int)cap, prm.ind_window, kRunsWindows,
                      nullptr, false, s, dc));
  if (caps.compact) HIP_TRY(launch_ind_gather(P, ws, ws.pair_val, sc->dev, ntiles, 0, (int)cap, s, entries));
  const size_t ncnt = 2 * (size_t)cap;
  HIP_TRY(fill_u32(ws.run_cnt, ncnt + 1, 0u, s));
  HIP_TRY(launch_runs(P, ws, ws.pair_val, poses_dev, ntiles, sc->dev, 0, (int)cap, prm.ind_window, kRunsCount,
                      nullptr, caps.compact, s, dc));
  HIP_TRY(sum_u32_u64(ws.run_cnt, ncnt, ws.counters + 9, s));
  HIP_TRY(exclusive_scan_u32(ws.run_cnt, (int)(ncnt + 1), ws, s));
  HIP_TRY(launch_runs(P, ws, ws.pair_val, poses_dev, ntiles, sc->dev, 0, (int)cap, prm.ind_window, kRunsEmit,
                      nullptr, caps.compact, s, dc));
  // runs beyond their room were not written: then no entry has runs (the images are
  // redone by the caller)
  hipLaunchKernelGGL(k_zero_if_overflow, dim3((unsigned)((ncnt + 1 + 255) / 256)), dim3(256), 0, s, ws.run_cnt,
                     ncnt + 1, (const unsigned long long *)(ws.counters + kOverflow));
  HIP_TRY(hipGetLastError());
  // segments past the count belong to the empty list nlists (ranges [0, 0))
  HIP_TRY(fill_u32(ws.seg_tile, caps.segments, (uint32_t)nlists, s));
  HIP_TRY(launch_segment_map(ws, (int)nlists, s, caps.segments));
  RotChunk c;
  c.list0 = 0;
  c.nl = (int)nlists;
  c.seg0 = 0;
  c.nseg = (int)caps.segments;
  c.L = L;
  c.pos0 = 0;
  c.gbase = 0;
  c.absolute = caps.absolute;
  HIP_TRY(launch_raster_general(P, ws, ws.pair_val, c, prm, lo, hi, s));
  return AR_OK;
}

}  // namespace ar

// ------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------
namespace ar {

int check_outputs(const float *lo, const float *hi) {
  if (!lo || !hi) return fail(AR_E_INVALID, "output image is NULL");
  hipPointerAttribute_t a{};
  for (const float *p : {lo, hi}) {
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess || a.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      return fail(AR_E_INVALID, "output images must be device memory");
    }
  }
  return AR_OK;
}

// Outputs that are both device memory (*host = false) or both host memory, pinned or
// pageable (*host = true: the images are rendered into workspace buffers and copied).
static int check_outputs_any(const float *lo, const float *hi, bool *host) {
  if (!lo || !hi) return fail(AR_E_INVALID, "output image is NULL");
  bool dev[2];
  int k = 0;
  for (const float *p : {lo, hi}) {
    hipPointerAttribute_t a{};
    const hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) (void)hipGetLastError();   // memory HIP does not know: pageable host memory
    dev[k++] = e == hipSuccess && a.type == hipMemoryTypeDevice;
  }
  if (dev[0] != dev[1]) return fail(AR_E_INVALID, "one output image is device memory and the other is not");
  *host = !dev[0];
  return AR_OK;
}

// Host outputs: the device images of `cells` cells (workspace buffers, grown as needed)
int ensure_out_stage(Workspace &ws, size_t floats) {
  if (floats <= ws.cap_out_stage && ws.out_stage) return AR_OK;
  HIP_TRY(grow(ws, ws.out_stage, 2 * floats));
  ws.cap_out_stage = floats;
  return AR_OK;
}

// Renders m cells of one launch into lo / hi, through the workspace's staging images when
// the outputs are host memory (copied back before returning).
static int render_cells_out(const ar_scene *sc, Workspace &ws, const Params &prm, const ar_pose_box *cells, int m,
                            int P, bool rot, float *lo, float *hi, bool host, hipStream_t s, ar_stats *st,
                            const ar_scene *const *cell_scenes = nullptr) {
  if (!host) return render_cells(sc, ws, prm, cells, m, P, rot, lo, hi, s, st, cell_scenes);
  const size_t n = (size_t)m * prm.width * prm.height * 3;
  int rc = ensure_out_stage(ws, n);
  if (rc) return rc;
  float *dlo = ws.out_stage, *dhi = ws.out_stage + n;
  rc = render_cells(sc, ws, prm, cells, m, P, rot, dlo, dhi, s, st, cell_scenes);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(lo, dlo, n * sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(hi, dhi, n * sizeof(float), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return AR_OK;
}

// Cells rendered as ar_render_batch in launches of up to 64 cells (or
// options.cells_per_launch) and united into lo / hi: minimum of the lower images,
// maximum of the upper ones.  stats (may be NULL) accumulates over the cells.
int render_union(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *cells, size_t ncells,
                 const ar_options *opts, float *lo_rgb, float *hi_rgb, hipStream_t s, ar_stats *stats) {
  const int per = opts && opts->cells_per_launch > 0 ? opts->cells_per_launch : 64;
  const size_t img = (size_t)intr->width * intr->height * 3;
  const int m_max = (int)std::min<size_t>(ncells, (size_t)per);
  Workspace &ws = const_cast<ar_scene *>(scene)->ws;
  if (2 * (size_t)m_max * img > ws.cap_union || !ws.union_img) {
    HIP_TRY(grow(ws, ws.union_img, 2 * (size_t)m_max * img));
    ws.cap_union = 2 * (size_t)m_max * img;
  }
  float *tlo = ws.union_img, *thi = ws.union_img + (size_t)m_max * img;
  ar_stats total{};
  for (size_t c0 = 0; c0 < ncells; c0 += (size_t)m_max) {
    const int m = (int)std::min<size_t>((size_t)m_max, ncells - c0);
    ar_stats st{};
    int rc = ar_render_batch(scene, intr, cells + c0, m, opts, tlo, thi, s, &st);
    if (rc) return rc;
    add_stats(total, st);
    hipLaunchKernelGGL(k_union, dim3((unsigned)((img + 255) / 256)), dim3(256), 0, s, tlo, thi, m, img, c0 == 0,
                       lo_rgb, hi_rgb);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (stats) *stats = total;
  return AR_OK;
}

__global__ void k_zero_u64_n(unsigned long long *p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Device memory released when the holder goes out of scope.
struct DeviceBuffer {
  void *p = nullptr;
  ~DeviceBuffer() {
    if (p) (void)hipFree(p);
  }
};

// Per cell: MatrixInv failures that the pruning test keeps somewhere in the image, and
// near-plane straddlers (counts[2c], counts[2c + 1]).  Runs of consecutive cells with
// the same pose variables share a launch of up to kClassifyCells cells.
int classify_cells(const ar_scene *sc, const Params &prm_in, const ar_pose_box *cells, int ncells, int64_t *counts,
                   hipStream_t s) {
  Params prm = prm_in;
  const int cap = std::min(ncells, kClassifyCells);
  std::vector<PoseForms> pf((size_t)cap);
  std::vector<unsigned long long> host((size_t)2 * cap);
  DeviceBuffer dpose, dcount;
  HIP_TRY(hipMalloc(&dpose.p, (size_t)cap * sizeof(PoseForms)));
  HIP_TRY(hipMalloc(&dcount.p, (size_t)2 * cap * sizeof(unsigned long long)));
  PoseForms *pd = static_cast<PoseForms *>(dpose.p);
  unsigned long long *cd = static_cast<unsigned long long *>(dcount.p);
  int i = 0;
  while (i < ncells) {
    bool rot = false;
    int P = 0;
    int rc = render_vars(sc, &cells[i], &rot, &P);
    if (rc) return rc;
    prm.pose_vars = P - sc->dev.nvar;
    int j = i + 1;
    while (j < ncells && j - i < cap) {
      bool r2 = false;
      int P2 = 0;
      if (render_vars(sc, &cells[j], &r2, &P2) || P2 != P) break;
      ++j;
    }
    const int m = j - i;
    for (int c = 0; c < m; ++c)
      if (pose_forms_host(cells[i + c], P, pf[c])) return fail(AR_E_INVALID, "unsupported pose variables %d", P);
    HIP_TRY(hipMemcpyAsync(pd, pf.data(), (size_t)m * sizeof(PoseForms), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_zero_u64_n, dim3((unsigned)((2 * m + 255) / 256)), dim3(256), 0, s, cd, (size_t)2 * m);
    HIP_TRY(hipGetLastError());
    HIP_TRY(launch_classify(P, sc->dev, pd, m, prm, cd, s));
    HIP_TRY(hipMemcpyAsync(host.data(), cd, (size_t)2 * m * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int c = 0; c < 2 * m; ++c) counts[2 * (size_t)i + c] = (int64_t)host[c];
    i = j;
  }
  return AR_OK;
}

// Per cell, the (list entry, list position) pairs of its tile lists whose Ind is undecided
// (Ind = 2; both orders of a pair count): the rotation path up to the Ind counting pass,
// in launches of cells with the same pose variables.  Boxes whose depth order cannot
// change (translation only, plain scenes) have none.
int count_ind_cells(const ar_scene *sc, const Params &prm_in, const ar_pose_box *cells, int ncells,
                    const ar_options *opts, int64_t *counts, hipStream_t s) {
  Workspace &ws = const_cast<ar_scene *>(sc)->ws;
  std::vector<unsigned long long> host;
  int i = 0;
  while (i < ncells) {
    bool rot = false;
    int P = 0;
    int rc = render_vars(sc, &cells[i], &rot, &P);
    if (rc) return rc;
    int j = i + 1;
    while (j < ncells) {
      bool r2 = false;
      int P2 = 0;
      if (render_vars(sc, &cells[j], &r2, &P2) || P2 != P || r2 != rot) break;
      ++j;
    }
    if (!rot) {
      for (int c = i; c < j; ++c) counts[c] = 0;
      i = j;
      continue;
    }
    while (i < j) {
      const int m = std::min(j - i, batch_cells(sc, ws, prm_in, P, rot, opts));
      if ((size_t)m > ws.cap_ind_und || !ws.ind_und) {
        HIP_TRY(grow(ws, ws.ind_und, (size_t)m));
        ws.cap_ind_und = (size_t)m;
      }
      hipLaunchKernelGGL(k_zero_u64_n, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, ws.ind_und, (size_t)m);
      HIP_TRY(hipGetLastError());
      Params prm = prm_in;
      prm.ind_und = ws.ind_und;
      prm.ind_only = 1;
      rc = render_cells(sc, ws, prm, cells + i, m, P, rot, nullptr, nullptr, s, nullptr);
      if (rc) return rc;
      host.resize((size_t)m);
      HIP_TRY(hipMemcpyAsync(host.data(), ws.ind_und, (size_t)m * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             s));
      HIP_TRY(hipStreamSynchronize(s));
      for (int c = 0; c < m; ++c) counts[i + c] = (int64_t)host[c];
      i += m;
    }
  }
  return AR_OK;
}

static int validate_scene_host(const ar_scene_desc *d, const float *mean, const float *cov, const float *op,
                               const float *rgb) {
  const size_t n = (size_t)d->n;
  for (size_t i = 0; i < 3 * n; ++i)
    if (!isfinite(mean[i])) return fail(AR_E_INVALID, "non-finite mean at index %zu", i);
  for (size_t i = 0; i < 9 * n; ++i)
    if (!isfinite(cov[i])) return fail(AR_E_INVALID, "non-finite covariance factor at index %zu", i);
  for (size_t i = 0; i < n; ++i)
    if (!(op[i] > 0.0f && op[i] <= 1.0f)) return fail(AR_E_INVALID, "opacity %g at %zu outside (0, 1]", op[i], i);
  for (size_t i = 0; i < 3 * n; ++i)
    if (!(rgb[i] >= 0.0f && rgb[i] <= 1.0f)) return fail(AR_E_INVALID, "colour %g at %zu outside [0, 1]", rgb[i], i);
  return AR_OK;
}

static int validate_set_host(size_t n, const ar_scene_set *st, const float *op, const float *rgb, const float *olo,
                             const float *rhi, const int32_t *mvar, const float *mdir) {
  if (st->nvar < 0 || st->nvar > ar::kMaxP) return fail(AR_E_INVALID, "scene set has %d variables (0..6)", st->nvar);
  for (int v = 0; v < st->nvar; ++v)
    if (!isfinite(st->lo[v]) || !isfinite(st->hi[v]) || st->lo[v] > st->hi[v])
      return fail(AR_E_INVALID, "scene variable %d has a bad range", v);
  if (st->nvar > 0 && (!mvar || !mdir)) return fail(AR_E_INVALID, "scene variables need mean_var and mean_dir");
  if (mvar)
    for (size_t i = 0; i < n; ++i)
      if (mvar[i] < -1 || mvar[i] >= st->nvar) return fail(AR_E_INVALID, "mean_var %d at %zu out of range", mvar[i], i);
  if (mdir)
    for (size_t i = 0; i < 3 * n; ++i)
      if (!isfinite(mdir[i])) return fail(AR_E_INVALID, "non-finite mean_dir at index %zu", i);
  if (olo)
    for (size_t i = 0; i < n; ++i)
      if (!(olo[i] >= 0.0f && olo[i] <= op[i])) return fail(AR_E_INVALID, "opacity_lo %g at %zu outside [0, opacity]", olo[i], i);
  if (rhi)
    for (size_t i = 0; i < 3 * n; ++i)
      if (!(rhi[i] >= rgb[i] && rhi[i] <= 1.0f)) return fail(AR_E_INVALID, "rgb_hi %g at %zu outside [rgb, 1]", rhi[i], i);
  return AR_OK;
}

// host copy of n elements of T from host or device memory (the validation reads it)
template <typename T>
static int host_view(const T *p, size_t n, bool on_device, hipStream_t s, std::vector<T> &buf, const T *&out) {
  out = p;
  if (!p || !on_device) return AR_OK;
  buf.resize(n);
  HIP_TRY(hipMemcpyAsync(buf.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out = buf.data();
  return AR_OK;
}

// Covariance factors Mw = R(q) diag(s) from quaternions (w, x, y, z; normalised) and
// scales, in FP64, rounded to float32, in the layout of ar_scene_desc.cov_factor.
static int cov_from_quat_scale(const ar_scene_desc *d, bool dev, hipStream_t s, std::vector<float> &out,
                               const float *&cov) {
  const size_t n = (size_t)d->n;
  std::vector<float> hq, hs;
  const float *q = nullptr, *sc = nullptr;
  int rc = host_view(d->quat, 4 * n, dev, s, hq, q);
  if (!rc) rc = host_view(d->scale, 3 * n, dev, s, hs, sc);
  if (rc) return rc;
  out.resize(9 * n);
  for (size_t i = 0; i < n; ++i) {
    double w = q[i], x = q[n + i], y = q[2 * n + i], z = q[3 * n + i];
    const double len = sqrt(w * w + x * x + y * y + z * z);
    if (!isfinite(len) || !(len > 0.0)) return fail(AR_E_INVALID, "quaternion %zu is zero or not finite", i);
    w /= len;
    x /= len;
    y /= len;
    z /= len;
    const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    for (int c = 0; c < 3; ++c) {
      const double sv = sc[c * n + i];
      if (!isfinite(sv) || sv < 0.0) return fail(AR_E_INVALID, "scale %g at %zu is negative or not finite", sv, i);
      for (int r = 0; r < 3; ++r) out[(3 * r + c) * n + i] = (float)(R[r][c] * sv);
    }
  }
  cov = out.data();
  return AR_OK;
}

// A scene handle for a scene (set == NULL) or a set of scenes.  Device layout, one
// allocation: mean 3n, cov 9n, opacity n, rgb 3n, opacity_lo n, rgb_hi 3n, ind_mean 3n,
// mean_dir 3n floats, then mean_var n int32.
int create_scene(const ar_scene_desc *desc, const ar_scene_set *set, void *hip_stream, ar_scene **out) {
  if (!out) return fail(AR_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(AR_E_INVALID, "scene description is NULL");
  if (desc->n < 1) return fail(AR_E_INVALID, "scene has n = %d Gaussians", desc->n);
  if (!desc->mean || !desc->opacity || !desc->rgb || (!desc->cov_factor && (!desc->quat || !desc->scale)))
    return fail(AR_E_INVALID, "scene array is NULL");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t n = (size_t)desc->n;
  std::vector<float> hm, hc, ho, hr, hol, hrh, hmd;
  std::vector<int32_t> hmv;
  const float *mean, *cov, *op, *rgb, *olo = nullptr, *rhi = nullptr, *mdir = nullptr;
  const int32_t *mvar = nullptr;
  const bool dev = desc->on_device != 0;
  int rc = host_view(desc->mean, 3 * n, dev, s, hm, mean);
  if (!rc && desc->cov_factor) rc = host_view(desc->cov_factor, 9 * n, dev, s, hc, cov);
  if (!rc && !desc->cov_factor) rc = cov_from_quat_scale(desc, dev, s, hc, cov);
  if (!rc) rc = host_view(desc->opacity, n, dev, s, ho, op);
  if (!rc) rc = host_view(desc->rgb, 3 * n, dev, s, hr, rgb);
  if (rc) return rc;
  rc = validate_scene_host(desc, mean, cov, op, rgb);
  if (rc) return rc;
  ar_scene_set none{};
  if (!set) set = &none;
  const bool sdev = set->on_device != 0;
  rc = host_view(set->opacity_lo, n, sdev, s, hol, olo);
  if (!rc) rc = host_view(set->rgb_hi, 3 * n, sdev, s, hrh, rhi);
  if (!rc) rc = host_view(set->mean_dir, 3 * n, sdev, s, hmd, mdir);
  if (!rc) rc = host_view(set->mean_var, n, sdev, s, hmv, mvar);
  if (rc) return rc;
  rc = validate_set_host(n, set, op, rgb, olo, rhi, mvar, mdir);
  if (rc) return rc;
  // the arrays the kernels read, on the host
  std::vector<float> img(26 * n);
  std::copy(mean, mean + 3 * n, img.begin());
  std::copy(cov, cov + 9 * n, img.begin() + 3 * n);
  std::copy(op, op + n, img.begin() + 12 * n);
  std::copy(rgb, rgb + 3 * n, img.begin() + 13 * n);
  std::copy(olo ? olo : op, (olo ? olo : op) + n, img.begin() + 16 * n);
  std::copy(rhi ? rhi : rgb, (rhi ? rhi : rgb) + 3 * n, img.begin() + 17 * n);
  bool moving = false;
  for (size_t i = 0; i < 3 * n; ++i) {
    const bool mv = set->nvar > 0 && mvar[i % n] >= 0;
    moving = moving || mv;
    img[20 * n + i] = mv ? NAN : mean[i];
    img[23 * n + i] = mdir ? mdir[i] : 0.0f;
  }
  ar_scene *sc = new ar_scene();
  float *base = nullptr;
  hipError_t e = hipMalloc((void **)&base, 27 * n * sizeof(float));
  if (e != hipSuccess) {
    delete sc;
    return fail(e == hipErrorOutOfMemory ? AR_E_OOM : AR_E_DEVICE, "scene allocation failed: %s", hipGetErrorString(e));
  }
  sc->base = base;
  ar::SceneDev &d = sc->dev;
  d.n = desc->n;
  d.mean = base;
  d.cov = base + 3 * n;
  d.opac = base + 12 * n;
  d.rgb = base + 13 * n;
  d.opac_lo = base + 16 * n;
  d.rgb_hi = base + 17 * n;
  d.ind_mean = moving ? base + 20 * n : base;
  d.mean_dir = base + 23 * n;
  d.mean_var = set->nvar > 0 ? reinterpret_cast<int32_t *>(base + 26 * n) : nullptr;
  d.nvar = set->nvar;
  d.moving = moving ? 1 : 0;
  for (int v = 0; v < ar::kMaxP; ++v) {
    d.s_mid[v] = v < set->nvar ? 0.5 * (set->lo[v] + set->hi[v]) : 0.0;
    d.s_rad[v] = v < set->nvar ? 0.5 * (set->hi[v] - set->lo[v]) : 0.0;
  }
  e = hipMemcpyAsync(base, img.data(), 26 * n * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && d.mean_var) e = hipMemcpyAsync(d.mean_var, mvar, n * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    ar_scene_destroy(sc);
    return fail(AR_E_DEVICE, "scene upload failed: %s", hipGetErrorString(e));
  }
  *out = sc;
  return AR_OK;
}

}  // namespace ar

extern "C" {

const char *ar_last_error(void) { return ar::g_error.c_str(); }

const char *ar_version(void) { return "abstract-render-gfx950 0.1"; }

int32_t ar_scene_size(const ar_scene *scene) { return scene ? scene->dev.n : 0; }

int ar_scene_create(const ar_scene_desc *desc, void *hip_stream, ar_scene **out) {
  return ar::create_scene(desc, nullptr, hip_stream, out);
}

int ar_scene_create_set(const ar_scene_desc *desc, const ar_scene_set *set, void *hip_stream, ar_scene **out) {
  if (!set) return fail(AR_E_INVALID, "scene set is NULL");
  return ar::create_scene(desc, set, hip_stream, out);
}

void ar_scene_destroy(ar_scene *sc) {
  if (!sc) return;
  ar::release_workspace(sc->ws);
  if (sc->base) (void)hipFree(sc->base);
  delete sc;
}


int ar_render_bounds(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *box,
                     const ar_options *opts, float *lo_rgb, float *hi_rgb, void *hip_stream, ar_stats *stats) {
  if (!scene) return fail(AR_E_INVALID, "scene is NULL");
  int rc = ar::validate_box(box);
  if (rc) return rc;
  ar::Params prm{};
  rc = ar::make_params(scene, intr, opts, prm);
  if (rc) return rc;
  bool host = false;
  rc = ar::check_outputs_any(lo_rgb, hi_rgb, &host);
  if (rc) return rc;
  if (stats) memset(stats, 0, sizeof(*stats));
  bool rot = false;
  int P = 0;
  rc = ar::render_vars(scene, box, &rot, &P);
  if (rc) return rc;
  return ar::render_cells_out(scene, const_cast<ar_scene *>(scene)->ws, prm, box, 1, P, rot, lo_rgb, hi_rgb, host,
                              (hipStream_t)hip_stream, stats);
}

int ar_render_batch(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *cells, int32_t ncells,
                    const ar_options *opts, float *lo_rgb, float *hi_rgb, void *hip_stream, ar_stats *stats) {
  if (!scene) return fail(AR_E_INVALID, "scene is NULL");
  if (!cells || ncells < 1) return fail(AR_E_INVALID, "batch needs at least one cell");
  for (int i = 0; i < ncells; ++i) {
    int rc = ar::validate_box(&cells[i]);
    if (rc) return rc;
  }
  ar::Params prm{};
  int rc = ar::make_params(scene, intr, opts, prm);
  if (rc) return rc;
  bool host = false;
  rc = ar::check_outputs_any(lo_rgb, hi_rgb, &host);
  if (rc) return rc;
  if (stats) memset(stats, 0, sizeof(*stats));
  const size_t img = (size_t)intr->width * intr->height * 3;
  // runs of consecutive cells with the same pose variables, in launches of at most
  // cells_per_launch cells (memory-bounded; see batch_cells)
  int i = 0;
  while (i < ncells) {
    bool rot = false;
    int P = 0;
    rc = ar::render_vars(scene, &cells[i], &rot, &P);
    if (rc) return rc;
    int j = i + 1;
    while (j < ncells) {
      bool r2 = false;
      int P2 = 0;
      if (ar::render_vars(scene, &cells[j], &r2, &P2) || P2 != P || r2 != rot) break;
      ++j;
    }
    while (i < j) {
      ar::Workspace &ws = const_cast<ar_scene *>(scene)->ws;
      const int m = std::min(j - i, ar::batch_cells(scene, ws, prm, P, rot, opts));
      rc = ar::render_cells_out(scene, ws, prm, cells + i, m, P, rot, lo_rgb + i * img, hi_rgb + i * img, host,
                                (hipStream_t)hip_stream, stats);
      if (rc) return rc;
      i += m;
    }
  }
  return AR_OK;
}

int ar_render_batch_scenes(const ar_scene *const *scenes, const ar_intrinsics *intr, const ar_pose_box *cells,
                           int32_t ncells, const ar_options *opts, float *lo_rgb, float *hi_rgb, void *hip_stream,
                           ar_stats *stats) {
  if (!scenes) return fail(AR_E_INVALID, "scenes is NULL");
  if (!cells || ncells < 1) return fail(AR_E_INVALID, "batch needs at least one cell");
  bool one = true;
  for (int i = 0; i < ncells; ++i) {
    if (!scenes[i]) return fail(AR_E_INVALID, "scene of cell %d is NULL", i);
    one = one && scenes[i] == scenes[0];
  }
  if (one) return ar_render_batch(scenes[0], intr, cells, ncells, opts, lo_rgb, hi_rgb, hip_stream, stats);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  for (int i = 0; i < ncells; ++i) {
    int rc = ar::validate_box(&cells[i]);
    if (rc) return rc;
    if (scenes[i]->dev.nvar > 0)
      return fail(AR_E_UNSUPPORTED, "cell %d: a set of scenes (scene variables) renders only with cells of its own", i);
    hipPointerAttribute_t at{};
    HIP_TRY(hipPointerGetAttributes(&at, scenes[i]->base));
    if (at.device != dev) return fail(AR_E_INVALID, "scene of cell %d is on device %d, not the current %d", i, at.device, dev);
  }
  ar::Params prm{};
  int rc = ar::make_params(scenes[0], intr, opts, prm);
  if (rc) return rc;
  bool host = false;
  rc = ar::check_outputs_any(lo_rgb, hi_rgb, &host);
  if (rc) return rc;
  if (stats) memset(stats, 0, sizeof(*stats));
  const size_t img = (size_t)intr->width * intr->height * 3;
  ar::Workspace &ws = const_cast<ar_scene *>(scenes[0])->ws;
  // runs of consecutive cells with the same pose variables, in launches sized as
  // ar_render_batch's for the largest scene of the run
  int i = 0;
  while (i < ncells) {
    bool rot = false;
    int P = 0;
    rc = ar::render_vars(scenes[i], &cells[i], &rot, &P);
    if (rc) return rc;
    int j = i + 1;
    const ar_scene *big = scenes[i];
    while (j < ncells) {
      bool r2 = false;
      int P2 = 0;
      if (ar::render_vars(scenes[j], &cells[j], &r2, &P2) || P2 != P || r2 != rot) break;
      if (scenes[j]->dev.n > big->dev.n) big = scenes[j];
      ++j;
    }
    while (i < j) {
      const int m = std::min(j - i, ar::batch_cells(big, ws, prm, P, rot, opts));
      rc = ar::render_cells_out(scenes[i], ws, prm, cells + i, m, P, rot, lo_rgb + i * img, hi_rgb + i * img, host,
                                (hipStream_t)hip_stream, stats, scenes + i);
      if (rc) return rc;
      i += m;
    }
  }
  return AR_OK;
}

int ar_render_partitioned(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *box,
                          const int32_t *splits, const ar_options *opts, float *lo_rgb, float *hi_rgb,
                          void *hip_stream, ar_stats *stats) {
  if (!scene) return fail(AR_E_INVALID, "scene is NULL");
  int rc = ar::validate_box(box);
  if (rc) return rc;
  if (!splits) return fail(AR_E_INVALID, "splits is NULL");
  if (!intr || intr->width < 1 || intr->height < 1) return fail(AR_E_INVALID, "bad intrinsics");
  rc = ar::check_outputs(lo_rgb, hi_rgb);
  if (rc) return rc;
  const int na = box->model == AR_POSE_ORBIT ? 1 : 6;
  int s[6] = {1, 1, 1, 1, 1, 1};
  size_t ncells = 1;
  for (int a = 0; a < na; ++a) {
    if (splits[a] < 1 || splits[a] > 65536) return fail(AR_E_INVALID, "splits[%d] = %d outside [1, 65536]", a, splits[a]);
    s[a] = box->hi[a] > box->lo[a] ? splits[a] : 1;
    ncells *= (size_t)s[a];
    if (ncells > 65536) return fail(AR_E_INVALID, "more than 65536 cells");
  }
  // the grid of cells; adjacent cells share the computed cut exactly, the last ends at hi
  std::vector<ar_pose_box> cells(ncells, *box);
  for (size_t c = 0; c < ncells; ++c) {
    size_t r = c;
    for (int a = 0; a < na; ++a) {
      const int k = (int)(r % (size_t)s[a]);
      r /= (size_t)s[a];
      if (s[a] == 1) continue;
      const double lo = box->lo[a], w = box->hi[a] - box->lo[a];
      cells[c].lo[a] = lo + w * k / s[a];
      cells[c].hi[a] = k + 1 == s[a] ? box->hi[a] : lo + w * (k + 1) / s[a];
    }
  }
  return ar::render_union(scene, intr, cells.data(), ncells, opts, lo_rgb, hi_rgb, (hipStream_t)hip_stream, stats);
}

int ar_classify_cells(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *cells, int32_t ncells,
                      const ar_options *opts, int64_t *counts, void *hip_stream) {
  if (!scene) return fail(AR_E_INVALID, "scene is NULL");
  if (!cells || ncells < 1) return fail(AR_E_INVALID, "classification needs at least one cell");
  if (!counts) return fail(AR_E_INVALID, "counts is NULL");
  for (int i = 0; i < ncells; ++i) {
    int rc = ar::validate_box(&cells[i]);
    if (rc) return rc;
  }
  ar::Params prm{};
  int rc = ar::make_params(scene, intr, opts, prm);
  if (rc) return rc;
  return ar::classify_cells(scene, prm, cells, ncells, counts, (hipStream_t)hip_stream);
}

int ar_count_ind_uncertain(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *cells,
                           int32_t ncells, const ar_options *opts, int64_t *counts, void *hip_stream) {
  if (!scene) return fail(AR_E_INVALID, "scene is NULL");
  if (!cells || ncells < 1) return fail(AR_E_INVALID, "counting needs at least one cell");
  if (!counts) return fail(AR_E_INVALID, "counts is NULL");
  for (int i = 0; i < ncells; ++i) {
    int rc = ar::validate_box(&cells[i]);
    if (rc) return rc;
  }
  ar::Params prm{};
  int rc = ar::make_params(scene, intr, opts, prm);
  if (rc) return rc;
  return ar::count_ind_cells(scene, prm, cells, ncells, opts, counts, (hipStream_t)hip_stream);
}

int ar_render_refined(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *box,
                      const ar_options *opts, int32_t max_cells, int32_t criteria, float *lo_rgb, float *hi_rgb,
                      void *hip_stream, ar_pose_box *cells_out, int32_t *ncells_out, ar_stats *stats) {
  if (!scene) return fail(AR_E_INVALID, "scene is NULL");
  int rc = ar::validate_box(box);
  if (rc) return rc;
  if (max_cells < 1 || max_cells > 65536) return fail(AR_E_INVALID, "max_cells %d outside [1, 65536]", max_cells);
  if (criteria == 0) criteria = AR_REFINE_MATINV;
  if (criteria & ~(AR_REFINE_MATINV | AR_REFINE_NEAR | AR_REFINE_IND))
    return fail(AR_E_INVALID, "unknown refinement criteria %d", criteria);
  ar::Params prm{};
  rc = ar::make_params(scene, intr, opts, prm);
  if (rc) return rc;
  rc = ar::check_outputs(lo_rgb, hi_rgb);
  if (rc) return rc;
  const hipStream_t s = (hipStream_t)hip_stream;
  // active axes of the box, in order (ORBIT: its angle)
  int axes[6], naxes = 0;
  const int na = box->model == AR_POSE_ORBIT ? 1 : 6;
  for (int a = 0; a < na; ++a)
    if (box->hi[a] > box->lo[a]) axes[naxes++] = a;
  // level by level: classify the level's cells, cut the flagged ones in order while the
  // number of cells stays within max_cells (lower half first), settle the others
  std::vector<ar_pose_box> level(1, *box), next, leaves;
  std::vector<int> depth(1, 0), next_depth;
  std::vector<int64_t> counts, und;
  size_t total = 1;
  while (!level.empty()) {
    counts.assign(2 * level.size(), 0);
    rc = ar::classify_cells(scene, prm, level.data(), (int)level.size(), counts.data(), s);
    if (rc) return rc;
    und.assign(level.size(), 0);
    if (criteria & AR_REFINE_IND) {
      rc = ar::count_ind_cells(scene, prm, level.data(), (int)level.size(), opts, und.data(), s);
      if (rc) return rc;
    }
    next.clear();
    next_depth.clear();
    for (size_t i = 0; i < level.size(); ++i) {
      const bool flagged = ((criteria & AR_REFINE_MATINV) && counts[2 * i] > 0) ||
                           ((criteria & AR_REFINE_NEAR) && counts[2 * i + 1] > 0) ||
                           ((criteria & AR_REFINE_IND) && und[i] > 0);
      if (flagged && naxes > 0 && depth[i] < ar::kMaxRefineDepth && total + 1 <= (size_t)max_cells) {
        const int a = axes[depth[i] % naxes];
        const double lo = level[i].lo[a], hi = level[i].hi[a], m = 0.5 * (lo + hi);
        if (lo < m && m < hi) {
          ++total;
          next.push_back(level[i]);
          next.back().hi[a] = m;
          next.push_back(level[i]);
          next.back().lo[a] = m;
          next_depth.push_back(depth[i] + 1);
          next_depth.push_back(depth[i] + 1);
          continue;
        }
      }
      leaves.push_back(level[i]);
    }
    level.swap(next);
    depth.swap(next_depth);
  }
  rc = ar::render_union(scene, intr, leaves.data(), leaves.size(), opts, lo_rgb, hi_rgb, s, stats);
  if (rc) return rc;
  if (cells_out) std::copy(leaves.begin(), leaves.end(), cells_out);
  if (ncells_out) *ncells_out = (int32_t)leaves.size();
  return AR_OK;
}

int ar_autotune(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *cells, int32_t ncells,
                const ar_options *opts, int32_t reps, float *lo_rgb, float *hi_rgb, void *hip_stream,
                ar_options *tuned, ar_stats *stats) {
  if (!tuned) return fail(AR_E_INVALID, "tuned options are NULL");
  if (reps < 1 || reps > 16) return fail(AR_E_INVALID, "reps %d outside [1, 16]", reps);
  if (!cells || ncells < 1) return fail(AR_E_INVALID, "batch needs at least one cell");
  ar_options base{};
  if (opts) base = *opts;
  bool rot = false;
  for (int i = 0; i < ncells; ++i) {
    bool r = false;
    int P = 0;
    int rc = ar::render_vars(scene, &cells[i], &r, &P);
    if (rc) return rc;
    rot = rot || r;
  }
  // translation boxes: both binning tiles unless the options fix one; per tile the
  // automatic length first, then candidates around it (rotation boxes: 8x8 tiles and
  // 32-128 positions)
  std::vector<int> tiles;
  if (rot || base.tile != 0) tiles.push_back(base.tile);
  else tiles = {ar::kTile, ar::kTileMax};
  int best = 0, best_tile = tiles[0];
  double best_ms = 1e300;
  for (int tile : tiles) {
    ar_options o = base;
    o.tile = tile;
    o.chunk = 0;
    ar_stats st{};
    int rc = ar_render_batch(scene, intr, cells, ncells, &o, lo_rgb, hi_rgb, hip_stream, &st);
    if (rc) return rc;
    const int L0 = std::max(8, (int)st.segment_length);
    std::vector<int> cand;
    if (rot) {
      cand = {32, 48, 64, 96, 128};
    } else {
      for (int num : {2, 3, 4, 5, 6}) {
        const int L = std::min(4096, std::max(8, (L0 * num / 4 + 7) / 8 * 8));
        if (std::find(cand.begin(), cand.end(), L) == cand.end()) cand.push_back(L);
      }
    }
    for (int L : cand) {
      o.chunk = L;
      double t = 1e300;
      for (int r = 0; r < reps; ++r) {
        ar_stats s1{};
        rc = ar_render_batch(scene, intr, cells, ncells, &o, lo_rgb, hi_rgb, hip_stream, &s1);
        if (rc) return rc;
        t = std::min(t, s1.total_ms);
      }
      if (t < best_ms) {
        best_ms = t;
        best = L;
        best_tile = tile;
      }
    }
  }
  int rc = AR_OK;
  *tuned = base;
  tuned->tile = best_tile;
  tuned->chunk = best;
  // cells per launch, for a batch: the automatic count (what fits the memory budget at the
  // density just measured) and fractions of it, by wall time (the launches' host
  // synchronisations count); a count is never above the automatic one
  if (ncells > 1 && base.cells_per_launch <= 0) {
    ar::Params prm{};
    rc = ar::make_params(scene, intr, tuned, prm);
    if (rc) return rc;
    int P = 0;
    rc = ar::render_vars(scene, &cells[0], &rot, &P);
    if (rc) return rc;
    const int automatic =
        std::min(ncells, ar::batch_cells(scene, const_cast<ar_scene *>(scene)->ws, prm, P, rot, nullptr));
    std::vector<int> cpl = {0};
    for (int c : {automatic / 2, automatic / 4, 16, 8})
      if (c >= 1 && c < automatic && std::find(cpl.begin(), cpl.end(), c) == cpl.end()) cpl.push_back(c);
    int best_c = 0;
    double best_t = 1e300;
    for (int c : cpl) {
      ar_options o = *tuned;
      o.cells_per_launch = c;
      double t = 1e300;
      for (int r = 0; r < reps; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        rc = ar_render_batch(scene, intr, cells, ncells, &o, lo_rgb, hi_rgb, hip_stream, nullptr);
        if (rc) return rc;
        t = std::min(t, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
      }
      if (t < best_t) {
        best_t = t;
        best_c = c;
      }
    }
    tuned->cells_per_launch = best_c;
  }
  return ar_render_batch(scene, intr, cells, ncells, tuned, lo_rgb, hi_rgb, hip_stream, stats);
}

}  // extern "C"
