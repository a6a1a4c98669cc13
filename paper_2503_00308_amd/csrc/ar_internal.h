// Internal declarations shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <unordered_map>

#include "../../include/ar.h"

#define HIP_RET(expr)                       \
  do {                                      \
    const hipError_t e_ = (expr);           \
    if (e_ != hipSuccess) return e_;        \
  } while (0)

namespace ar {

constexpr int kMaxP = 6;        // pose variables: 3 translations + 3 angles
constexpr int kOverflow = 15;   // statistics counter set when a planned launch outgrows a buffer
constexpr int kIndBorder = 10;  // statistics counter of Ind tests decided within rounding of a threshold
constexpr int kTile = 8;        // pixel side of the block one 64-lane wave covers (a tile, or a
                                // quarter of a 16x16 binning tile on the translation path)
constexpr int kTilePix = kTile * kTile;
constexpr int kTileMax = 16;    // largest binning tile side
constexpr int kListBox = 13;   // per tile list: box of the means, box of their parts across m, max |mean|

// Gaussian categories decided in the per-Gaussian stage.
enum GaussType : int32_t {
  kNormal = 0,    // full relational alpha bounds
  kFallback = 1,  // MatrixInv assertion failed: alpha in [0, footprint bound]
  kWild = 2,      // straddles the near plane (or unbounded footprint): alpha in [0, o]
  kDropped = 3    // behind the near plane at every pose: never contributes
};

// Per-Gaussian FP64 record consumed by the pixel loops (offsets in doubles).
// Every pair of linear forms (lower l(e), upper h(e)) is stored in mid-radius form
// m = (l + h) / 2, r = (h - l) / 2, so that l = m - r and h = m + r coefficient-wise:
// scaling by a number a of either sign is then a m, |a| r with no per-lane choice of
// which form to take.  Conversion rounding is absorbed into the constant of r.
// The header holds the float32 pruning data (mean box, r^2, type) read first.
template <int P>
struct Rec {
  static constexpr int F = P + 1;
  // header (16 doubles)
  static constexpr int PRUNE = 0;            // float[0..3] mean box, float[4] r^2, int32[5] type
  static constexpr int O = 3, LAM = 4;       // opacity (upper bound), footprint eigenvalue bound
  static constexpr int C = 5;                // colour: float[0..3) lower, float[3..6) upper bounds
  static constexpr int OLO = 15;             // opacity lower bound
  static constexpr int MD2 = 8;              // sum_j |dm_j| + |dr_j|
  static constexpr int MDUP = 9;             // (2) the same for d*up_k
  static constexpr int MBB = 11;             // (2) max_n sum_j (|Bm| + |Br|) + 2 BMAX, for B_kn
  static constexpr int BMAX = 13;            // (2) max_n max(|ylo|, |yhi|) of B_kn
  static constexpr int HDR = 16;
  static constexpr int DM = HDR, DR = HDR + F;   // d^2
  static constexpr int PM = HDR + 2 * F;         // d*up_k, [2][F]
  static constexpr int PR = HDR + 4 * F;         // [2][F]
  static constexpr int BM = HDR + 6 * F;         // B = Conic*Mp, entry e = 3k+n, [6][F]
  static constexpr int BR = HDR + 12 * F;        // [6][F]
  static constexpr int CM = HDR + 18 * F;        // McCormick weights of B_e: [6][4]
  static constexpr int STRIDE = ((CM + 24) + 7) / 8 * 8;
};

inline int rec_stride(int P) {
  return ((16 + 18 * (P + 1) + 24) + 7) / 8 * 8;
}

// Squared distance from the mean box to the rectangle [ux0, ux1] x [uy0, uy1] (float32,
// no contraction): the per-pixel pruning test evaluated at the nearest point.
__device__ __forceinline__ float dist2_rect(const float *mu, float ux0, float ux1, float uy0, float uy1) {
#pragma clang fp contract(off)
  const float dx = fmaxf(fmaxf(mu[0] - ux1, 0.0f), ux0 - mu[1]);
  const float dy = fmaxf(fmaxf(mu[2] - uy1, 0.0f), uy0 - mu[3]);
  return dx * dx + dy * dy;
}

template <int P>
__device__ __forceinline__ const float *rec_prune(const double *rec) {
  return reinterpret_cast<const float *>(rec + Rec<P>::PRUNE);
}

template <int P>
__device__ __forceinline__ int rec_type(const double *rec) {
  return reinterpret_cast<const int32_t *>(rec + Rec<P>::PRUNE)[5];
}

// Pose set as linear forms over e in [-1,1]^P (FP64): uc = A (uw - tau) + beta.
struct PoseForms {
  int32_t P;
  int32_t pad;
  double A[9][2][kMaxP + 1];
  double tau[3][2][kMaxP + 1];
  double beta[3][2][kMaxP + 1];
  double Zm[3][kMaxP + 1], Zr[3][kMaxP + 1];   // depth row of A in mid-radius form (Ind tests)
  // per l, above |Zr[l][kMaxP]| + sum_k (|Zm[l][k]| + |Zr[l][k]|) by 2^-46 of itself
  // plus |Zm[l][kMaxP]| (the quick test of an Ind pair)
  double Zq[3];
};

struct Params {
  int32_t width, height;
  double fx, fy, cx, cy;
  int32_t taylor_k;
  double z_near;
  double cull_budget;  // cull budget per pixel
  double eps_cull;     // cull_budget / n
  double E;            // widening for pruning
  double t_min;
  int32_t tile;        // binning tile side in pixels: 8, or 16 (translation boxes: four waves per tile)
  int32_t ntx, nty;    // tiles
  int32_t ind_window, chunk;
  int32_t prefix_entries;   // rotation path: list entries per pixel-loop launch
  int32_t nominal_order;    // rotation path: order lists by the nominal depth (else by the upper bound)
  int32_t abs_sums, ind_copy, ind_masks;   // rotation path layouts: 0 automatic, 1 on, 2 off
  int32_t group_entries;    // rotation path: list entries per group of the Ind passes (0: default)
  int32_t inverse;          // conic: 0 MatrixInv (forward), 1 MatrixInv bounded backward, 2 adjugate
  int32_t pose_vars;        // pose variables; scene variables follow them in the forms
  int32_t group_runs;       // rotation path: most Ind runs per list group (0: the uint32 limit)
  int32_t ind_quick;        // rotation path: quick Ind test (0, 1 on; 2 off)
  // rotation path: per cell of the launch, the number of (list entry, list position) pairs
  // whose Ind is undecided, added here by the counting pass when not null; with ind_only
  // the render stops after that pass (no images)
  unsigned long long *ind_und;
  int32_t ind_only;
};

// The quick Ind test switched off for a cell: an infinite Zq never decides.
inline void ind_quick_off(PoseForms &pf) { pf.Zq[0] = pf.Zq[1] = pf.Zq[2] = __builtin_inf(); }

// Waves per binning tile: each covers one kTile x kTile block of it (row-major).
__host__ __device__ inline int tile_subs(const Params &p) {
  const int k = p.tile / kTile;
  return k * k;
}

// A scene, or a set of scenes (Sec. 4.6): colour and opacity intervals per Gaussian,
// means moved along a direction by scene variables s_v in [s_mid - s_rad, s_mid + s_rad].
struct SceneDev {
  int32_t n;
  float *mean;      // [3][n]
  float *cov;       // [9][n]
  float *opac;      // [n] opacity (the upper bound in a set)
  float *rgb;       // [3][n] colour (the lower bound in a set)
  float *opac_lo;   // [n] opacity lower bound (= opac for a plain scene)
  float *rgb_hi;    // [3][n] colour upper bound (= rgb for a plain scene)
  float *ind_mean;  // [3][n] means read by the Ind tests: mean, NaN for a moved Gaussian
  int32_t *mean_var;  // [n] variable moving the mean (-1: none); null without scene variables
  float *mean_dir;  // [3][n] its direction
  int32_t nvar;     // scene variables (after the pose variables in the forms)
  int32_t moving;   // some mean moves
  double s_mid[kMaxP], s_rad[kMaxP];
};

// A pose cell's scene in a launch whose cells render different scenes: the cell's
// Gaussians are the items [off, off + sc.n) of the launch (local Gaussian g at item
// off + g), and eps_cull is its scene's cull threshold (the budget over its size).  A
// launch of one scene has no table: cell c's items start at c * n.
struct CellScene {
  SceneDev sc;
  uint64_t off;
  double eps_cull;
};

// The scene of cell c, and the first item of cell c (tab: the launch's table, or null).
__host__ __device__ inline const SceneDev &cell_scene(const SceneDev &sc, const CellScene *tab, int c) {
  return tab ? tab[c].sc : sc;
}
__host__ __device__ inline size_t cell_first(const SceneDev &sc, const CellScene *tab, int c) {
  return tab ? (size_t)tab[c].off : (size_t)c * (size_t)sc.n;
}
// Cell of item i: i / n in a launch of one scene, else the last c with item_off[c] <= i
// (item_off[0 .. ncells]: the cells' first items, then the total).
__host__ __device__ inline int item_cell(const uint32_t *item_off, int ncells, int n, uint32_t i) {
  if (!item_off) return (int)(i / (uint32_t)n);
  int lo = 0, hi = ncells - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (item_off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// List density of a launch, used to estimate the workspace of the next one on the same
// scene: list entries per Gaussian item and, on the rotation path, Ind runs and stored
// mask words per list entry and whether the compact copy was used (largest over groups).
struct Density {
  double pairs_per_item = 0.0;
  double runs_per_entry = 0.0;
  double mask_words_per_entry = 0.0;
  bool compact = false;
};

// Sizes of the last launch of cells (render_cells), from which a planned launch takes
// its capacities: list entries, segments of the pixel loop, Ind runs, the segment length,
// list groups, and the rotation path's layout choices.
struct LaunchSizes {
  uint64_t entries = 0, segments = 0, runs = 0;
  int L = 0, groups = 0;
  bool compact = false, absolute = false;
};

// Capacities of a planned launch (render_cells_planned): every count is kept on the
// device and checked against these; the segment length and layouts are fixed.
struct PlanCaps {
  uint32_t entries = 0, segments = 0, runs = 0;
  int L = 0;
  bool compact = false, absolute = false;
};

// Device workspace (grown on demand, owned by a scene handle).
struct Workspace {
  LaunchSizes last;              // sizes of the last launch
  size_t cap_n = 0, cap_pairs = 0, cap_tiles = 0, cap_scratch = 0, cap_rec = 0, cap_cells = 0;
  size_t bytes = 0;                              // device bytes held by the buffers below
  std::unordered_map<void *, size_t> sizes;      // allocation -> bytes
  Density density;               // of the last launch
  PoseForms *pose_dev = nullptr;   // [cells] pose forms of a launch
  PoseForms *pose_host = nullptr;  // [cells] pinned staging
  // launches whose cells render different scenes: the cells' table and their first items
  // ([cells + 1], the total last) in device memory, set for the duration of such a launch
  // (null otherwise), with their pinned staging and capacity
  CellScene *tab = nullptr;
  uint32_t *tab_off = nullptr;
  int tab_cells = 0;
  double *cbox = nullptr;    // rotation path: boxes of the kChunk-position chunks (Ind windows)
  size_t cap_cbox = 0;
  CellScene *tab_dev = nullptr, *tab_host = nullptr;
  uint32_t *tab_off_dev = nullptr, *tab_off_host = nullptr;
  size_t cap_tab = 0;
  double *rec = nullptr;       // [n][stride]
  uint64_t *key = nullptr;     // [n] depth key (by gid, kept for tie tests)
  uint64_t *key_sort = nullptr;  // [n] copy of the keys, sorted in place
  uint64_t *key_alt = nullptr; // [n]
  uint32_t *perm = nullptr;    // [n] rank -> gid
  uint32_t *perm_alt = nullptr;
  uint32_t *cell_key = nullptr, *cell_key_alt = nullptr;  // [items] cell of an item (stable cell pass)
  int32_t *rect = nullptr;     // [n][4] tile rectangle
  double *dform = nullptr;     // [n][2][kMaxP+1] depth forms (FP64, by gid)
  uint32_t *count = nullptr;   // [n+1] tiles per Gaussian (rank order), then offsets
  uint32_t *pair_key = nullptr, *pair_key_alt = nullptr;  // [pairs] tile id
  uint32_t *pair_val = nullptr, *pair_val_alt = nullptr;  // [pairs] gid
  uint32_t *tile_range = nullptr;  // [tiles][2]
  uint32_t *hist = nullptr;    // radix histograms
  size_t cap_hist = 0;
  uint32_t *scan_tmp = nullptr;
  size_t cap_scan = 0;
  unsigned long long *counters = nullptr;  // [8] stats
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // call start, pixel kernel start / end, call end
  unsigned long long *host_counters = nullptr;  // pinned
  // translation path: segments of the tile lists and their partial results
  uint32_t *seg_off = nullptr;   // [tiles + 1] first segment of each tile, then the total
  uint32_t *seg_tile = nullptr;  // [segments] tile of each segment
  size_t cap_seg = 0, cap_seg_off = 0;
  double *part = nullptr;        // [segments][fields][64]
  size_t cap_part = 0;           // doubles
  // general (rotation) path
  double *dint = nullptr;      // [n][2] (nominal depth, upper depth bound) by item
  double *lbox = nullptr;      // [lists][kListBox] bounding boxes of a list's means (see k_list_box)
  uint32_t *run_cnt = nullptr; // [pairs][2] + 1: Def / May run counts, then offsets
  size_t cap_run_cnt = 0;
  uint32_t *runs = nullptr;    // [runs][2] list-position ranges [start, end)
  size_t cap_runs = 0;
  uint32_t *win = nullptr;     // [pairs][2] Ind window [ps, qe) of each list position
  uint32_t *woff = nullptr;    // [pairs + 1] mask words of each long window, then offsets
  size_t cap_win = 0;
  unsigned long long *masks = nullptr;   // Ind masks of the long windows (two words per 64 positions)
  size_t cap_masks = 0;
  float *cmean = nullptr;      // [pairs][4] means by list position (compact copy for the Ind tests)
  double *cform = nullptr;     // [pairs][2][P + 1] depth forms by list position
  size_t cap_compact = 0;      // doubles of cform
  size_t cap_cmean = 0;        // positions of cmean
  float *union_img = nullptr;  // cell images of a partitioned render (lower, then upper)
  size_t cap_union = 0;
  double *pre = nullptr;       // two planes [pairs][64]: running sums of log(1 - a_lo), log(1 - a_hi)
  size_t cap_pre = 0;
  uint32_t *host_ranges = nullptr;   // pinned copy of tile_range (rotation path)
  size_t cap_host_ranges = 0;
  uint32_t *host_seg = nullptr;      // pinned: segment offsets of the lists, then segment -> list
  size_t cap_host_seg = 0;
  double *segsum = nullptr;          // [segments][64][2] segment totals, then offsets
  size_t cap_segsum = 0;
  double *listlo = nullptr;          // [lists of a launch][64] list totals of log(1 - a_lo)
  size_t cap_listlo = 0;
  unsigned long long *ind_und = nullptr;   // [cells of a launch] undecided Ind pairs
  size_t cap_ind_und = 0;
  float *out_stage = nullptr;        // host outputs: the device images (lower, then upper)
  size_t cap_out_stage = 0;
  // Arena mode (the allocation-free entry point): buffers are carved from [arena,
  // arena + arena_cap) by a bump pointer instead of hipMalloc; nothing is freed, pinned
  // host blocks and events are not created (pose_host / host_counters point to host
  // storage set by the caller), and arena_overflow records a request past the end.
  unsigned char *arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  bool arena_overflow = false;
  bool no_events = false;        // a planned launch's workspace: no timing events recorded
};

// ---- launchers (ar_project.hip) ----
int pose_forms_host(const ar_pose_box &box, int P, PoseForms &out);
// one pose box (pose by value, poses_dev == nullptr) or ncells boxes (poses_dev[ncells]);
// outputs at global index cell * n + g
hipError_t launch_project(int P, const SceneDev &sc, const PoseForms &pose, const PoseForms *poses_dev, int ncells,
                          const Params &prm,
                          Workspace &ws, hipStream_t s);
// types only for ncells boxes (poses_dev[ncells]); counts[2 * ncells] (zeroed by the
// caller) receive per cell the MatrixInv failures kept somewhere in the image and the
// near-plane straddlers
hipError_t launch_classify(int P, const SceneDev &sc, const PoseForms *poses_dev, int ncells, const Params &prm,
                           unsigned long long *counts, hipStream_t s);
// ---- sorting / scans (ar_sort.hip) ----
hipError_t radix_sort_u64(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt, int n,
                          int begin_bit, int end_bit, Workspace &ws, hipStream_t s, bool *result_in_alt);
hipError_t radix_sort_u32(uint32_t *keys, uint32_t *keys_alt, uint32_t *vals, uint32_t *vals_alt, int n,
                          int begin_bit, int end_bit, Workspace &ws, hipStream_t s, bool *result_in_alt);
hipError_t exclusive_scan_u32(uint32_t *data, int n, Workspace &ws, hipStream_t s);
// *total (zeroed by the caller) += sum of data[0 .. n) in 64 bits (the true total of counts
// whose 32-bit scan may wrap)
hipError_t sum_u32_u64(const uint32_t *data, size_t n, unsigned long long *total, hipStream_t s);
// keys[i] = cell of the global item items[i] (item_cell; item_off null: items[i] / n_cell)
hipError_t launch_cell_keys(const uint32_t *items, int n_total, int n_cell, uint32_t *keys, hipStream_t s,
                            const uint32_t *item_off = nullptr, int ncells = 0);
hipError_t ensure_hist(Workspace &ws, size_t n_entries);

// (Re)allocate p for `need` elements, keeping the workspace's byte count; old contents
// are not kept.
template <typename T>
inline hipError_t grow(Workspace &ws, T *&p, size_t need) {
  if (ws.arena) {
    const size_t b = std::max(need, (size_t)64) * sizeof(T);
    const size_t at = (ws.arena_used + 255) / 256 * 256;
    if (at > ws.arena_cap || b > ws.arena_cap - at) {
      ws.arena_overflow = true;
      return hipErrorOutOfMemory;
    }
    p = reinterpret_cast<T *>(ws.arena + at);
    ws.arena_used = at + b;
    return hipSuccess;
  }
  if (p) {
    auto it = ws.sizes.find((void *)p);
    if (it != ws.sizes.end()) {
      ws.bytes -= it->second;
      ws.sizes.erase(it);
    }
    const hipError_t e = hipFree(p);
    p = nullptr;
    if (e != hipSuccess) return e;
  }
  const size_t b = std::max(need, (size_t)64) * sizeof(T);
  const hipError_t e = hipMalloc((void **)&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    return e;
  }
  ws.sizes[(void *)p] = b;
  ws.bytes += b;
  return hipSuccess;
}

// Free every buffer, event and pinned block of a workspace and reset it.
void release_workspace(Workspace &ws);
// ---- binning and pixel loops (ar_raster.hip) ----
// items in depth-rank order perm[r] = cell * n_cell + gid; list id = cell * ntiles + tile
hipError_t launch_count_tiles(int P, const Workspace &ws, int n_total, int n_cell, const Params &prm, hipStream_t s);
// cap (planned launches): more list entries than cap are not written and set the overflow counter
hipError_t launch_emit_tiles(int P, const Workspace &ws, int n_total, int n_cell, const Params &prm, hipStream_t s,
                             uint32_t cap = 0);
// p[i] = v for *n_dev <= i < cap
hipError_t launch_fill_tail(uint32_t *p, const uint32_t *n_dev, size_t cap, uint32_t v, hipStream_t s);
hipError_t launch_tile_ranges(const uint32_t *keys, int npairs, uint32_t *ranges, int ntiles, hipStream_t s);
int part_fields(int P);
// waves of the translation pixel kernel the device holds at once
int seg_resident_waves(int P);
hipError_t launch_segments(const Workspace &ws, int nlists, int L, hipStream_t s, int nsub = 1);
hipError_t launch_segment_map(const Workspace &ws, int nlists, hipStream_t s, uint32_t cap = 0);
// records ev[1] / ev[2] around the per-segment pixel kernel; lists cell * ntiles + tile,
// images [cell][H][W][3]
hipError_t launch_raster_translation(int P, const Workspace &ws, const uint32_t *lists, int nlists, const Params &prm,
                                     int L, int nseg_max, float *lo, float *hi, hipStream_t s);
// general path (ar_general.hip)
hipError_t launch_list_box(const Workspace &ws, const uint32_t *lists, const PoseForms *poses, int nlists, int ntiles,
                           const SceneDev &sc,
                           hipStream_t s);
// poses_dev[cell] for list ids cell * ntiles + tile
// passes of the Ind runs kernel
constexpr int kRunsWindows = 0;   // the window [ps, qe) of each entry and its mask words
constexpr int kRunsCount = 1;     // Ind tests; run counts; masks of the long windows stored
constexpr int kRunsEmit = 2;      // runs written (long windows from the stored masks)
// one pass of the Ind runs kernel over the list entries pbase .. pbase + ng - 1 (a group
// of whole lists; win, woff, run_cnt, runs and the compact copy are indexed relative to
// pbase); masks (the long windows' Ind masks) may be null
// Counts a planned launch keeps on the device (all null / zero on the ordinary path):
// entries, the number of list entries (the kernels take at most that many of their ng);
// runs_cap, the room for Ind runs (more are not written and set the overflow counter).
struct DevCounts {
  const uint32_t *entries = nullptr;
  uint32_t runs_cap = 0;
  unsigned long long *ind_und = nullptr;   // counting pass: undecided Ind pairs per cell (or null)
  const double *cbox = nullptr;            // windows pass: boxes of the kChunk-position chunks (or null)
};
// list positions per chunk box of the Ind windows' trimming
constexpr int kChunkLog = 6;
constexpr int kChunk = 1 << kChunkLog;
// Boxes of the chunks of kChunk list positions [kChunk c, kChunk (c + 1)) of the launch (npos
// positions): per chunk the box of the means the Ind tests read (lo[3], hi[3]; +inf /
// -inf when one is NaN) and the range of the nominal depths [cmin, cmax], 8 doubles.
hipError_t launch_chunk_boxes(const Workspace &ws, const uint32_t *lists, const SceneDev &sc, int ntiles, size_t npos,
                              double *cbox, hipStream_t s);
hipError_t launch_runs(int P, const Workspace &ws, const uint32_t *lists, const PoseForms *poses_dev, int ntiles,
                       const SceneDev &sc, uint32_t pbase, int ng, int window_mode, int mode,
                       unsigned long long *masks, bool compact, hipStream_t s, const DevCounts &dc = DevCounts{});
// the compact copy (cmean, cform) of the items' means and depth forms by list position,
// for the entries pbase .. pbase + ng - 1
hipError_t launch_ind_gather(int P, const Workspace &ws, const uint32_t *lists, const SceneDev &sc, int ntiles,
                             uint32_t pbase, int ng, hipStream_t s, const uint32_t *ng_dev = nullptr);
// one launch of the rotation pixel loop: lists list0 .. list0 + nl - 1 with entries from
// position pos0, their segments seg0 .. seg0 + nseg - 1 of L positions
struct RotChunk {
  int list0, nl, seg0, nseg, L;
  uint32_t pos0;
  uint32_t gbase;  // first list position of the list group whose run counts and runs are held
  bool absolute;   // add the segment offsets to the running sums in a pass of their own
};
hipError_t launch_raster_general(int P, const Workspace &ws, const uint32_t *lists, const RotChunk &c,
                                 const Params &prm, float *lo, float *hi, hipStream_t s);

}  // namespace ar
