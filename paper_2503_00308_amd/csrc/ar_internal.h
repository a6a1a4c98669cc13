// Internal declarations shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ar.h"

namespace ar {

constexpr int kMaxP = 6;        // pose variables: 3 translations + 3 angles
constexpr int kTile = 8;        // pixel tile side (one 64-lane wave covers a tile)
constexpr int kTilePix = kTile * kTile;

// Gaussian categories decided in the per-Gaussian stage.
enum GaussType : int32_t {
  kNormal = 0,    // full relational alpha bounds
  kFallback = 1,  // MatrixInv assertion failed: alpha in [0, footprint bound]
  kWild = 2,      // straddles the near plane (or unbounded footprint): alpha in [0, o]
  kDropped = 3    // behind the near plane at every pose: never contributes
};

// Per-Gaussian FP32 record consumed by the pixel loop.  Forms are (P coefficients,
// constant); every stored lower form is rounded down and every upper form up.
// d^2 and d*up are stored as two-float sums (hi + lo, about 48 bits): v = u d^2 - d up
// cancels them, and the rounding of a single float would dominate v near the mean.
template <int P>
struct Rec {
  static constexpr int F = P + 1;
  static constexpr int D2 = 0;          // d^2: lower (hi, lo), upper (hi, lo)
  static constexpr int DUP = 4 * F;     // d*up_k, k = 0,1: lower (hi, lo), upper (hi, lo) each
  static constexpr int B = 12 * F;      // B = Conic*Mp, entry e = 3k+n: (lower, upper)
  static constexpr int BI = 24 * F;     // interval of B: lo[6], hi[6]
  static constexpr int SC = 24 * F + 12;
  // scalars (offsets from SC)
  static constexpr int MD2 = 0, MDUP0 = 1, MDUP1 = 2, MBB0 = 3, MBB1 = 4, BMAX0 = 5, BMAX1 = 6;
  static constexpr int O = 7, C0 = 8, C1 = 9, C2 = 10;
  static constexpr int MU0LO = 11, MU0HI = 12, MU1LO = 13, MU1HI = 14, R2 = 15, LAM = 16;
  static constexpr int TYPE = 17;
  static constexpr int NSC = 20;
  static constexpr int STRIDE = ((SC + NSC) + 3) / 4 * 4;
};

inline int rec_stride(int P) {
  return ((24 * (P + 1) + 12 + 20) + 3) / 4 * 4;
}

// Pose set as linear forms over e in [-1,1]^P (FP64): uc = A (uw - tau) + beta.
struct PoseForms {
  int32_t P;
  int32_t pad;
  double A[9][2][kMaxP + 1];
  double tau[3][2][kMaxP + 1];
  double beta[3][2][kMaxP + 1];
};

struct Params {
  int32_t width, height;
  double fx, fy, cx, cy;
  int32_t taylor_k;
  double z_near;
  double eps_cull;     // cull_budget / n
  double E;            // widening for pruning
  double t_min;
  int32_t ntx, nty;    // tiles
  int32_t groups, chunk;
};

struct SceneDev {
  int32_t n;
  float *mean;   // [3][n]
  float *cov;    // [9][n]
  float *opac;   // [n]
  float *rgb;    // [3][n]
};

// Device workspace (grown on demand, owned by a scene handle).
struct Workspace {
  size_t cap_n = 0, cap_pairs = 0, cap_tiles = 0, cap_scratch = 0;
  void *pose = nullptr;        // PoseForms (one per cell)
  int32_t cap_cells = 0;
  float *rec = nullptr;        // [n][stride]
  uint64_t *key = nullptr;     // [n] depth key (by gid, kept for tie tests)
  uint64_t *key_sort = nullptr;  // [n] copy of the keys, sorted in place
  uint64_t *key_alt = nullptr; // [n]
  uint32_t *perm = nullptr;    // [n] rank -> gid
  uint32_t *perm_alt = nullptr;
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
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // call start, raster start, raster end
  unsigned long long *host_counters = nullptr;  // pinned
  // general (rotation) path
  double *dint = nullptr;      // [n][2] depth interval (lo, hi) by gid
  double *wmax = nullptr;      // [tiles] widest depth interval of the tile's list
  uint32_t *run_cnt = nullptr; // [pairs][2] + 1: Def / May run counts, then offsets
  size_t cap_run_cnt = 0;
  uint32_t *runs = nullptr;    // [runs][2] list-position ranges [start, end)
  size_t cap_runs = 0;
  double *pre = nullptr;       // [pairs][64][2] per-pixel prefix sums of log(1 - a_lo), log(1 - a_hi)
  uint32_t *prez = nullptr;    // [pairs][64] per-pixel prefix counts of a_hi == 1
  size_t cap_pre = 0;
};

// ---- launchers (ar_project.hip) ----
hipError_t launch_pose(const ar_pose_box *boxes_dev, int ncells, int P, PoseForms *out, hipStream_t s);
hipError_t launch_pose_value(const ar_pose_box &box, int P, PoseForms *out, hipStream_t s);
hipError_t launch_project(int P, const SceneDev &sc, const PoseForms *pose, const Params &prm,
                          Workspace &ws, hipStream_t s);
// ---- sorting / scans (ar_sort.hip) ----
hipError_t radix_sort_u64(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt, int n,
                          int begin_bit, int end_bit, Workspace &ws, hipStream_t s, bool *result_in_alt);
hipError_t radix_sort_u32(uint32_t *keys, uint32_t *keys_alt, uint32_t *vals, uint32_t *vals_alt, int n,
                          int begin_bit, int end_bit, Workspace &ws, hipStream_t s, bool *result_in_alt);
hipError_t exclusive_scan_u32(uint32_t *data, int n, Workspace &ws, hipStream_t s);
hipError_t ensure_hist(Workspace &ws, size_t n_entries);
// ---- binning and pixel loops (ar_raster.hip) ----
hipError_t launch_count_tiles(int P, const Workspace &ws, int n, const Params &prm, hipStream_t s);
hipError_t launch_emit_tiles(int P, const Workspace &ws, int n, const Params &prm, hipStream_t s);
hipError_t launch_tile_ranges(const uint32_t *keys, int npairs, uint32_t *ranges, int ntiles, hipStream_t s);
hipError_t launch_raster_translation(int P, const Workspace &ws, const uint32_t *lists, const SceneDev &sc,
                                     const Params &prm, float *lo, float *hi, hipStream_t s);
// general path (ar_general.hip)
hipError_t launch_tile_wmax(const Workspace &ws, const uint32_t *lists, int ntiles, hipStream_t s);
hipError_t launch_runs(int P, const Workspace &ws, const uint32_t *lists, const PoseForms *pose, const SceneDev &sc,
                       int npairs, bool emit, hipStream_t s);
hipError_t launch_raster_general(int P, const Workspace &ws, const uint32_t *lists, const Params &prm, float *lo,
                                 float *hi, hipStream_t s);

}  // namespace ar
