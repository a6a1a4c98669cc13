// General pixel loop for pose boxes whose depth order can change (rotations), gfx950.
//
// BlendInd (Alg. BlendInd) with the three-valued Ind(d_i - d_j):
//   T_hi[i] = prod_{j: Ind_ij = 1} (1 - a_lo[j]),   T_lo[i] = prod_{j: Ind_ij != 0} (1 - a_hi[j]).
// Ind is a property of the Gaussian pair, not of the pixel, so it is decided once per
// tile list in FP64 (k_runs) on two sound bounds of d_i - d_j: the identity
// A_z (uw_i - uw_j) and the literal difference of the depth forms (1e-10 margin).
// Lists are in order of the nominal depth c = m . uw (m: the depth row of A at the box
// centre).  The identity bound lies within sum_l R_l |uw_i,l - uw_j,l| of c_i - c_j,
// R_l the total radius of the form A_z,l over the box.  Two bounds of that sum hold for
// every j of a tile list:
//   (box)   rho_i = sum_l R_l times the distance of uw_i,l to the far side of the box of
//           the list's means;
//   (split) uw_i - uw_j = ((c_i - c_j) / |m|^2) m + (v_i - v_j) with v the part of uw
//           across m, so the sum is at most beta |c_i - c_j| + alpha_i, beta =
//           sum_l R_l |m_l| / |m|^2 and alpha_i the box bound on the v parts; then
//           |c_i - c_j| > alpha_i / (1 - beta) suffices.
// A Gaussian whose mean a scene variable moves (sets of scenes, Sec. 4.6) is not the constant
// uw_i of the identity: its entry in the means the Ind tests read (ind_mean) is NaN, which
// makes both comparisons of the identity bound false, so the literal bound decides every
// pair that involves it; such scenes test every pair of a list (window mode 2).
// A tile list spans a long stretch of depth but little across it, so the split bound is
// usually far smaller.  Every j with c_j < c_i - rho_i has Ind_ij = 1 and every j with
// c_j > c_i + rho_i has Ind_ij = 0 (rho_i the smaller bound, plus rounding margins); only
// the window between needs the pairwise test.  Translation uncertainty cancels in
// d_i - d_j, so the window is much narrower than one from depth intervals.  The sets
// {j: Ind_ij = 1} and {j: Ind_ij != 0} are
// stored as runs of list positions.
//
// The pixel loop works on segments of L list positions, one wave per segment, one lane
// per pixel of the 8x8 tile:
//   A (k_rot_prefix): per pixel, running sums of log(1 - a_lo) and log(1 - a_hi) (FP64;
//      a_hi = 1 enters as log 2^-60, see below), and the segment totals;
//   k_rot_offsets: per list, the running totals in front of each segment, and
//   k_rot_absolute: those totals added to the segments' running sums;
//   B (k_rot_blend): for each Gaussian i, the product over a run [a, b) is
//      exp(S(b-1) - S(a-1)), S the absolute running sum, so T_lo[i] and T_hi[i]
//      cost one load per run end; the colour forms are accumulated with these
//      absolute transmittances, so a tile's bounds are the sum over its segments
//      (k_rot_merge).
// Equal-length segments spread a long tile list over many waves.  The prefix sums
// carry a rounding bound that is added outward before exp.  A factor 1 - a_hi = 0 (an
// alpha that may reach 1) enters the upper sums as 2^-60 instead, so a lower
// transmittance that should be 0 is at most 2^-60; the merge widens every lower bound
// by n 2^-60 (n list entries), which keeps it sound without a count row per pixel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ar_blend.h"
#include "ar_internal.h"

namespace ar {

constexpr double kIndMargin = 1e-10;   // margin of the literal depth-difference test
constexpr double kWinMargin = 1e-9;    // margin of the depth-interval window
constexpr double kZeroFactor = 0x1p-60; // stands for a factor 1 - a_hi = 0 in the upper log sums

// Per tile list (items cell * n + g): the box of the Gaussians' means uw [0, 6), the box
// of their parts across the nominal depth direction m, v = uw - (m . uw / |m|^2) m,
// [6, 12), and the largest |uw_l| [12] (the scale of the rounding margins).
__global__ __launch_bounds__(256) void k_list_box(const uint32_t *__restrict__ ranges,
                                                  const uint32_t *__restrict__ lists,
                                                  const PoseForms *__restrict__ poses, SceneDev scene, int ntiles,
                                                  double *__restrict__ lbox, const CellScene *__restrict__ tab) {
  __shared__ double red[kListBox][256];
  const int lst = blockIdx.x;
  const int cell = lst / ntiles;
  const SceneDev &sc = cell_scene(scene, tab, cell);
  const size_t gbase = cell_first(scene, tab, cell);
  const PoseForms &pose = poses[cell];
  double m[3], mm = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    m[l] = 0.5 * (pose.A[6 + l][0][kMaxP] + pose.A[6 + l][1][kMaxP]);
    mm += m[l] * m[l];
  }
  const uint32_t beg = ranges[2 * lst], end = ranges[2 * lst + 1];
  double v[kListBox];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    v[l] = INFINITY;
    v[3 + l] = -INFINITY;
    v[6 + l] = INFINITY;
    v[9 + l] = -INFINITY;
  }
  v[12] = 0.0;
  for (uint32_t p = beg + threadIdx.x; p < end; p += 256) {
    const size_t g = lists[p] - gbase;
    double u[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) u[l] = (double)sc.ind_mean[(size_t)l * sc.n + g];
    const double c = (m[0] * u[0] + m[1] * u[1] + m[2] * u[2]) / mm;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const double w = u[l] - c * m[l];
      v[l] = fmin(v[l], u[l]);
      v[3 + l] = fmax(v[3 + l], u[l]);
      v[6 + l] = fmin(v[6 + l], w);
      v[9 + l] = fmax(v[9 + l], w);
      v[12] = fmax(v[12], fabs(u[l]));
    }
  }
#pragma unroll
  for (int k = 0; k < kListBox; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        red[l][threadIdx.x] = fmin(red[l][threadIdx.x], red[l][threadIdx.x + off]);
        red[3 + l][threadIdx.x] = fmax(red[3 + l][threadIdx.x], red[3 + l][threadIdx.x + off]);
        red[6 + l][threadIdx.x] = fmin(red[6 + l][threadIdx.x], red[6 + l][threadIdx.x + off]);
        red[9 + l][threadIdx.x] = fmax(red[9 + l][threadIdx.x], red[9 + l][threadIdx.x + off]);
      }
      red[12][threadIdx.x] = fmax(red[12][threadIdx.x], red[12][threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x < kListBox) lbox[kListBox * (size_t)lst + threadIdx.x] = red[threadIdx.x][0];
}

// The quick Ind test of ind_pair for every list position of a chunk at once: 1 when it
// decides Ind = 1 (surely in front) for all of them, 0 when Ind = 0 for all, else -1.
// cb: the chunk's box of means lo[3], hi[3] and nominal depths [cb[6], cb[7]]; uwi, ci:
// entry i's mean and nominal depth.  For a position j of the chunk, q_j = sum_l (uw_i -
// uw_j)_l Zm[l][kMaxP] = c_i - c_j (the nominal depths use the same multipliers) lies in
// [c_i - cmax, c_i - cmin], and sum_l |D_l| Zq_l <= R = sum_l Zq_l max|uw_i,l - box_l|, so
// beyond R and the borderline band 1e-12 (1 + sum_l max|D_l|) every position's quick
// test (and so its Ind) is decided; the margin 2^-40 (E + R), E = 1 + sum_l
// |Zm[l][kMaxP]| (|uw_i,l| + max|box_l|), covers the rounding of the nominal depths and of
// each pair's test.
__device__ __forceinline__ int chunk_quick(const PoseForms &pose, const double *uwi, double ci,
                                           const double *__restrict__ cb) {
  double R = 0.0, Dsum = 0.0, E = 1.0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const double lo = cb[l], hi = cb[3 + l];
    const double dmax = fmax(fabs(uwi[l] - lo), fabs(uwi[l] - hi));
    R = fma(dmax, pose.Zq[l], R);
    Dsum += dmax;
    E = fma(fabs(pose.Zm[l][kMaxP]), fabs(uwi[l]) + fmax(fabs(lo), fabs(hi)), E);
  }
  const double band = 1e-12 * (1.0 + Dsum) + 0x1p-40 * (E + R);
  if ((ci - cb[7]) - R - band > 0.0) return 1;
  if ((ci - cb[6]) + R + band < 0.0) return 0;
  return -1;
}

// Boxes of the chunks of kChunk list positions (see launch_chunk_boxes): lane t of a wave
// takes position 64 w + t, and the lanes of each chunk reduce their values together.
__global__ __launch_bounds__(256) void k_chunk_boxes(const uint32_t *__restrict__ pkey,
                                                     const uint32_t *__restrict__ lists,
                                                     const double *__restrict__ dint, SceneDev scene, int ntiles,
                                                     size_t npos, double *__restrict__ cbox,
                                                     const CellScene *__restrict__ tab) {
  const int lane = threadIdx.x & 63;
  const size_t w = (size_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const size_t q = w * 64 + lane;
  if (w * 64 >= npos) return;
  double v[8] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, INFINITY, -INFINITY};
  bool nan = false;
  if (q < npos) {
    const uint32_t g = lists[q];
    const int cell = (int)(pkey[q] / (uint32_t)ntiles);
    const SceneDev &sc = cell_scene(scene, tab, cell);
    const size_t lg = g - cell_first(scene, tab, cell);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const double u = (double)sc.ind_mean[(size_t)l * sc.n + lg];
      nan = nan || u != u;
      v[l] = u;
      v[3 + l] = u;
    }
    v[6] = v[7] = dint[2 * (size_t)g];
  }
  for (int off = kChunk / 2; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double o = __shfl_xor(v[k], off);
      v[k] = (k < 3 || k == 6) ? fmin(v[k], o) : fmax(v[k], o);
    }
  }
  // a NaN mean anywhere in the chunk: the box decides nothing
  const unsigned long long nb = __ballot(nan);
  nan = (nb >> (lane & ~(kChunk - 1))) & ((kChunk == 64) ? ~0ull : ((1ull << kChunk) - 1ull));
  if ((lane & (kChunk - 1)) == 0 && q < npos) {
    double *o = cbox + (q >> kChunkLog) * 8;
#pragma unroll
    for (int k = 0; k < 6; ++k) o[k] = nan ? (k < 3 ? INFINITY : -INFINITY) : v[k];
    o[6] = v[6];
    o[7] = v[7];
  }
}

// Ind(d_i - d_j) in {0, 1, 2 = unknown} (see the file comment).  Depth forms: the lower
// form's coefficients at [0, P) and its constant at [S - 1], the upper form's at
// [S, S + P) and [2S - 1] (S = kMaxP + 1 by item, S = P + 1 in the compact copy).
// BORDER: *border is set when the deciding bound lies within rounding of its threshold
// (1e-12 (1 + |uw_i - uw_j|_1) of 0 for the identity, of +-kIndMargin for the literal
// bound, which decides only where the identity does not; an exact tie of the identity,
// both ends 0, is not borderline): a decision another order of operations might flip.
template <int P, int S = kMaxP + 1, bool BORDER = false>
__device__ __forceinline__ int ind_pair(const PoseForms &pose, const double *uwi, const double *uwj,
                                        const double *dfi, const double *dfj, bool *border = nullptr) {
  // Quick test first.  With D = uw_i - uw_j (as rounded) the identity bound below has
  // lower end >= q - sum_l |D_l| R_l and upper end <= q + sum_l |D_l| R_l, q = sum_l D_l
  // Zm[l][kMaxP] its constant and R_l = |Zr[l][kMaxP]| + sum_k (|Zm[l][k]| + |Zr[l][k]|)
  // (triangle inequality on each coefficient).  Zq_l exceeds R_l by 2^-45 (|Zm[l][kMaxP]|
  // + R_l), more than the rounding of both computations (< 32 u (sum_l |D_l| (|Zm[l][kMaxP]|
  // + R_l))), so a quick decision beyond the borderline band is the identity's own
  // decision, with the same borderline flag (false); the result does not change.
  double qc = 0.0, qr = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const double d = uwi[l] - uwj[l];
    qc = fma(d, pose.Zm[l][kMaxP], qc);
    qr = fma(fabs(d), pose.Zq[l], qr);
  }
  const double qt = BORDER ? 1e-12 * (1.0 + fabs(uwi[0] - uwj[0]) + fabs(uwi[1] - uwj[1]) + fabs(uwi[2] - uwj[2]))
                           : 0.0;
  if (qc - qr > qt) {
    if (BORDER) *border = false;
    return 1;
  }
  if (qc + qr < -qt) {
    if (BORDER) *border = false;
    return 0;
  }
  // identity bound: sum_l A_z,l * (uw_i - uw_j)_l, each term a scaled form; with A_z,l
  // in mid-radius form (m, r), c A_z,l has lower form c m - |c| r and upper c m + |c| r
  double mid[P + 1], rad[P + 1];
#pragma unroll
  for (int k = 0; k <= P; ++k) { mid[k] = 0.0; rad[k] = 0.0; }
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const double c = uwi[l] - uwj[l], ac = fabs(c);
#pragma unroll
    for (int k = 0; k < P; ++k) {
      mid[k] = fma(c, pose.Zm[l][k], mid[k]);
      rad[k] = fma(ac, pose.Zr[l][k], rad[k]);
    }
    mid[P] = fma(c, pose.Zm[l][kMaxP], mid[P]);
    rad[P] = fma(ac, pose.Zr[l][kMaxP], rad[P]);
  }
  double slo = 0.0, sup = 0.0;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    slo += fabs(mid[k] - rad[k]);
    sup += fabs(mid[k] + rad[k]);
  }
  const double lo_r = (mid[P] - rad[P]) - slo, hi_r = (mid[P] + rad[P]) + sup;
  double sb = 0.0;
  if (BORDER) {
    sb = 1e-12 * (1.0 + fabs(uwi[0] - uwj[0]) + fabs(uwi[1] - uwj[1]) + fabs(uwi[2] - uwj[2]));
    *border = !(lo_r == 0.0 && hi_r == 0.0) && (fabs(lo_r) < sb || fabs(hi_r) < sb);
  }
  // both bounds are sound, so when the identity decides the literal bound cannot
  // contradict it; its form loads are skipped
  if (lo_r > 0.0) return 1;
  if (hi_r <= 0.0) return 0;
  // literal bound: d_i.lower - d_j.upper and d_i.upper - d_j.lower
  double sl = 0.0, sh = 0.0;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    sl += fabs(dfi[k] - dfj[S + k]);
    sh += fabs(dfi[S + k] - dfj[k]);
  }
  const double lo_l = (dfi[S - 1] - dfj[2 * S - 1]) - sl;
  const double hi_l = (dfi[2 * S - 1] - dfj[S - 1]) + sh;
  if (BORDER) *border = *border || fabs(lo_l - kIndMargin) < sb || fabs(hi_l + kIndMargin) < sb;
  if (lo_l > kIndMargin) return 1;
  if (hi_l <= -kIndMargin) return 0;
  return 2;
}

// sums[key] += v for every lane of the wave (key < 0: nothing): one atomic per distinct
// key of the wave rather than one per lane (a wave's entries mostly share their cell, and
// per-lane atomics on one address serialise).  Called by the whole wave.
__device__ __forceinline__ void wave_add_by_key(unsigned long long *sums, int key, unsigned long long v) {
  bool pend = key >= 0 && v != 0ull;
  for (;;) {
    const unsigned long long m = __ballot(pend);
    if (!m) break;
    const int l0 = __builtin_ctzll(m);
    const int k0 = __builtin_amdgcn_readlane(key, l0);
    const bool mine = pend && key == k0;
    unsigned long long t = mine ? v : 0ull;
    for (int off = 32; off > 0; off >>= 1) t += (unsigned long long)__shfl_xor(t, off);
    if ((int)(threadIdx.x & 63) == l0) atomicAdd(&sums[k0], t);
    pend = pend && !mine;
  }
}

__device__ __forceinline__ double readlane_d(double x, int k) {
  const unsigned long long b = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, k);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), k);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Where the Ind tests read the mean and the depth forms of list position j: by item
// (gathers), or from a copy laid out by list position (COMPACT: consecutive positions
// are consecutive in memory, so a wave's 64 tests load contiguous data).
template <int P, bool COMPACT>
struct IndSrc {
  static constexpr int S = COMPACT ? P + 1 : kMaxP + 1;
  const uint32_t *list;      // the list's items
  const float *mean;         // scene means [3][n] (by item)
  const double *dform;       // depth forms by item, or by list position (COMPACT)
  const float4 *cmean;       // means by list position (COMPACT)
  int n;                     // scene size
  size_t gbase;              // the cell's first item
  size_t pos0;               // the list's first position relative to the group's first (COMPACT)

  __device__ __forceinline__ void mean_of(int j, double *uw) const {
    if (COMPACT) {
      const float4 m = cmean[pos0 + j];
      uw[0] = m.x;
      uw[1] = m.y;
      uw[2] = m.z;
    } else {
      const size_t lj = list[j] - gbase;
      uw[0] = mean[lj];
      uw[1] = mean[n + lj];
      uw[2] = mean[2 * (size_t)n + lj];
    }
  }
  __device__ __forceinline__ const double *forms_of(int j) const {
    return COMPACT ? dform + (pos0 + j) * (size_t)(2 * S) : dform + (size_t)list[j] * (2 * S);
  }
};

// Compact copy for the Ind tests: per list position of a group (positions pbase + q,
// q < ng), the item's mean (float4) and depth forms (lower then upper, P + 1 doubles
// each), at index q.
// ng_dev (planned launches, may be null): the number of entries, when below ng.
template <int P>
__global__ __launch_bounds__(256) void k_ind_gather(const uint32_t *__restrict__ pkey,
                                                    const uint32_t *__restrict__ lists, const double *__restrict__ dform,
                                                    SceneDev scene, int ntiles, uint32_t pbase, int ng,
                                                    const uint32_t *__restrict__ ng_dev,
                                                    float4 *__restrict__ cmean, double *__restrict__ cform,
                                                    const CellScene *__restrict__ tab) {
  constexpr int F = P + 1;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (ng_dev) ng = min(ng, (int)*ng_dev);
  if (q >= ng) return;
  const size_t p = (size_t)pbase + q;
  const uint32_t g = lists[p];
  const int cell = (int)(pkey[p] / (uint32_t)ntiles);
  const SceneDev &sc = cell_scene(scene, tab, cell);
  const size_t lg = g - cell_first(scene, tab, cell);
  cmean[q] = make_float4(sc.ind_mean[lg], sc.ind_mean[sc.n + lg], sc.ind_mean[2 * (size_t)sc.n + lg], 0.0f);
  const double *d = dform + (size_t)g * 2 * (kMaxP + 1);
  double *o = cform + (size_t)q * 2 * F;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    o[k] = d[k];
    o[F + k] = d[kMaxP + 1 + k];
  }
  o[P] = d[kMaxP];
  o[F + P] = d[2 * kMaxP + 1];
}

// Runs of one list position i over its window [ps, qe), the whole wave at once: lane b
// tests j = t + b (or, when emitting from stored masks, reads the chunk's two mask
// words), and ballots give the run starts (in the set, previous not) and ends (not in
// the set, previous in it).  Starts and ends are ranked separately, so a run that spans
// two chunks gets its start and end from different iterations.  Returns the number of
// runs of each set (wave-uniform) and, when tested, the number of undecided pairs (Ind
// = 2: in the second set and not in the first).  masks: two words (Ind = 1, Ind != 0)
// per chunk of 64 window positions, or null.
template <int P, int MODE, bool COMPACT>
__device__ __forceinline__ void wave_runs(const PoseForms &pose, const IndSrc<P, COMPACT> &src, int i, int ps,
                                          int qe, const double *uwi, const double *dfi,
                                          unsigned long long *masks, uint32_t *out_def, uint32_t *out_may,
                                          int lane, uint32_t &ndef, uint32_t &nmay, uint32_t &nund,
                                          uint32_t &nbord) {
  constexpr bool EMIT = MODE == kRunsEmit;
  uint32_t sd = 0, ed = 0, sm = 0, em = 0;      // run starts / ends so far
  bool cd = ps > 0, cm = ps > 0;                // the position before the chunk is in the set
  if (ps > 0) {
    // open runs [0, ps) of certain occluders
    if (EMIT && lane == 0) {
      out_def[0] = 0u;
      out_may[0] = 0u;
    }
    sd = sm = 1;
  }
  const unsigned long long below = (1ull << lane) - 1ull;
  nund = 0;
  nbord = 0;
  for (int t = ps, c = 0; t < qe; t += 64, ++c) {
    const int j = t + lane;
    const bool valid = j < qe;
    const unsigned long long V = __ballot(valid);
    unsigned long long D, M;
    if (EMIT && masks) {
      D = masks[2 * (size_t)c];
      M = masks[2 * (size_t)c + 1];
    } else {
      int ind = 0;
      bool bd = false;
      if (valid && j != i) {
        double uwj[3];
        src.mean_of(j, uwj);
        ind = ind_pair<P, IndSrc<P, COMPACT>::S, MODE == kRunsCount>(pose, uwi, uwj, dfi, src.forms_of(j), &bd);
      }
      D = __ballot(valid && ind == 1);
      M = __ballot(valid && ind != 0);
      nund += (uint32_t)__popcll(M & ~D);
      if (MODE == kRunsCount) nbord += (uint32_t)__popcll(__ballot(bd));
      if (MODE == kRunsCount && masks && lane == 0) {
        masks[2 * (size_t)c] = D;
        masks[2 * (size_t)c + 1] = M;
      }
    }
    const unsigned long long Dp = (D << 1) | (cd ? 1ull : 0ull), Mp = (M << 1) | (cm ? 1ull : 0ull);
    const unsigned long long sD = D & ~Dp, eD = ~D & Dp & V, sM = M & ~Mp, eM = ~M & Mp & V;
    if (EMIT) {
      if ((sD >> lane) & 1ull) out_def[2 * (sd + __popcll(sD & below))] = (uint32_t)j;
      if ((eD >> lane) & 1ull) out_def[2 * (ed + __popcll(eD & below)) + 1] = (uint32_t)j;
      if ((sM >> lane) & 1ull) out_may[2 * (sm + __popcll(sM & below))] = (uint32_t)j;
      if ((eM >> lane) & 1ull) out_may[2 * (em + __popcll(eM & below)) + 1] = (uint32_t)j;
    }
    sd += __popcll(sD);
    ed += __popcll(eD);
    sm += __popcll(sM);
    em += __popcll(eM);
    const int last = min(64, qe - t) - 1;
    cd = (D >> last) & 1ull;
    cm = (M >> last) & 1ull;
  }
  if (cd) {
    if (EMIT && lane == 0) out_def[2 * ed + 1] = (uint32_t)qe;
    ++ed;
  }
  if (cm) {
    if (EMIT && lane == 0) out_may[2 * em + 1] = (uint32_t)qe;
    ++em;
  }
  ndef = ed;
  nmay = em;
}

// Windows longer than this go to the whole wave, one list position at a time; shorter
// ones are walked by their own lane.
constexpr int kWaveWindow = 64;

// Runs of {j: Ind_ij = 1} and {j: Ind_ij != 0} for 64 consecutive (tile, list position)
// entries per wave and step, over the entries pbase .. pbase + ng - 1 of a group of whole
// lists (win, woff, cnt, the compact copy and the runs are indexed relative to the group),
// in three passes (MODE):
//   kRunsWindows: each lane finds its entry's window [ps, qe) (win) and the number of
//     mask words a long window needs (wc: two per 64 positions, scanned into offsets);
//   kRunsCount: the Ind tests and the run counts (cnt); a short window is walked by its
//     own lane, the wave takes the long ones together (wave_runs) and stores their
//     masks when masks is not null;
//   kRunsEmit: the runs; long windows from their masks (no Ind tests) when stored.
template <int P, int MODE, bool COMPACT>
__global__ __launch_bounds__(256) void k_runs(const uint32_t *__restrict__ pkey, const uint32_t *__restrict__ ranges,
                                              const uint32_t *__restrict__ lists, const double *__restrict__ dint,
                                              const double *__restrict__ dform, const float4 *__restrict__ cmean,
                                              const double *__restrict__ cform, const double *__restrict__ lbox,
                                              const PoseForms *__restrict__ poses, int ntiles, SceneDev scene,
                                              uint32_t pbase, int ng, int window_mode, uint32_t *__restrict__ win,
                                              uint32_t *__restrict__ woff, unsigned long long *__restrict__ masks,
                                              uint32_t *__restrict__ cnt, uint32_t *__restrict__ runs,
                                              unsigned long long *__restrict__ counters,
                                              const uint32_t *__restrict__ ng_dev, uint32_t runs_cap,
                                              unsigned long long *__restrict__ ind_und,
                                              const CellScene *__restrict__ tab,
                                              const double *__restrict__ cbox) {
  constexpr bool EMIT = MODE == kRunsEmit;
  const int lane = threadIdx.x & 63;
  // planned launches: the entries counted on the device, and no runs past the buffer
  if (ng_dev) ng = min(ng, (int)*ng_dev);
  if (EMIT && runs_cap && cnt[2 * (size_t)ng] > runs_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) counters[kOverflow] = 1ull;
    return;
  }
  const int wave0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  const int nwaves = (int)(gridDim.x * (blockDim.x >> 6));
  unsigned long long wmax = 0, wsum = 0;   // window statistics of this lane's entries
  for (int p0 = wave0 * 64; p0 < ng; p0 += nwaves * 64) {
    const int p = p0 + lane;                       // entry of the group; list position pbase + p
    const bool have = p < ng;
    int cell = 0, beg = 0, i = 0, ps = 0, qe = 0;
    uint32_t gi = 0;
    double uwi[3] = {0.0, 0.0, 0.0};
    if (have) {
      const uint32_t tile = pkey[(size_t)pbase + p];   // list id: cell * ntiles + tile
      cell = (int)(tile / (uint32_t)ntiles);
      beg = (int)ranges[2 * tile];
      i = (int)(pbase + (uint32_t)p) - beg;
      const uint32_t *list = lists + beg;
      gi = list[i];
      const SceneDev &sc = cell_scene(scene, tab, cell);
      const size_t li = gi - cell_first(scene, tab, cell);
      uwi[0] = sc.ind_mean[li];
      uwi[1] = sc.ind_mean[sc.n + li];
      uwi[2] = sc.ind_mean[2 * sc.n + li];
      if (MODE != kRunsWindows) {
        ps = (int)win[2 * (size_t)p];
        qe = (int)win[2 * (size_t)p + 1];
      } else {
        const PoseForms &pose = poses[cell];
        const int n = (int)ranges[2 * tile + 1] - beg;
        // rho_i: |c_i - c_j| > rho_i decides Ind_ij (see the file comment)
        const double *bx = lbox + kListBox * (size_t)tile;
        double m[3], mm = 0.0, msum = 0.0, rsum = 0.0, rho_box = 0.0, mr = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          const double *fl = pose.A[6 + l][0], *fu = pose.A[6 + l][1];
          m[l] = 0.5 * (fl[kMaxP] + fu[kMaxP]);
          double R = 0.5 * (fu[kMaxP] - fl[kMaxP]);
          for (int k = 0; k < kMaxP; ++k) R += fmax(fabs(fl[k]), fabs(fu[k]));
          mm += m[l] * m[l];
          msum += fabs(m[l]);
          rsum += R;
          mr += R * fabs(m[l]);
          rho_box += R * fmax(uwi[l] - bx[l], bx[3 + l] - uwi[l]);
        }
        const double beta = mr / mm;
        const double ci_m = (m[0] * uwi[0] + m[1] * uwi[1] + m[2] * uwi[2]) / mm;
        double alpha = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          const double *fl = pose.A[6 + l][0], *fu = pose.A[6 + l][1];
          double R = 0.5 * (fu[kMaxP] - fl[kMaxP]);
          for (int k = 0; k < kMaxP; ++k) R += fmax(fabs(fl[k]), fabs(fu[k]));
          const double w = uwi[l] - ci_m * m[l];
          alpha += R * fmax(w - bx[6 + l], bx[9 + l] - w);
        }
        double rho = rho_box;
        if (beta < 0.5 && window_mode == 0) rho = fmin(rho, alpha / (1.0 - beta));
        if (window_mode == 2) rho = INFINITY;   // every pair of the list tested
        // rounding of c, v and the sums: relative 2^-40 and an absolute margin on the
        // scale of the means
        rho = rho * (1.0 + 0x1p-40) + 2.0 * (kWinMargin + 0x1p-40 * (1.0 + rsum) * (msum * bx[12] + 1.0));
        const double c_i = dint[2 * (size_t)gi];
        // first position with c >= c_i - rho (all before are in front for sure)
        int a = 0, b = i;
        const double t1 = c_i - rho;
        while (a < b) {
          const int mid = (a + b) >> 1;
          if (dint[2 * (size_t)list[mid]] < t1) a = mid + 1; else b = mid;
        }
        ps = a;
        // first position with c > c_i + rho (all from there are behind for sure)
        a = i;
        b = n;
        const double t2 = c_i + rho;
        while (a < b) {
          const int mid = (a + b) >> 1;
          if (dint[2 * (size_t)list[mid]] <= t2) a = mid + 1; else b = mid;
        }
        qe = a;
        // Trim the window's ends by whole chunks of kChunk list positions that the quick test
        // decides at once (chunk_quick, with the borderline band the counting pass uses):
        // surely in front at the start, surely behind at the end.  The tests and runs see
        // the same decisions, so only the number of tests changes.  (Window mode 2, every
        // pair tested, is left whole.)
        if (cbox && window_mode != 2) {
          while (ps < i) {
            const size_t q = (size_t)beg + ps;
            if (chunk_quick(pose, uwi, c_i, cbox + (q >> kChunkLog) * 8) != 1) break;
            ps = (int)min((long long)i, (long long)(((q >> kChunkLog) + 1) << kChunkLog) - (long long)beg);
          }
          while (qe > i + 1) {
            const size_t q = (size_t)beg + qe - 1;
            if (chunk_quick(pose, uwi, c_i, cbox + (q >> kChunkLog) * 8) != 0) break;
            qe = (int)max((long long)i + 1, (long long)((q >> kChunkLog) << kChunkLog) - (long long)beg);
          }
        }
        win[2 * (size_t)p] = (uint32_t)ps;
        win[2 * (size_t)p + 1] = (uint32_t)qe;
      }
    }
    const int W = qe - ps;
    const bool wide = W > kWaveWindow;
    if (MODE == kRunsWindows) {
      if (have) woff[p] = wide ? 2u * (uint32_t)((W + 63) / 64) : 0u;
      wmax = max(wmax, (unsigned long long)W);
      wsum += (unsigned long long)W;
      continue;
    }
    uint32_t *out_def = nullptr, *out_may = nullptr;
    if (EMIT && have) {
      out_def = runs + 2 * (size_t)cnt[2 * (size_t)p];
      out_may = runs + 2 * (size_t)cnt[2 * (size_t)p + 1];
    }
    uint32_t ndef = 0, nmay = 0, nund = 0, nbord = 0;
    if (have && !wide) {
      const PoseForms &pose = poses[cell];
      const SceneDev &sc = cell_scene(scene, tab, cell);
      const IndSrc<P, COMPACT> src{lists + beg, sc.ind_mean, COMPACT ? cform : dform, cmean, sc.n,
                                   cell_first(scene, tab, cell), (size_t)((uint32_t)beg - pbase)};
      const double *dfi = src.forms_of(i);
      int def_start = ps > 0 ? 0 : -1;   // open run [0, ps) of certain occluders
      int may_start = ps > 0 ? 0 : -1;
      for (int j = ps; j < qe; ++j) {
        int ind = 0;
        bool bd = false;
        if (j != i) {
          double uwj[3];
          src.mean_of(j, uwj);
          ind = ind_pair<P, IndSrc<P, COMPACT>::S, MODE == kRunsCount>(pose, uwi, uwj, dfi, src.forms_of(j), &bd);
        }
        const bool d1 = ind == 1, m1 = ind != 0;
        nund += ind == 2 ? 1u : 0u;
        nbord += bd ? 1u : 0u;
        if (d1 && def_start < 0) def_start = j;
        if (!d1 && def_start >= 0) {
          if (EMIT) { out_def[2 * ndef] = (uint32_t)def_start; out_def[2 * ndef + 1] = (uint32_t)j; }
          ++ndef;
          def_start = -1;
        }
        if (m1 && may_start < 0) may_start = j;
        if (!m1 && may_start >= 0) {
          if (EMIT) { out_may[2 * nmay] = (uint32_t)may_start; out_may[2 * nmay + 1] = (uint32_t)j; }
          ++nmay;
          may_start = -1;
        }
      }
      if (def_start >= 0) {
        if (EMIT) { out_def[2 * ndef] = (uint32_t)def_start; out_def[2 * ndef + 1] = (uint32_t)qe; }
        ++ndef;
      }
      if (may_start >= 0) {
        if (EMIT) { out_may[2 * nmay] = (uint32_t)may_start; out_may[2 * nmay + 1] = (uint32_t)qe; }
        ++nmay;
      }
    }
    // long windows, emitted from their stored masks: each lane turns its own entry's mask
    // words into runs with bit operations (the runs wave_runs would write, at the same
    // places: starts and ends in order, the open run [0, ps) and a run reaching qe), which
    // takes a few instructions per 64 positions instead of a wave-wide pass per entry
    if (EMIT && masks && have && wide) {
      const unsigned long long *mk = masks + woff[p];
      uint32_t sd = 0, ed = 0, sm = 0, em = 0;
      bool cd = ps > 0, cm = ps > 0;
      if (ps > 0) {
        out_def[0] = 0u;
        out_may[0] = 0u;
        sd = sm = 1;
      }
      for (int t = ps, c = 0; t < qe; t += 64, ++c) {
        const int nv = min(64, qe - t);
        const unsigned long long V = nv == 64 ? ~0ull : ((1ull << nv) - 1ull);
        const unsigned long long D = mk[2 * (size_t)c], M = mk[2 * (size_t)c + 1];
        const unsigned long long Dp = (D << 1) | (cd ? 1ull : 0ull), Mp = (M << 1) | (cm ? 1ull : 0ull);
        unsigned long long sD = D & ~Dp, eD = ~D & Dp & V, sM = M & ~Mp, eM = ~M & Mp & V;
        for (; sD; sD &= sD - 1ull) out_def[2 * sd++] = (uint32_t)(t + __builtin_ctzll(sD));
        for (; eD; eD &= eD - 1ull) out_def[2 * ed++ + 1] = (uint32_t)(t + __builtin_ctzll(eD));
        for (; sM; sM &= sM - 1ull) out_may[2 * sm++] = (uint32_t)(t + __builtin_ctzll(sM));
        for (; eM; eM &= eM - 1ull) out_may[2 * em++ + 1] = (uint32_t)(t + __builtin_ctzll(eM));
        cd = (D >> (nv - 1)) & 1ull;
        cm = (M >> (nv - 1)) & 1ull;
      }
      if (cd) out_def[2 * ed++ + 1] = (uint32_t)qe;
      if (cm) out_may[2 * em++ + 1] = (uint32_t)qe;
      ndef = ed;
      nmay = em;
    }
    // long windows otherwise: the whole wave on one entry at a time (all values
    // wave-uniform)
    unsigned long long todo = __ballot(have && wide && !(EMIT && masks));
    while (todo) {
      const int k = __builtin_ctzll(todo);
      todo &= todo - 1ull;
      const int kc = __builtin_amdgcn_readlane(cell, k), kb = __builtin_amdgcn_readlane(beg, k);
      const int ki = __builtin_amdgcn_readlane(i, k), kps = __builtin_amdgcn_readlane(ps, k);
      const int kqe = __builtin_amdgcn_readlane(qe, k);
      const double kuw[3] = {readlane_d(uwi[0], k), readlane_d(uwi[1], k), readlane_d(uwi[2], k)};
      const size_t kp = (size_t)(p0 + k);
      uint32_t *kod = nullptr, *kom = nullptr;
      if (EMIT) {
        kod = runs + 2 * (size_t)cnt[2 * kp];
        kom = runs + 2 * (size_t)cnt[2 * kp + 1];
      }
      unsigned long long *km_ = masks ? masks + woff[kp] : nullptr;
      const SceneDev &ksc = cell_scene(scene, tab, kc);
      const IndSrc<P, COMPACT> src{lists + kb, ksc.ind_mean, COMPACT ? cform : dform, cmean, ksc.n,
                                   cell_first(scene, tab, kc), (size_t)((uint32_t)kb - pbase)};
      uint32_t kd, km, ku, kbd;
      wave_runs<P, MODE, COMPACT>(poses[kc], src, ki, kps, kqe, kuw, src.forms_of(ki), km_, kod, kom, lane, kd, km,
                                  ku, kbd);
      if (lane == k) {
        ndef = kd;
        nmay = km;
        nund = ku;
        nbord = kbd;
      }
    }
    if (!EMIT && have) {
      cnt[2 * (size_t)p] = ndef;
      cnt[2 * (size_t)p + 1] = nmay;
    }
    // undecided pairs of the cell (counted when asked for)
    if (!EMIT && ind_und) wave_add_by_key(ind_und, have ? cell : -1, nund);
    if (MODE == kRunsCount) {
      // borderline decisions: one atomic per wave
      unsigned long long b = nbord;
      for (int off = 32; off > 0; off >>= 1) b += (unsigned long long)__shfl_xor(b, off);
      if (lane == 0 && b) atomicAdd(&counters[kIndBorder], b);
    }
  }
  if (MODE == kRunsWindows) {
    // window statistics: one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
      wmax = max(wmax, (unsigned long long)__shfl_xor(wmax, off));
      wsum += (unsigned long long)__shfl_xor(wsum, off);
    }
    if (lane == 0) {
      atomicMax(&counters[5], wmax);
      atomicAdd(&counters[1], wsum);
    }
  }
}

// Counting pass for long windows (the compact copy in use): the lanes hold 64 consecutive
// entries and walk the union of their windows together, so list position j is the same
// for every lane and its mean and depth forms are scalar loads shared by the wave (the
// wave-wide walk of wave_runs loads them per lane, once for every entry whose window
// holds j).  Entries of different lists in one wave are taken list by list.  Each lane
// counts its runs and stores its long window's masks in the layout of wave_runs.
template <int P>
__global__ __launch_bounds__(256) void k_runs_count_lanes(const uint32_t *__restrict__ pkey,
                                                          const uint32_t *__restrict__ ranges,
                                                          const uint32_t *__restrict__ lists,
                                                          const float4 *__restrict__ cmean,
                                                          const double *__restrict__ cform,
                                                          const PoseForms *__restrict__ poses, int ntiles,
                                                          SceneDev sc, uint32_t pbase, int ng,
                                                          const uint32_t *__restrict__ win,
                                                          const uint32_t *__restrict__ woff,
                                                          unsigned long long *__restrict__ masks,
                                                          uint32_t *__restrict__ cnt,
                                                          const uint32_t *__restrict__ ng_dev,
                                                          unsigned long long *__restrict__ ind_und,
                                                          unsigned long long *__restrict__ counters) {
  using Src = IndSrc<P, true>;
  constexpr int S = Src::S;
  const int lane = threadIdx.x & 63;
  if (ng_dev) ng = min(ng, (int)*ng_dev);
  const int wave0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  const int nwaves = (int)(gridDim.x * (blockDim.x >> 6));
  for (int p0 = wave0 * 64; p0 < ng; p0 += nwaves * 64) {
    const int p = p0 + lane;                       // entry of the group; list position pbase + p
    const bool have = p < ng;
    uint32_t tile = 0;
    int beg = 0, i = 0, ps = 0, qe = 0;
    double uwi[3] = {0.0, 0.0, 0.0}, dfi[2 * S];
#pragma unroll
    for (int k = 0; k < 2 * S; ++k) dfi[k] = 0.0;
    if (have) {
      tile = pkey[(size_t)pbase + p];
      beg = (int)ranges[2 * tile];
      i = (int)(pbase + (uint32_t)p) - beg;
      ps = (int)win[2 * (size_t)p];
      qe = (int)win[2 * (size_t)p + 1];
      const float4 m = cmean[p];
      uwi[0] = m.x;
      uwi[1] = m.y;
      uwi[2] = m.z;
#pragma unroll
      for (int k = 0; k < 2 * S; ++k) dfi[k] = cform[(size_t)p * (2 * S) + k];
    }
    uint32_t ndef = 0, nmay = 0, nund = 0, nbord = 0;
    bool pending = have;
    for (;;) {
      const unsigned long long pend = __ballot(pending);
      if (!pend) break;
      const int l0 = __builtin_ctzll(pend);
      const uint32_t gtile = (uint32_t)__builtin_amdgcn_readlane((int)tile, l0);
      const bool mine = pending && tile == gtile;
      pending = pending && !mine;
      // the union of the group's windows
      int lo = mine ? ps : 0x7fffffff, hi = mine ? qe : 0;
      for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off));
        hi = max(hi, __shfl_xor(hi, off));
      }
      lo = __builtin_amdgcn_readfirstlane(lo);
      hi = __builtin_amdgcn_readfirstlane(hi);
      const int gbeg = __builtin_amdgcn_readlane(beg, l0);
      const int gcell = (int)(gtile / (uint32_t)ntiles);
      const PoseForms &pose = poses[gcell];
      // (the compact copy holds the means and forms by position: the scene's arrays are not read)
      const Src src{lists + gbeg, sc.ind_mean, cform, cmean, sc.n, (size_t)gcell * sc.n, (size_t)((uint32_t)gbeg - pbase)};
      int def_start = (mine && ps > 0) ? 0 : -1;   // open run [0, ps) of certain occluders
      int may_start = def_start;
      uint32_t nd = 0, nm = 0;
      const bool store = mine && masks != nullptr && qe - ps > kWaveWindow;
      unsigned long long *mk = store ? masks + woff[p] : nullptr;
      unsigned long long wd = 0, wm = 0;
      for (int j = lo; j < hi; ++j) {
        double uwj[3];
        src.mean_of(j, uwj);
        const double *dfj = src.forms_of(j);
        if (mine && j >= ps && j < qe) {
          bool bd = false;
          const int ind = j != i ? ind_pair<P, S, true>(pose, uwi, uwj, dfi, dfj, &bd) : 0;
          const bool d1 = ind == 1, m1 = ind != 0;
          nund += ind == 2 ? 1u : 0u;
          nbord += bd ? 1u : 0u;
          if (d1 && def_start < 0) def_start = j;
          if (!d1 && def_start >= 0) {
            ++nd;
            def_start = -1;
          }
          if (m1 && may_start < 0) may_start = j;
          if (!m1 && may_start >= 0) {
            ++nm;
            may_start = -1;
          }
          if (store) {
            const int b = (j - ps) & 63;
            if (d1) wd |= 1ull << b;
            if (m1) wm |= 1ull << b;
            if (b == 63 || j == qe - 1) {
              const int w = (j - ps) >> 6;
              mk[2 * w] = wd;
              mk[2 * w + 1] = wm;
              wd = 0;
              wm = 0;
            }
          }
        }
      }
      if (mine) {
        ndef = nd + (def_start >= 0 ? 1u : 0u);
        nmay = nm + (may_start >= 0 ? 1u : 0u);
      }
    }
    if (have) {
      cnt[2 * (size_t)p] = ndef;
      cnt[2 * (size_t)p + 1] = nmay;
    }
    if (ind_und) wave_add_by_key(ind_und, have ? (int)(tile / (uint32_t)ntiles) : -1, nund);
    unsigned long long b = nbord;
    for (int off = 32; off > 0; off >>= 1) b += (unsigned long long)__shfl_xor(b, off);
    if (lane == 0 && b) atomicAdd(&counters[kIndBorder], b);
  }
}

// ---------------------------------------------------------------------------------
// pixel loop over list segments (one wave per segment of L list positions)
// ---------------------------------------------------------------------------------
// Segment s of list l covers positions [(s - seg_off[l]) L, ...) of the list.  All
// arrays of a launch are relative to its first segment seg0 and its first list entry
// pos0 (a launch covers a chunk of consecutive lists).

struct SegRef {
  int list, beg, n, i0, i1;
};

// Workgroups are handed to the eight XCDs round robin (block b runs on XCD b % 8), and
// each XCD has its own L2.  xcd_block renumbers the blocks so that every XCD takes runs of
// kXcdChunk consecutive logical blocks: the waves of one tile list then share one L2.
// A bijection of [0, nb); the blocks past the last whole round keep their numbers.
constexpr int kXcds = 8;
constexpr int kXcdChunk = 32;

__device__ __forceinline__ int xcd_block(int b, int nb) {
  constexpr int per = kXcds * kXcdChunk;
  if (b >= nb / per * per) return b;
  const int round = b / per, r = b % per;
  return round * per + (r % kXcds) * kXcdChunk + r / kXcds;
}

__device__ __forceinline__ SegRef seg_ref(const uint32_t *__restrict__ ranges, const uint32_t *__restrict__ seg_off,
                                          const uint32_t *__restrict__ seg_tile, int s, int L) {
  SegRef r;
  r.list = (int)seg_tile[s];
  r.beg = (int)ranges[2 * r.list];
  r.n = (int)ranges[2 * r.list + 1] - r.beg;
  r.i0 = (s - (int)seg_off[r.list]) * L;
  r.i1 = min(r.i0 + L, r.n);
  return r;
}

// Rows of the per-pixel running sums (64 doubles each, one per pixel): the lists of a
// launch in order, each a row S(0) = 0 followed by S(1) .. S(n), S(p) the sum over list
// positions [0, p).  A list's first row is at its entry offset in the launch plus its
// index among the launch's lists.
__device__ __forceinline__ size_t row0(const SegRef &r, uint32_t pos0, int list0) {
  return (size_t)((uint32_t)r.beg - pos0) + (size_t)(r.list - list0);
}

// A: per pixel, running sums of log(1 - a_lo) and log(max(1 - a_hi, 2^-60)) over the
// segment (from zero at its start), and the segment totals; the list's first segment
// also writes its zero row.
template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_rot_prefix(const double *__restrict__ recs,
                                                    const uint32_t *__restrict__ ranges,
                                                    const uint32_t *__restrict__ lists,
                                                    const uint32_t *__restrict__ seg_off,
                                                    const uint32_t *__restrict__ seg_tile, int L, int seg0, int nseg,
                                                    uint32_t pos0, int list0, Params prm, double *__restrict__ preL,
                                                    double *__restrict__ preH, double2 *__restrict__ segsum,
                                                    unsigned long long *__restrict__ counters) {
  using R = Rec<P>;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (w >= nseg) return;
  const long long c0 = clock64();
  const SegRef r = seg_ref(ranges, seg_off, seg_tile, seg0 + w, L);
  const int ntiles = prm.ntx * prm.nty;
  const int tile = r.list % ntiles;
  const int tx = tile % prm.ntx, ty = tile / prm.ntx;
  const int col = tx * kTile + (lane & 7), row = ty * kTile + (lane >> 3);
  const bool inimg = col < prm.width && row < prm.height;
  const double uxd = (double)col + 0.5 - prm.cx, uyd = (double)row + 0.5 - prm.cy;
  const float ux = (float)uxd, uy = (float)uyd;
  const uint32_t *items = lists + r.beg;
  const size_t rb = row0(r, pos0, list0) + 1;   // row of S(1)
  // (an empty list has no rows: the padding segments of a planned launch belong to one)
  if (r.i0 == 0 && r.n > 0) {
    preL[(rb - 1) * 64 + lane] = 0.0;
    preH[(rb - 1) * 64 + lane] = 0.0;
  }
  double Ll = 0.0, Lh = 0.0;
  Lookahead la;
  for (int j = r.i0; j < r.i1; ++j) {
    const int k = (j - r.i0) & 63;
    if (k == 0) la.fetch<P>(recs, items, j + lane, r.i1);
    const uint32_t gid = la.gid(k);
    const double *rec = recs + (size_t)gid * R::STRIDE;
    const int type = la.type(k);
    if (inimg && la.kept(k, type, ux, uy)) {
      double alo, ahi;
      alpha_interval<P>(rec, type, uxd, uyd, alo, ahi, exp_table(gid));
      Ll += log(1.0 - alo);
      Lh += log(ahi >= 1.0 ? kZeroFactor : 1.0 - ahi);
    }
    preL[(rb + j) * 64 + lane] = Ll;
    preH[(rb + j) * 64 + lane] = Lh;
  }
  segsum[(size_t)w * 64 + lane] = make_double2(Ll, Lh);
  if (lane == 0) atomicAdd(&counters[6], (unsigned long long)(clock64() - c0));
}

// per list: exclusive running totals of its segments' sums (in place), and the list's
// total of log(1 - a_lo) per pixel (listlo[k][64])
__global__ __launch_bounds__(256) void k_rot_offsets(const uint32_t *__restrict__ seg_off, int list0, int nl, int seg0,
                                                     double2 *__restrict__ segsum, double *__restrict__ listlo) {
  const int lane = threadIdx.x & 63;
  const int k = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (k >= nl) return;
  const int s0 = (int)seg_off[list0 + k] - seg0, s1 = (int)seg_off[list0 + k + 1] - seg0;
  double al = 0.0, ah = 0.0;
  for (int s = s0; s < s1; ++s) {
    const double2 t = segsum[(size_t)s * 64 + lane];
    segsum[(size_t)s * 64 + lane] = make_double2(al, ah);
    al += t.x;
    ah += t.y;
  }
  listlo[(size_t)k * 64 + lane] = al;
}

// Running sums made absolute: each segment's offset (the totals of the list's segments
// in front) added to its positions, so S(p) is one load in the blend.  The sum is the
// one the blend would form itself, so its rounding is unchanged.
__global__ __launch_bounds__(256) void k_rot_absolute(const uint32_t *__restrict__ ranges,
                                                      const uint32_t *__restrict__ seg_off,
                                                      const uint32_t *__restrict__ seg_tile, int L, int seg0,
                                                      int nseg, uint32_t pos0, int list0,
                                                      const double2 *__restrict__ segoff, double *__restrict__ preL,
                                                      double *__restrict__ preH) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (w >= nseg) return;
  const SegRef r = seg_ref(ranges, seg_off, seg_tile, seg0 + w, L);
  if (r.i0 == 0) return;   // the list's first segment: nothing in front
  const double2 o = segoff[(size_t)w * 64 + lane];
  const size_t rb = row0(r, pos0, list0) + 1;
  for (int j = r.i0; j < r.i1; ++j) {
    const size_t x = (rb + j) * 64 + lane;
    preL[x] += o.x;
    preH[x] += o.y;
  }
}

// B1 (k_rot_trans): the transmittance bounds of every (entry, pixel) from the runs
// (absolute: everything in front of the Gaussian), stored as floats rounded outward (T_lo
// down, T_hi up: any T' in [0, T] gives a lower colour form below T a_i c_i, as the alpha
// lower form is below a_i >= 0, and the same above for T_hi), one row per entry in the
// third plane.
// Run counts (then offsets) cnt and the runs are those of the list group that starts at
// list position gbase.
// Every entry's transmittances come from the list's running sums, so any split of a
// list's entries over its K waves gives the same values.  Wave k of the list takes
// positions k, k + K, k + 2K, ...: the waves of a list then advance through the list side
// by side, and the run ends they read (within the entries' Ind windows) lie in one band of
// positions that the L2 of their XCD holds (xcd_block), where contiguous segments would
// spread the reads over the whole list.  The kernel holds few registers, so many waves
// keep their run-end loads in flight together.
// ABS: the running sums were made absolute (k_rot_absolute); otherwise each run end
// adds its segment's offset here.
template <int P, bool ABS>
__global__ __launch_bounds__(256) void k_rot_trans(const double *__restrict__ recs, const uint32_t *__restrict__ ranges,
                                                   const uint32_t *__restrict__ lists,
                                                   const uint32_t *__restrict__ seg_off,
                                                   const uint32_t *__restrict__ seg_tile, int L, int seg0, int nseg,
                                                   uint32_t pos0, uint32_t gbase, const uint32_t *__restrict__ cnt,
                                                   const uint32_t *__restrict__ runs, Params prm,
                                                   const double *__restrict__ preL, const double *__restrict__ preH,
                                                   const double2 *__restrict__ segoff, float2 *__restrict__ tpl,
                                                   unsigned long long *__restrict__ counters,
                                                   const double *__restrict__ listlo, int list0,
                                                   const uint32_t *__restrict__ win) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(
      (int)(xcd_block((int)blockIdx.x, (int)gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (w >= nseg) return;
  const long long c0 = clock64();
  const SegRef r = seg_ref(ranges, seg_off, seg_tile, seg0 + w, L);
  // this wave's positions: sidx + m K for m < nent
  const int sidx = r.i0 / L;
  const int K = r.n > 0 ? (int)(seg_off[r.list + 1] - seg_off[r.list]) : 1;
  const int nent = r.n > sidx ? (r.n - sidx + K - 1) / K : 0;
  const int ntiles = prm.ntx * prm.nty;
  const int tile = r.list % ntiles;
  const int tx = tile % prm.ntx, ty = tile / prm.ntx;
  const int col = tx * kTile + (lane & 7), row = ty * kTile + (lane >> 3);
  const bool inimg = col < prm.width && row < prm.height;
  const float ux = (float)((double)col + 0.5 - prm.cx), uy = (float)((double)row + 0.5 - prm.cy);
  const uint32_t *items = lists + r.beg;
  const size_t rb = row0(r, pos0, list0);          // row of S(0)
  const double nn = (double)(r.n + 2);
  const int sl = (int)seg_off[r.list] - seg0;     // the list's first segment, relative
  // When no pair of the list has a positive lower alpha at any pixel of the tile (every
  // log(1 - a_lo) is 0, so the list's total is exactly 0), every sum over the runs of
  // certain occluders is exactly 0 and their run ends are not read.
  const bool zero_lo = __all(listlo[(size_t)(r.list - list0) * 64 + lane] == 0.0);
  Lookahead la;
  uint32_t cv0 = 0, cv1 = 0, cv2 = 0;   // run offsets of the looked-ahead positions
  uint32_t pv = 0;                      // their Ind window starts
  for (int m = 0; m < nent; ++m) {
    const int k = m & 63;
    const int i = sidx + m * K;
    if (k == 0) {
      const int pl = sidx + (m + lane) * K;   // position looked ahead by this lane
      la.fetch<P>(recs, items, pl, r.n);
      if (pl < r.n) {
        const size_t sl2 = 2 * (size_t)((uint32_t)(r.beg + pl) - gbase);
        cv0 = cnt[sl2];
        cv1 = cnt[sl2 + 1];
        cv2 = cnt[sl2 + 2];
        pv = win[sl2];
      }
    }
    const int type = la.type(k);
    const bool kept = inimg && la.kept(k, type, ux, uy);
    // The list positions [0, ps) before the entry's Ind window are surely (so possibly) in
    // front of it, so T_lo <= prod_{[0, ps)} (1 - a_hi).  When that bound times the number
    // of list entries is below t_min, T_lo is taken as 0 (a lower transmittance, so sound;
    // the lower bound moves by less than t_min over the list) and the runs of possible
    // occluders are not read.
    bool tlo_zero = false;
    if (prm.t_min > 0.0) {
      const uint32_t ps = (uint32_t)__builtin_amdgcn_readlane((int)pv, k);
      if (ps > 0u) {
        double S = preH[(rb + ps) * 64 + lane];
        if (!ABS) S += segoff[(size_t)(sl + (int)(ps - 1) / L) * 64 + lane].y;
        tlo_zero = exp(S + nn * (0x1p-51 * fabs(S) + 0x1p-52)) * (1.0 + 0x1p-50) * nn < prm.t_min;
      }
    }
    // Runs of certain occluders and of possible occluders: the log sum over [a, b) is
    // S(b) - S(a), S(p) in row rb + p (plus, unless ABS, the offset of the segment holding
    // position p - 1; for p = 0 the zero row and the list's first offset, also 0).  Every
    // S(p) is <= 0, so the ends are summed apart, A = sum S(a), B = sum S(b), and
    // |A| + |B| is the sum of the ends' magnitudes that bounds the rounding.
    const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)cv0, k);
    const uint32_t d1 = (uint32_t)__builtin_amdgcn_readlane((int)cv1, k);
    const uint32_t m0 = d1, m1 = (uint32_t)__builtin_amdgcn_readlane((int)cv2, k);
    double A_l = 0.0, B_l = 0.0, A_h = 0.0, B_h = 0.0;
    if (ABS) {
      // many runs per entry: the runs are read 64 at a time (one per lane) and their ends
      // eight runs at a time, so sixteen loads are in flight; the sums are taken in run
      // order.  The run ends are read back with readlane from the lane that loaded them,
      // so every lane takes part (a lane whose pixel is not kept uses none of the sums);
      // entries no lane keeps are skipped as a whole.
      if (!__any(kept)) continue;
      const uint2 *runs2 = reinterpret_cast<const uint2 *>(runs);
      constexpr int kRunGroup = 8;
      // groups of kRunGroup runs; each run end is one load of a row at a wave-uniform
      // address (the lane's pixel is the load's offset).  Lanes past the last run hold the
      // run (0, 0), whose ends are the zero row (u + t <= 63: u < nq <= 64 in steps of 8).
      auto run_sums = [&](const double *rows, uint32_t q0, uint32_t q1, double &A, double &B) {
        for (uint32_t qb = q0; qb < q1; qb += 64) {
          const int nq = (int)min(64u, q1 - qb);
          uint2 abv = make_uint2(0u, 0u);
          if (lane < nq) abv = runs2[qb + lane];
          for (int u = 0; u < nq; u += kRunGroup) {
            double La[kRunGroup], Lb[kRunGroup];
#pragma unroll
            for (int t = 0; t < kRunGroup; ++t) {
              const uint32_t pa = (uint32_t)__builtin_amdgcn_readlane((int)abv.x, u + t);
              const uint32_t pe = (uint32_t)__builtin_amdgcn_readlane((int)abv.y, u + t);
              La[t] = (rows + (size_t)pa * 64)[lane];
              Lb[t] = (rows + (size_t)pe * 64)[lane];
            }
#pragma unroll
            for (int t = 0; t < kRunGroup; ++t) {
              A += La[t];
              B += Lb[t];
            }
          }
        }
      };
      run_sums(preL + rb * 64, d0, zero_lo ? d0 : d1, A_l, B_l);
      // possible occluders' runs, unless no kept lane needs T_lo
      run_sums(preH + rb * 64, m0, __all(!kept || tlo_zero) ? m0 : m1, A_h, B_h);
    } else {
      // few runs per entry: one run at a time, kept lanes only
      if (!kept) continue;
      auto S_at = [&](const double *pre, uint32_t p, int half) -> double {
        const double2 o = segoff[(size_t)(sl + (p > 0 ? (int)(p - 1) / L : 0)) * 64 + lane];
        return pre[(rb + p) * 64 + lane] + (half ? o.y : o.x);
      };
      for (uint32_t q = d0; q < (zero_lo ? d0 : d1); ++q) {
        const uint2 ab = *reinterpret_cast<const uint2 *>(runs + 2 * (size_t)q);
        A_l += S_at(preL, ab.x, 0);
        B_l += S_at(preL, ab.y, 0);
      }
      for (uint32_t q = m0; q < (tlo_zero ? m0 : m1); ++q) {
        const uint2 ab = *reinterpret_cast<const uint2 *>(runs + 2 * (size_t)q);
        A_h += S_at(preH, ab.x, 1);
        B_h += S_at(preH, ab.y, 1);
      }
    }
    if (!kept) continue;
    // Rounding: a stored S(p) is within p u of the exact sum through the roundings of the
    // factors 1 - a (the runs of one set are disjoint, so at most n u over all of them)
    // and within (p + 2) u |S(p)| through the logs and the additions; the sums A and B
    // and the difference add (runs + 1) u (|A| + |B|).  nn 2^-51 (|A| + |B|) + nn 2^-52
    // covers the total, and the factor 1 +- 2^-50 the rounding of exp.
    const double thi = exp((B_l - A_l) + nn * (0x1p-51 * (fabs(A_l) + fabs(B_l)) + 0x1p-52)) * (1.0 + 0x1p-50);
    const double tlo =
        tlo_zero ? 0.0 : exp((B_h - A_h) - nn * (0x1p-51 * (fabs(A_h) + fabs(B_h)) + 0x1p-52)) * (1.0 - 0x1p-50);
    tpl[(rb + 1 + i) * 64 + lane] = make_float2(__double2float_rd(tlo), __double2float_ru(fmin(thi, 1.0)));
  }
  if (lane == 0) atomicAdd(&counters[7], (unsigned long long)(clock64() - c0));
}

// B2 (k_rot_blend): colour forms of every kept pair with its stored transmittances,
// accumulated per segment; the tile's bounds are the sum over its segments.
template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_rot_blend(const double *__restrict__ recs, const uint32_t *__restrict__ ranges,
                                                   const uint32_t *__restrict__ lists,
                                                   const uint32_t *__restrict__ seg_off,
                                                   const uint32_t *__restrict__ seg_tile, int L, int seg0, int nseg,
                                                   uint32_t pos0, int list0, Params prm,
                                                   const float2 *__restrict__ tpl, double *__restrict__ part,
                                                   unsigned long long *__restrict__ counters) {
  using R = Rec<P>;
  using Q = Part<P>;
  constexpr int F = P + 1;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (w >= nseg) return;
  const long long c0 = clock64();
  const SegRef r = seg_ref(ranges, seg_off, seg_tile, seg0 + w, L);
  const int ntiles = prm.ntx * prm.nty;
  const int tile = r.list % ntiles;
  const int tx = tile % prm.ntx, ty = tile / prm.ntx;
  const int col = tx * kTile + (lane & 7), row = ty * kTile + (lane >> 3);
  const bool inimg = col < prm.width && row < prm.height;
  const double uxd = (double)col + 0.5 - prm.cx, uyd = (double)row + 0.5 - prm.cy;
  const float ux = (float)uxd, uy = (float)uyd;
  const uint32_t *items = lists + r.beg;
  const float2 *trow = tpl + (row0(r, pos0, list0) + 1) * 64 + lane;   // entry j: trow[j * 64]
  Acc<P> acc;
  acc_zero<P>(acc);
  unsigned npairs = 0;
  Lookahead la;
  // the next entry's transmittances are loaded while this one is evaluated (rows of
  // entries no lane keeps were not written; their values are not used)
  float2 tn = r.i0 < r.i1 ? trow[(size_t)r.i0 * 64] : make_float2(0.0f, 0.0f);
  for (int j = r.i0; j < r.i1; ++j) {
    const int k = (j - r.i0) & 63;
    if (k == 0) la.fetch<P>(recs, items, j + lane, r.i1);
    const float2 t = tn;
    if (j + 1 < r.i1) tn = trow[(size_t)(j + 1) * 64];
    const uint32_t gid = la.gid(k);
    const double *rec = recs + (size_t)gid * R::STRIDE;
    const int type = la.type(k);
    if (!(inimg && la.kept(k, type, ux, uy))) continue;
    double alo, ahi;
    pair_contrib<P>(rec, type, uxd, uyd, (double)t.x, (double)t.y, acc, alo, ahi, exp_table(gid));
    ++npairs;
  }
  unsigned c = npairs;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  double *q = part + (size_t)w * Q::NF * 64 + lane;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
#pragma unroll
    for (int j = 0; j < F; ++j) {
      q[(Q::LO + ch * F + j) * 64] = acc.lo[ch][j];
      q[(Q::HI + ch * F + j) * 64] = acc.hi[ch][j];
    }
    q[(Q::IHI + ch) * 64] = acc.ihi[ch];
  }
  float2 mg;
  mg.x = acc.magl;
  mg.y = acc.magh;
  q[Q::MAG * 64] = __builtin_bit_cast(double, mg);
  q[Q::CNT * 64] = (double)c;
  if (lane == 0) atomicAdd(&counters[7], (unsigned long long)(clock64() - c0));
}

// per list and colour channel (three waves): sum of the segments' colour sums, then the
// pixel bounds
template <int P>
__global__ __launch_bounds__(192) void k_rot_merge(const uint32_t *__restrict__ ranges,
                                                   const uint32_t *__restrict__ seg_off, int list0, int seg0,
                                                   const double *__restrict__ part, Params prm,
                                                   float *__restrict__ out_lo, float *__restrict__ out_hi,
                                                   unsigned long long *__restrict__ counters) {
  using Q = Part<P>;
  constexpr int F = P + 1;
  const int lane = threadIdx.x & 63;
  const int ch = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int ntiles = prm.ntx * prm.nty;
  const int list = list0 + (int)blockIdx.x;
  const int cell = list / ntiles, tile = list % ntiles;
  const int tx = tile % prm.ntx, ty = tile / prm.ntx;
  const int col = tx * kTile + (lane & 7), row = ty * kTile + (lane >> 3);
  const bool inimg = col < prm.width && row < prm.height;
  const int s0 = (int)seg_off[list] - seg0, s1 = (int)seg_off[list + 1] - seg0;
  double lo[F], hi[F], ihi = 0.0;
#pragma unroll
  for (int j = 0; j < F; ++j) { lo[j] = 0.0; hi[j] = 0.0; }
  float magl = 0.0f, magh = 0.0f;
  unsigned long long cn = 0;
  for (int s = s0; s < s1; ++s) {
    const double *q = part + (size_t)s * Q::NF * 64 + lane;
#pragma unroll
    for (int j = 0; j < F; ++j) {
      lo[j] += q[(Q::LO + ch * F + j) * 64];
      hi[j] += q[(Q::HI + ch * F + j) * 64];
    }
    ihi += q[(Q::IHI + ch) * 64];
    const float2 mg = __builtin_bit_cast(float2, q[Q::MAG * 64]);
    magl = (magl + mg.x) * (1.0f + 4.0f * kU32);
    magh = (magh + mg.y) * (1.0f + 4.0f * kU32);
    cn += (unsigned long long)q[Q::CNT * 64];
  }
  if (ch == 0 && lane == 0 && cn) atomicAdd(&counters[0], cn);
  if (!inimg) return;
  const int n = (int)(ranges[2 * list + 1] - ranges[2 * list]);
  const size_t img = (size_t)cell * prm.width * prm.height;
  // widened by n 2^-59: each lower transmittance that should be 0 is at most 2^-60 (with
  // its rounding), and colours and alphas are at most 1
  write_channel<P>(lo, hi, ihi, magl, magh, (double)(n + 2 * (s1 - s0)), prm.E + (double)n * 0x1p-59, 0.0,
                   out_lo, out_hi, (img + (size_t)row * prm.width + col) * 3 + ch);
}

// ---------------------------------------------------------------------------------
hipError_t launch_chunk_boxes(const Workspace &ws, const uint32_t *lists, const SceneDev &sc, int ntiles, size_t npos,
                              double *cbox, hipStream_t s) {
  const size_t nwaves = (npos + 63) / 64;
  if (nwaves == 0) return hipSuccess;
  hipLaunchKernelGGL(k_chunk_boxes, dim3((unsigned)((nwaves + 3) / 4)), dim3(256), 0, s, ws.pair_key, lists, ws.dint,
                     sc, ntiles, npos, cbox, ws.tab);
  return hipGetLastError();
}

hipError_t launch_list_box(const Workspace &ws, const uint32_t *lists, const PoseForms *poses, int nlists, int ntiles,
                           const SceneDev &sc, hipStream_t s) {
  hipLaunchKernelGGL(k_list_box, dim3(nlists), dim3(256), 0, s, ws.tile_range, lists, poses, sc, ntiles, ws.lbox,
                     ws.tab);
  return hipGetLastError();
}

template <int P, int MODE, bool COMPACT>
static hipError_t launch_runs_pm(const Workspace &ws, const uint32_t *lists, const PoseForms *poses_dev, int ntiles,
                                 const SceneDev &sc, uint32_t pbase, int ng, int window_mode,
                                 unsigned long long *masks, const DevCounts &dc, hipStream_t s) {
  // 64 entries per wave and step; at most 8192 blocks, each looping over its share
  const dim3 grid((unsigned)std::min<size_t>(((size_t)ng + 255) / 256, 8192)), block(256);
  hipLaunchKernelGGL((k_runs<P, MODE, COMPACT>), grid, block, 0, s, ws.pair_key, ws.tile_range, lists, ws.dint,
                     ws.dform, (const float4 *)ws.cmean, ws.cform, ws.lbox, poses_dev, ntiles, sc, pbase, ng,
                     window_mode, ws.win, ws.woff, masks, ws.run_cnt, ws.runs, ws.counters, dc.entries, dc.runs_cap,
                     dc.ind_und, ws.tab, dc.cbox);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_runs_p(const Workspace &ws, const uint32_t *lists, const PoseForms *poses_dev, int ntiles,
                                const SceneDev &sc, uint32_t pbase, int ng, int window_mode, int mode,
                                unsigned long long *masks, bool compact, const DevCounts &dc, hipStream_t s) {
  if (mode == kRunsWindows)
    return launch_runs_pm<P, kRunsWindows, false>(ws, lists, poses_dev, ntiles, sc, pbase, ng, window_mode, masks, dc,
                                                  s);
  if (compact) {
    if (mode == kRunsCount) {
      const dim3 grid((unsigned)std::min<size_t>(((size_t)ng + 255) / 256, 8192)), block(256);
      hipLaunchKernelGGL(k_runs_count_lanes<P>, grid, block, 0, s, ws.pair_key, ws.tile_range, lists,
                         (const float4 *)ws.cmean, ws.cform, poses_dev, ntiles, sc, pbase, ng, ws.win, ws.woff, masks,
                         ws.run_cnt, dc.entries, dc.ind_und, ws.counters);
      return hipGetLastError();
    }
    return launch_runs_pm<P, kRunsEmit, true>(ws, lists, poses_dev, ntiles, sc, pbase, ng, window_mode, masks, dc, s);
  }
  if (mode == kRunsCount)
    return launch_runs_pm<P, kRunsCount, false>(ws, lists, poses_dev, ntiles, sc, pbase, ng, window_mode, masks, dc,
                                                s);
  return launch_runs_pm<P, kRunsEmit, false>(ws, lists, poses_dev, ntiles, sc, pbase, ng, window_mode, masks, dc, s);
}

template <int P>
static hipError_t launch_ind_gather_p(const Workspace &ws, const uint32_t *lists, const SceneDev &sc, int ntiles,
                                      uint32_t pbase, int ng, const uint32_t *ng_dev, hipStream_t s) {
  hipLaunchKernelGGL(k_ind_gather<P>, dim3((unsigned)(((size_t)ng + 255) / 256)), dim3(256), 0, s, ws.pair_key,
                     lists, ws.dform, sc, ntiles, pbase, ng, ng_dev, (float4 *)ws.cmean, ws.cform, ws.tab);
  return hipGetLastError();
}

hipError_t launch_ind_gather(int P, const Workspace &ws, const uint32_t *lists, const SceneDev &sc, int ntiles,
                             uint32_t pbase, int ng, hipStream_t s, const uint32_t *ng_dev) {
  if (ng <= 0) return hipSuccess;
  switch (P) {
    case 0: return launch_ind_gather_p<0>(ws, lists, sc, ntiles, pbase, ng, ng_dev, s);
    case 1: return launch_ind_gather_p<1>(ws, lists, sc, ntiles, pbase, ng, ng_dev, s);
    case 2: return launch_ind_gather_p<2>(ws, lists, sc, ntiles, pbase, ng, ng_dev, s);
    case 3: return launch_ind_gather_p<3>(ws, lists, sc, ntiles, pbase, ng, ng_dev, s);
    case 4: return launch_ind_gather_p<4>(ws, lists, sc, ntiles, pbase, ng, ng_dev, s);
    case 5: return launch_ind_gather_p<5>(ws, lists, sc, ntiles, pbase, ng, ng_dev, s);
    case 6: return launch_ind_gather_p<6>(ws, lists, sc, ntiles, pbase, ng, ng_dev, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_runs(int P, const Workspace &ws, const uint32_t *lists, const PoseForms *poses_dev, int ntiles,
                       const SceneDev &sc, uint32_t pbase, int ng, int window_mode, int mode,
                       unsigned long long *masks, bool compact, hipStream_t s, const DevCounts &dc) {
  if (ng <= 0) return hipSuccess;
  switch (P) {
#define AR_RUNS_CASE(PP) \
    case PP: return launch_runs_p<PP>(ws, lists, poses_dev, ntiles, sc, pbase, ng, window_mode, mode, masks, compact, \
                                      dc, s);
    AR_RUNS_CASE(0) AR_RUNS_CASE(1) AR_RUNS_CASE(2) AR_RUNS_CASE(3) AR_RUNS_CASE(4) AR_RUNS_CASE(5) AR_RUNS_CASE(6)
#undef AR_RUNS_CASE
  }
  return hipErrorInvalidValue;
}

template <int P>
static hipError_t launch_rot_p(const Workspace &ws, const uint32_t *lists, const RotChunk &c, const Params &prm,
                               float *lo, float *hi, hipStream_t s) {
  const dim3 blk(256), grid((unsigned)((c.nseg + 3) / 4));
  double *preL = ws.pre, *preH = ws.pre + ws.cap_pre * kTilePix;
  if (c.nseg > 0) {
    hipLaunchKernelGGL(k_rot_prefix<P>, grid, blk, 0, s, ws.rec, ws.tile_range, lists, ws.seg_off, ws.seg_tile, c.L,
                       c.seg0, c.nseg, c.pos0, c.list0, prm, preL, preH, (double2 *)ws.segsum, ws.counters);
    hipLaunchKernelGGL(k_rot_offsets, dim3((unsigned)((c.nl + 3) / 4)), blk, 0, s, ws.seg_off, c.list0, c.nl, c.seg0,
                       (double2 *)ws.segsum, ws.listlo);
    float2 *tpl = reinterpret_cast<float2 *>(ws.pre + 2 * ws.cap_pre * kTilePix);
    if (c.absolute) {
      hipLaunchKernelGGL(k_rot_absolute, grid, blk, 0, s, ws.tile_range, ws.seg_off, ws.seg_tile, c.L, c.seg0, c.nseg,
                         c.pos0, c.list0, (const double2 *)ws.segsum, preL, preH);
      hipLaunchKernelGGL((k_rot_trans<P, true>), grid, blk, 0, s, ws.rec, ws.tile_range, lists, ws.seg_off,
                         ws.seg_tile, c.L, c.seg0, c.nseg, c.pos0, c.gbase, ws.run_cnt, ws.runs, prm, preL,
                         preH, (const double2 *)ws.segsum, tpl, ws.counters, ws.listlo, c.list0, ws.win);
    } else {
      hipLaunchKernelGGL((k_rot_trans<P, false>), grid, blk, 0, s, ws.rec, ws.tile_range, lists, ws.seg_off,
                         ws.seg_tile, c.L, c.seg0, c.nseg, c.pos0, c.gbase, ws.run_cnt, ws.runs, prm, preL, preH,
                         (const double2 *)ws.segsum, tpl, ws.counters, ws.listlo, c.list0, ws.win);
    }
    hipLaunchKernelGGL(k_rot_blend<P>, grid, blk, 0, s, ws.rec, ws.tile_range, lists, ws.seg_off, ws.seg_tile, c.L,
                       c.seg0, c.nseg, c.pos0, c.list0, prm, (const float2 *)tpl, ws.part, ws.counters);
  }
  hipLaunchKernelGGL(k_rot_merge<P>, dim3((unsigned)c.nl), dim3(192), 0, s, ws.tile_range, ws.seg_off, c.list0, c.seg0,
                     ws.part, prm, lo, hi, ws.counters);
  return hipGetLastError();
}

hipError_t launch_raster_general(int P, const Workspace &ws, const uint32_t *lists, const RotChunk &c,
                                 const Params &prm, float *lo, float *hi, hipStream_t s) {
  switch (P) {
    case 0: return launch_rot_p<0>(ws, lists, c, prm, lo, hi, s);
    case 1: return launch_rot_p<1>(ws, lists, c, prm, lo, hi, s);
    case 2: return launch_rot_p<2>(ws, lists, c, prm, lo, hi, s);
    case 3: return launch_rot_p<3>(ws, lists, c, prm, lo, hi, s);
    case 4: return launch_rot_p<4>(ws, lists, c, prm, lo, hi, s);
    case 5: return launch_rot_p<5>(ws, lists, c, prm, lo, hi, s);
    case 6: return launch_rot_p<6>(ws, lists, c, prm, lo, hi, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ar
