// Binning of Gaussians to 8x8 pixel tiles and the per-pixel BlendInd loop, gfx950.
//
// Binning keeps Gaussian i for tile t when the pruning test passes at the rectangle
// of the tile's pixel centres (the same float32 arithmetic as the per-pixel test, so
// by monotonicity of rounding every Gaussian a pixel keeps is in its tile's list).
// Lists are emitted in depth-rank order and sorted stably by tile id.
//
// The pixel loop for pose boxes without rotation ("translation" path): the depth
// order is the same at every pose (Ind(d_i - d_j) is exact: d_i - d_j does not depend
// on the pose), so BlendInd's transmittance of Gaussian i is the product of (1 - a_j)
// over the Gaussians strictly in front, i.e. a prefix product in depth order with
// equal depths sharing one value (the V and T steps of Alg. BlendInd):
//     T_hi[i] = prod_{front} (1 - a_lo[j]),   T_lo[i] = prod_{front} (1 - a_hi[j]).
// Colour (the pc step) is accumulated as linear forms in FP64:
//     lo: sum_i c_i T_lo[i] a_i^lower(e),   hi: sum_i c_i T_hi[i] a_i^upper(e)
// plus the interval upper sum sum_i c_i T_hi[i] a_hi[i].
//
// Work decomposition: each tile's depth-ordered list is cut into segments of L list
// positions (cuts moved to the next depth change so ties never straddle a cut); one
// wave per segment, one lane per pixel, accumulates with transmittances starting at 1
// and writes its partial sums and transmittance products.  A merge kernel combines a
// tile's segments front to back (the blend of a concatenation is the blend of the
// front part plus its transmittance times the blend of the back part).  Equal-length
// segments keep every wave's work the same whatever the tile's list length.  Once every
// pixel's upper transmittance inside a segment is below t_min the segment stops; the
// remaining Gaussians of the tile can add at most that transmittance (scaled by the one
// in front), which the merge adds to the upper bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "ar_internal.h"
#include "ar_blend.h"

namespace ar {

// ---------------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------------
__device__ __forceinline__ float tile_dist2(const float *mu, int tx, int ty, const Params &prm) {
  const int x0 = tx * prm.tile, y0 = ty * prm.tile;
  const int x1 = min(x0 + prm.tile, prm.width) - 1, y1 = min(y0 + prm.tile, prm.height) - 1;
  const float ux0 = (float)((double)x0 + 0.5 - prm.cx), ux1 = (float)((double)x1 + 0.5 - prm.cx);
  const float uy0 = (float)((double)y0 + 0.5 - prm.cy), uy1 = (float)((double)y1 + 0.5 - prm.cy);
  return dist2_rect(mu, ux0, ux1, uy0, uy1);
}

// Binning of global item r (depth-rank order; perm[r] = cell * n_cell + gid, or the
// cell's first item + gid when the cells render different scenes: item_off) to the lists
// cell * ntiles + tile.  Small inputs: one wave per item, the lanes walk the tile
// rectangle 64 tiles at a time and a ballot gives each kept tile its slot.  Large
// inputs (many cells): one thread per item walking its rectangle.  Both emit an item's
// tiles in row-major order at [counts[r], counts[r + 1]).
// cap (emitting, planned launches): when the scanned total counts[n_total] exceeds it,
// nothing is written and overflow[0] is set (the caller renders again with more room).
template <int P, bool EMIT>
__global__ __launch_bounds__(256) void k_bin(const double *__restrict__ recs, const int32_t *__restrict__ rect,
                                             const uint32_t *__restrict__ perm, int n_total, int n_cell, Params prm,
                                             uint32_t *__restrict__ counts, uint32_t *__restrict__ pkey,
                                             uint32_t *__restrict__ pval, uint32_t cap,
                                             unsigned long long *__restrict__ overflow,
                                             const uint32_t *__restrict__ item_off, int ncells) {
  using R = Rec<P>;
  const int lane = threadIdx.x & 63;
  const int r = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (r >= n_total) return;
  if (EMIT && cap && counts[n_total] > cap) {
    if (r == 0 && lane == 0) overflow[0] = 1ull;
    return;
  }
  const uint32_t gid = perm[r];
  const uint32_t lbase = (uint32_t)item_cell(item_off, ncells, n_cell, gid) * (uint32_t)(prm.ntx * prm.nty);
  const double *rec = recs + (size_t)gid * R::STRIDE;
  const int type = rec_type<P>(rec);
  const int32_t *rc = rect + 4 * (size_t)gid;
  uint32_t c = 0;
  const uint32_t off = EMIT ? counts[r] : 0u;
  if (type != kDropped && rc[0] <= rc[2] && rc[1] <= rc[3]) {
    const float *mu = rec_prune<P>(rec);
    const float r2 = mu[4];
    const int w = rc[2] - rc[0] + 1;
    const int total = w * (rc[3] - rc[1] + 1);
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int i0 = 0; i0 < total; i0 += 64) {
      const int i = i0 + lane;
      const int tx = rc[0] + i % w, ty = rc[1] + i / w;
      const bool keep = i < total && ((type == kWild) || (tile_dist2(mu, tx, ty, prm) <= r2));
      const uint64_t bal = __ballot(keep);
      if (EMIT && keep) {
        const uint32_t pos = off + c + (uint32_t)__popcll(bal & below);
        pkey[pos] = lbase + (uint32_t)(ty * prm.ntx + tx);
        pval[pos] = gid;
      }
      c += (uint32_t)__popcll(bal);
    }
  }
  if (!EMIT && lane == 0) counts[r] = c;
}

template <int P, bool EMIT>
__global__ __launch_bounds__(256) void k_bin_thread(const double *__restrict__ recs, const int32_t *__restrict__ rect,
                                                    const uint32_t *__restrict__ perm, int n_total, int n_cell,
                                                    Params prm, uint32_t *__restrict__ counts,
                                                    uint32_t *__restrict__ pkey, uint32_t *__restrict__ pval,
                                                    uint32_t cap, unsigned long long *__restrict__ overflow,
                                                    const uint32_t *__restrict__ item_off, int ncells) {
  using R = Rec<P>;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_total) return;
  if (EMIT && cap && counts[n_total] > cap) {
    if (r == 0) overflow[0] = 1ull;
    return;
  }
  const uint32_t gid = perm[r];
  const uint32_t lbase = (uint32_t)item_cell(item_off, ncells, n_cell, gid) * (uint32_t)(prm.ntx * prm.nty);
  const double *rec = recs + (size_t)gid * R::STRIDE;
  const int type = rec_type<P>(rec);
  const int32_t *rc = rect + 4 * (size_t)gid;
  uint32_t c = 0;
  const uint32_t off = EMIT ? counts[r] : 0u;
  if (type != kDropped && rc[0] <= rc[2] && rc[1] <= rc[3]) {
    const float *mu = rec_prune<P>(rec);
    const float r2 = mu[4];
    for (int ty = rc[1]; ty <= rc[3]; ++ty)
      for (int tx = rc[0]; tx <= rc[2]; ++tx) {
        const bool keep = (type == kWild) || (tile_dist2(mu, tx, ty, prm) <= r2);
        if (keep) {
          if (EMIT) {
            pkey[off + c] = lbase + (uint32_t)(ty * prm.ntx + tx);
            pval[off + c] = gid;
          }
          ++c;
        }
      }
  }
  if (!EMIT) counts[r] = c;
}

__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_tile_ranges(const uint32_t *__restrict__ keys, int npairs, uint32_t *__restrict__ ranges,
                              uint32_t nlists) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const uint32_t t = keys[p];
  if (t >= nlists) return;
  if (p == 0 || keys[p - 1] != t) ranges[2 * t] = (uint32_t)p;
  if (p == npairs - 1 || keys[p + 1] != t) ranges[2 * t + 1] = (uint32_t)(p + 1);
}

constexpr int kBinWaveMax = 65536;   // up to this many items: one wave per item

template <int P>
static hipError_t launch_bin_p(const Workspace &ws, int n_total, int n_cell, const Params &prm, bool emit,
                               uint32_t cap, hipStream_t s) {
  unsigned long long *ovf = ws.counters + kOverflow;
  if (n_total <= kBinWaveMax) {
    const dim3 grid((unsigned)((n_total + 3) / 4));   // four waves (items) per block
    if (emit)
      hipLaunchKernelGGL((k_bin<P, true>), grid, dim3(256), 0, s, ws.rec, ws.rect, ws.perm, n_total, n_cell, prm,
                         ws.count, ws.pair_key, ws.pair_val, cap, ovf, ws.tab_off, ws.tab_cells);
    else
      hipLaunchKernelGGL((k_bin<P, false>), grid, dim3(256), 0, s, ws.rec, ws.rect, ws.perm, n_total, n_cell, prm,
                         ws.count, ws.pair_key, ws.pair_val, 0u, ovf, ws.tab_off, ws.tab_cells);
  } else {
    const dim3 grid((unsigned)((n_total + 255) / 256));
    if (emit)
      hipLaunchKernelGGL((k_bin_thread<P, true>), grid, dim3(256), 0, s, ws.rec, ws.rect, ws.perm, n_total, n_cell,
                         prm, ws.count, ws.pair_key, ws.pair_val, cap, ovf, ws.tab_off, ws.tab_cells);
    else
      hipLaunchKernelGGL((k_bin_thread<P, false>), grid, dim3(256), 0, s, ws.rec, ws.rect, ws.perm, n_total, n_cell,
                         prm, ws.count, ws.pair_key, ws.pair_val, 0u, ovf, ws.tab_off, ws.tab_cells);
  }
  return hipGetLastError();
}

static hipError_t launch_bin(int P, const Workspace &ws, int n_total, int n_cell, const Params &prm, bool emit,
                             uint32_t cap, hipStream_t s) {
  switch (P) {
    case 0: return launch_bin_p<0>(ws, n_total, n_cell, prm, emit, cap, s);
    case 1: return launch_bin_p<1>(ws, n_total, n_cell, prm, emit, cap, s);
    case 2: return launch_bin_p<2>(ws, n_total, n_cell, prm, emit, cap, s);
    case 3: return launch_bin_p<3>(ws, n_total, n_cell, prm, emit, cap, s);
    case 4: return launch_bin_p<4>(ws, n_total, n_cell, prm, emit, cap, s);
    case 5: return launch_bin_p<5>(ws, n_total, n_cell, prm, emit, cap, s);
    case 6: return launch_bin_p<6>(ws, n_total, n_cell, prm, emit, cap, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_count_tiles(int P, const Workspace &ws, int n_total, int n_cell, const Params &prm, hipStream_t s) {
  return launch_bin(P, ws, n_total, n_cell, prm, false, 0u, s);
}

hipError_t launch_emit_tiles(int P, const Workspace &ws, int n_total, int n_cell, const Params &prm, hipStream_t s,
                             uint32_t cap) {
  return launch_bin(P, ws, n_total, n_cell, prm, true, cap, s);
}

// keys >= nlists (the padding of a planned launch, sorted to the end) belong to no list
hipError_t launch_tile_ranges(const uint32_t *keys, int npairs, uint32_t *ranges, int ntiles, hipStream_t s) {
  const size_t m = 2 * (size_t)ntiles + 2;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, ranges, m, 0u);
  if (npairs > 0)
    hipLaunchKernelGGL(k_tile_ranges, dim3((npairs + 255) / 256), dim3(256), 0, s, keys, npairs, ranges,
                       (uint32_t)ntiles);
  return hipGetLastError();
}

// p[i] = v for *n_dev <= i < cap (the unused tail of a planned launch's buffer)
__global__ void k_fill_tail_u32(uint32_t *__restrict__ p, const uint32_t *__restrict__ n_dev, size_t cap, uint32_t v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cap && i >= (size_t)*n_dev) p[i] = v;
}

hipError_t launch_fill_tail(uint32_t *p, const uint32_t *n_dev, size_t cap, uint32_t v, hipStream_t s) {
  if (cap == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_tail_u32, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, p, n_dev, cap, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// translation pixel loop
// ---------------------------------------------------------------------------------
// first list position >= p that starts a new depth value (or n)
__device__ __forceinline__ int cut_at(const uint32_t *__restrict__ list, const uint64_t *__restrict__ keys, int n, int p) {
  if (p <= 0) return 0;
  if (p >= n) return n;
  uint64_t prev = keys[list[p - 1]];
  while (p < n) {
    const uint64_t k = keys[list[p]];
    if (k != prev) break;
    prev = k;
    ++p;
  }
  return p;
}

int part_fields(int P) { return 6 * (P + 1) + 8; }

// Segments: tile t's list is cut into ceil(n_t / L) pieces of L positions, once for each
// of the tile's nsub wave blocks (block-major: block b's pieces follow block b - 1's).
__global__ void k_seg_count(const uint32_t *__restrict__ ranges, int ntiles, int L, int nsub,
                            uint32_t *__restrict__ seg_off) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntiles) {
    const uint32_t n = ranges[2 * t + 1] - ranges[2 * t];
    seg_off[t] = (n + (uint32_t)L - 1u) / (uint32_t)L * (uint32_t)nsub;
  } else if (t == ntiles) {
    seg_off[t] = 0u;
  }
}

// seg_off (scanned): first segment of each tile, then the total; seg_tile[s] = tile of s
// cap (planned launches): no entry at or past it is written; a total above it sets
// overflow[0]
__global__ void k_seg_map(const uint32_t *__restrict__ seg_off, int ntiles, uint32_t *__restrict__ seg_tile,
                          uint32_t cap, unsigned long long *__restrict__ overflow) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  if (cap && t == 0 && seg_off[ntiles] > cap) overflow[0] = 1ull;
  const uint32_t e = cap ? min(seg_off[t + 1], cap) : seg_off[t + 1];
  for (uint32_t s = seg_off[t]; s < e; ++s) seg_tile[s] = (uint32_t)t;
}

// One wave per segment, one lane per pixel of the segment's 8x8 block: the whole tile,
// or with 16x16 tiles the block the segment belongs to (the four blocks of a tile walk
// the same list, each with its own pixels; the per-pixel pruning test drops the entries
// that miss a block).  The segment's cut points are moved to the next depth change, so a
// group of equal depths is never split.  Transmittances start at 1; the merge scales by
// the product in front.
template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_raster_seg(const double *__restrict__ recs, const uint64_t *__restrict__ keys,
                                                    const uint32_t *__restrict__ ranges,
                                                    const uint32_t *__restrict__ lists,
                                                    const uint32_t *__restrict__ seg_off,
                                                    const uint32_t *__restrict__ seg_tile, int L, int nlists,
                                                    Params prm, double *__restrict__ part) {
  using R = Rec<P>;
  using Q = Part<P>;
  constexpr int F = P + 1;
  const int lane = threadIdx.x & 63;
  const int ntiles = prm.ntx * prm.nty;
  const int s = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (s >= (int)seg_off[nlists]) return;
  const int list = (int)seg_tile[s];           // cell * ntiles + tile
  const int nsub = tile_subs(prm), side = prm.tile / kTile;
  const int s0 = (int)seg_off[list];
  const int nch = ((int)seg_off[list + 1] - s0) / nsub;   // pieces per block
  const int sub = (s - s0) / nch, i = s - s0 - sub * nch;
  const int tile = list % ntiles;
  const int tx = tile % prm.ntx, ty = tile / prm.ntx;
  const int col = tx * prm.tile + (sub % side) * kTile + (lane & 7);
  const int row = ty * prm.tile + (sub / side) * kTile + (lane >> 3);
  const bool inimg = col < prm.width && row < prm.height;
  const double uxd = (double)col + 0.5 - prm.cx, uyd = (double)row + 0.5 - prm.cy;
  const float ux = (float)uxd, uy = (float)uyd;
  const int beg = (int)ranges[2 * list];
  const int n = (int)ranges[2 * list + 1] - beg;
  const uint32_t *items = lists + beg;
  const int p0 = cut_at(items, keys, n, i * L);
  // a block wholly outside the image (right or bottom edge of a 16x16 tile) walks nothing
  const int p1 = __any(inimg) ? cut_at(items, keys, n, (i + 1) * L) : p0;

  Acc<P> acc;
  acc_zero<P>(acc);
  double tl_lo = 1.0, tl_hi = 1.0;   // transmittance of the segment so far
  double tg_lo = 1.0, tg_hi = 1.0;   // ... in front of the current depth value
  uint64_t prev_key = ~0ull;
  bool stop = false;
  unsigned npairs = 0;
  // item, key and pruning data of the next 64 list positions, fetched ahead
  Lookahead la;
  for (int p = p0; p < p1; ++p) {
    const int k = (p - p0) & 63;
    if (k == 0) la.fetch<P>(recs, items, p + lane, p1, keys);
    const uint32_t gid = la.gid(k);
    const uint64_t key = la.key(k);
    if (key != prev_key) {
      // everything from here on lies behind the processed Gaussians
      if (prm.t_min > 0.0 && __all(!inimg || tl_hi < prm.t_min)) {
        stop = true;
        break;
      }
      tg_lo = tl_lo;
      tg_hi = tl_hi;
      prev_key = key;
    }
    const double *rec = recs + (size_t)gid * R::STRIDE;
    const int type = la.type(k);
    const bool kept = inimg && la.kept(k, type, ux, uy);
    // alpha under the lane mask, accumulation for every lane (zero when not kept)
    PairAlpha<P> pa;
    pair_alpha<P>(rec, type, kept, uxd, uyd, pa, exp_table(gid));
    acc_pair<P>(acc, rec, pa, tg_lo, tg_hi);
    tl_lo *= 1.0 - pa.a_hi;
    tl_hi *= 1.0 - pa.a_lo;
    npairs += kept ? 1u : 0u;
  }
  unsigned cnt = npairs;
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);

  double *q = part + (size_t)s * Q::NF * 64 + lane;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int j = 0; j < F; ++j) {
      q[(Q::LO + c * F + j) * 64] = acc.lo[c][j];
      q[(Q::HI + c * F + j) * 64] = acc.hi[c][j];
    }
    q[(Q::IHI + c) * 64] = acc.ihi[c];
  }
  q[Q::TLO * 64] = tl_lo;
  q[Q::THI * 64] = tl_hi;
  float2 mg;
  mg.x = acc.magl;
  mg.y = acc.magh;
  q[Q::MAG * 64] = __builtin_bit_cast(double, mg);
  q[Q::STOP * 64] = stop ? 1.0 : 0.0;
  q[Q::CNT * 64] = (double)cnt;
}

// Waves per colour channel in the merge: each combines a quarter of the tile's segments,
// then the quarters are combined in order.
constexpr int kMergeWaves = 4;

// Front-to-back composition of consecutive segments (or runs of segments):
//   acc += T * acc_s,  T *= T_s  (lower with T_lo, upper with T_hi).
// A segment that stopped early ends the tile: everything behind its stop point adds at
// most T_hi (in front) * T_hi (segment at the stop).
template <int P>
struct MergeAcc {
  double lo[P + 1], hi[P + 1], ihi;
  double T_lo, T_hi, extra;
  float magl, magh;
  int stopped;
  unsigned cnt;

  __device__ __forceinline__ void init() {
#pragma unroll
    for (int j = 0; j <= P; ++j) { lo[j] = 0.0; hi[j] = 0.0; }
    ihi = 0.0;
    T_lo = 1.0;
    T_hi = 1.0;
    extra = 0.0;
    magl = 0.0f;
    magh = 0.0f;
    stopped = 0;
    cnt = 0;
  }
  // append b (the part right behind this one)
  __device__ __forceinline__ void append(const MergeAcc &b) {
    if (stopped) return;
#pragma unroll
    for (int j = 0; j <= P; ++j) {
      lo[j] = fma(T_lo, b.lo[j], lo[j]);
      hi[j] = fma(T_hi, b.hi[j], hi[j]);
    }
    ihi = fma(T_hi, b.ihi, ihi);
    magl = fmaf((float)T_lo, b.magl, magl) * (1.0f + 4.0f * kU32);
    magh = fmaf((float)T_hi, b.magh, magh) * (1.0f + 4.0f * kU32);
    cnt += b.cnt;
    if (b.stopped) {
      extra = T_hi * b.extra * (1.0 + 0x1p-50);
      stopped = 1;
      return;
    }
    T_lo *= b.T_lo;
    T_hi *= b.T_hi;
  }
};

// One workgroup per 8x8 block of a tile: kMergeWaves waves per colour channel, each composing a
// contiguous quarter of the tile's segments (loads of four segments issued together),
// then wave 0 of the channel composes the quarters in order and writes the pixel bounds.
template <int P>
__global__ __launch_bounds__(192 * kMergeWaves) void k_merge(const uint32_t *__restrict__ ranges,
                                                             const uint32_t *__restrict__ seg_off,
                                                             const double *__restrict__ part, Params prm,
                                                             float *__restrict__ out_lo, float *__restrict__ out_hi,
                                                             unsigned long long *__restrict__ counters) {
  using Q = Part<P>;
  using M = MergeAcc<P>;
  constexpr int F = P + 1;
  __shared__ M red[3][kMergeWaves - 1][64];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int c = wid / kMergeWaves, w = wid % kMergeWaves;   // colour channel, quarter
  const int ntiles = prm.ntx * prm.nty;
  const int nsub = tile_subs(prm), side = prm.tile / kTile;
  const int list = (int)blockIdx.x / nsub;     // cell * ntiles + tile
  const int sub = (int)blockIdx.x - list * nsub;
  const int cell = list / ntiles, tile = list % ntiles;
  const int tx = tile % prm.ntx, ty = tile / prm.ntx;
  const int col = tx * prm.tile + (sub % side) * kTile + (lane & 7);
  const int row = ty * prm.tile + (sub / side) * kTile + (lane >> 3);
  const bool inimg = col < prm.width && row < prm.height;
  const int nch = ((int)seg_off[list + 1] - (int)seg_off[list]) / nsub;
  const int s0 = (int)seg_off[list] + sub * nch, s1 = s0 + nch;
  const int per = (s1 - s0 + kMergeWaves - 1) / kMergeWaves;
  const int a0 = min(s1, s0 + w * per), a1 = min(s1, a0 + per);
  M m;
  m.init();
  constexpr int kGroup = 4;
  for (int sb = a0; sb < a1 && !m.stopped; sb += kGroup) {
    M v[kGroup];
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int s = min(sb + u, a1 - 1);
      const double *q = part + (size_t)s * Q::NF * 64 + lane;
#pragma unroll
      for (int j = 0; j < F; ++j) {
        v[u].lo[j] = q[(Q::LO + c * F + j) * 64];
        v[u].hi[j] = q[(Q::HI + c * F + j) * 64];
      }
      v[u].ihi = q[(Q::IHI + c) * 64];
      const float2 mg = __builtin_bit_cast(float2, q[Q::MAG * 64]);
      v[u].magl = mg.x;
      v[u].magh = mg.y;
      v[u].T_lo = q[Q::TLO * 64];
      v[u].T_hi = q[Q::THI * 64];
      v[u].extra = v[u].T_hi;
      v[u].stopped = q[Q::STOP * 64] != 0.0;
      v[u].cnt = (unsigned)q[Q::CNT * 64];
    }
#pragma unroll
    for (int u = 0; u < kGroup; ++u)
      if (sb + u < a1) m.append(v[u]);
  }
  if (w > 0) red[c][w - 1][lane] = m;
  __syncthreads();
  if (w > 0) return;
#pragma unroll
  for (int k = 0; k < kMergeWaves - 1; ++k) m.append(red[c][k][lane]);
  if (c == 0 && lane == 0 && m.cnt) atomicAdd(&counters[0], (unsigned long long)m.cnt);
  if (!inimg) return;
  const int n = (int)(ranges[2 * list + 1] - ranges[2 * list]);
  const size_t img = (size_t)cell * prm.width * prm.height;
  write_channel<P>(m.lo, m.hi, m.ihi, m.magl, m.magh, (double)(n + 2 * (s1 - s0)), prm.E, m.extra, out_lo, out_hi,
                   ((img + (size_t)row * prm.width + col) * 3 + c));
}

template <int P>
static hipError_t launch_trans_p(const Workspace &ws, const uint32_t *lists, int nlists, const Params &prm, int L,
                                 int nseg_max, float *lo, float *hi, hipStream_t s) {
  if (ws.ev[1]) HIP_RET(hipEventRecord(ws.ev[1], s));
  if (nseg_max > 0)
    hipLaunchKernelGGL(k_raster_seg<P>, dim3((nseg_max + 3) / 4), dim3(256), 0, s, ws.rec, ws.key, ws.tile_range,
                       lists, ws.seg_off, ws.seg_tile, L, nlists, prm, ws.part);
  if (ws.ev[2]) HIP_RET(hipEventRecord(ws.ev[2], s));
  hipLaunchKernelGGL(k_merge<P>, dim3(nlists * tile_subs(prm)), dim3(192 * kMergeWaves), 0, s, ws.tile_range,
                     ws.seg_off, ws.part, prm, lo, hi, ws.counters);
  return hipGetLastError();
}

hipError_t launch_segments(const Workspace &ws, int nlists, int L, hipStream_t s, int nsub) {
  hipLaunchKernelGGL(k_seg_count, dim3((nlists + 1 + 255) / 256), dim3(256), 0, s, ws.tile_range, nlists, L, nsub,
                     ws.seg_off);
  return hipGetLastError();
}

hipError_t launch_segment_map(const Workspace &ws, int nlists, hipStream_t s, uint32_t cap) {
  hipLaunchKernelGGL(k_seg_map, dim3((nlists + 255) / 256), dim3(256), 0, s, ws.seg_off, nlists, ws.seg_tile, cap,
                     ws.counters + kOverflow);
  return hipGetLastError();
}

// Waves of k_raster_seg<P> the device holds at once (occupancy times CUs), cached per
// device and P.
int seg_resident_waves(int P) {
  static std::atomic<int> cache[16][4];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16 || P < 0 || P > 3) return 4096;
  int v = cache[dev][P].load(std::memory_order_relaxed);
  if (v > 0) return v;
  const void *fn = P == 0 ? (const void *)k_raster_seg<0>
                 : P == 1 ? (const void *)k_raster_seg<1>
                 : P == 2 ? (const void *)k_raster_seg<2>
                          : (const void *)k_raster_seg<3>;
  int blocks = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, 256, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 4096;
  }
  v = std::max(1, blocks) * 4 * std::max(1, cus);
  cache[dev][P].store(v, std::memory_order_relaxed);
  return v;
}

hipError_t launch_raster_translation(int P, const Workspace &ws, const uint32_t *lists, int nlists, const Params &prm,
                                     int L, int nseg_max, float *lo, float *hi, hipStream_t s) {
  switch (P) {
    case 0: return launch_trans_p<0>(ws, lists, nlists, prm, L, nseg_max, lo, hi, s);
    case 1: return launch_trans_p<1>(ws, lists, nlists, prm, L, nseg_max, lo, hi, s);
    case 2: return launch_trans_p<2>(ws, lists, nlists, prm, L, nseg_max, lo, hi, s);
    case 3: return launch_trans_p<3>(ws, lists, nlists, prm, L, nseg_max, lo, hi, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ar
