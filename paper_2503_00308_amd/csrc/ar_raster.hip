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
// equal depths sharing one value (Alg. BlendInd lines 1-2):
//     T_hi[i] = prod_{front} (1 - a_lo[j]),   T_lo[i] = prod_{front} (1 - a_hi[j]).
// Colour (line 3) is accumulated as linear forms in FP64:
//     lo: sum_i c_i T_lo[i] a_i^lower(e),   hi: sum_i c_i T_hi[i] a_i^upper(e)
// plus the interval upper sum sum_i c_i T_hi[i] a_hi[i].
//
// Work decomposition: one workgroup per tile, one lane per pixel, G waves.  The tile's
// depth-ordered list is cut into chunks of C Gaussians (cuts moved to the next depth
// change so ties never straddle a cut); in each round wave g takes chunk g of the
// round and accumulates with a local transmittance starting at 1.  At the round's end
// the waves exchange their chunk transmittance products through LDS and scale their
// local sums by the product of everything in front.  Once every pixel's upper
// transmittance is below t_min the tile stops; the remaining Gaussians can add at
// most that transmittance, which is added to the upper bound.
#include <hip/hip_runtime.h>

#include "ar_internal.h"
#include "ar_blend.h"

namespace ar {

// ---------------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------------
// squared distance from the mean box to the rectangle [ux0, ux1] x [uy0, uy1] (float32,
// no contraction): the per-pixel test of dist2_box evaluated at the nearest point
__device__ __forceinline__ float dist2_rect(const float *mu, float ux0, float ux1, float uy0, float uy1) {
#pragma clang fp contract(off)
  const float dx = fmaxf(fmaxf(mu[0] - ux1, 0.0f), ux0 - mu[1]);
  const float dy = fmaxf(fmaxf(mu[2] - uy1, 0.0f), uy0 - mu[3]);
  return dx * dx + dy * dy;
}

__device__ __forceinline__ float tile_dist2(const float *mu, int tx, int ty, const Params &prm) {
  const int x0 = tx * kTile, y0 = ty * kTile;
  const int x1 = min(x0 + kTile, prm.width) - 1, y1 = min(y0 + kTile, prm.height) - 1;
  const float ux0 = (float)((double)x0 + 0.5 - prm.cx), ux1 = (float)((double)x1 + 0.5 - prm.cx);
  const float uy0 = (float)((double)y0 + 0.5 - prm.cy), uy1 = (float)((double)y1 + 0.5 - prm.cy);
  return dist2_rect(mu, ux0, ux1, uy0, uy1);
}

template <int P, bool EMIT>
__global__ __launch_bounds__(256) void k_bin(const float *__restrict__ recs, const int32_t *__restrict__ rect,
                                             const uint32_t *__restrict__ perm, int n, Params prm,
                                             uint32_t *__restrict__ counts, uint32_t *__restrict__ pkey,
                                             uint32_t *__restrict__ pval) {
  using R = Rec<P>;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t gid = perm[r];
  const float *rec = recs + (size_t)gid * R::STRIDE;
  const int type = __float_as_int(rec[R::SC + R::TYPE]);
  const int32_t *rc = rect + 4 * (size_t)gid;
  uint32_t c = 0;
  uint32_t off = EMIT ? counts[r] : 0u;
  if (type != kDropped && rc[0] <= rc[2] && rc[1] <= rc[3]) {
    const float *mu = rec + R::SC + R::MU0LO;
    const float r2 = rec[R::SC + R::R2];
    for (int ty = rc[1]; ty <= rc[3]; ++ty)
      for (int tx = rc[0]; tx <= rc[2]; ++tx) {
        const bool keep = (type == kWild) || (tile_dist2(mu, tx, ty, prm) <= r2);
        if (keep) {
          if (EMIT) {
            pkey[off + c] = (uint32_t)(ty * prm.ntx + tx);
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

__global__ void k_tile_ranges(const uint32_t *__restrict__ keys, int npairs, uint32_t *__restrict__ ranges) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const uint32_t t = keys[p];
  if (p == 0 || keys[p - 1] != t) ranges[2 * t] = (uint32_t)p;
  if (p == npairs - 1 || keys[p + 1] != t) ranges[2 * t + 1] = (uint32_t)(p + 1);
}

template <int P>
static hipError_t launch_bin_p(const Workspace &ws, int n, const Params &prm, bool emit, hipStream_t s) {
  if (emit)
    hipLaunchKernelGGL((k_bin<P, true>), dim3((n + 255) / 256), dim3(256), 0, s, ws.rec, ws.rect, ws.perm, n, prm,
                       ws.count, ws.pair_key, ws.pair_val);
  else
    hipLaunchKernelGGL((k_bin<P, false>), dim3((n + 255) / 256), dim3(256), 0, s, ws.rec, ws.rect, ws.perm, n, prm,
                       ws.count, ws.pair_key, ws.pair_val);
  return hipGetLastError();
}

static hipError_t launch_bin(int P, const Workspace &ws, int n, const Params &prm, bool emit, hipStream_t s) {
  switch (P) {
    case 0: return launch_bin_p<0>(ws, n, prm, emit, s);
    case 1: return launch_bin_p<1>(ws, n, prm, emit, s);
    case 2: return launch_bin_p<2>(ws, n, prm, emit, s);
    case 3: return launch_bin_p<3>(ws, n, prm, emit, s);
    case 4: return launch_bin_p<4>(ws, n, prm, emit, s);
    case 5: return launch_bin_p<5>(ws, n, prm, emit, s);
    case 6: return launch_bin_p<6>(ws, n, prm, emit, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_count_tiles(int P, const Workspace &ws, int n, const Params &prm, hipStream_t s) {
  return launch_bin(P, ws, n, prm, false, s);
}

hipError_t launch_emit_tiles(int P, const Workspace &ws, int n, const Params &prm, hipStream_t s) {
  return launch_bin(P, ws, n, prm, true, s);
}

hipError_t launch_tile_ranges(const uint32_t *keys, int npairs, uint32_t *ranges, int ntiles, hipStream_t s) {
  const size_t m = 2 * (size_t)ntiles;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, ranges, m, 0u);
  if (npairs > 0)
    hipLaunchKernelGGL(k_tile_ranges, dim3((npairs + 255) / 256), dim3(256), 0, s, keys, npairs, ranges);
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

template <int P>
__global__ __launch_bounds__(512) void k_raster_translation(const float *__restrict__ recs,
                                                            const uint64_t *__restrict__ keys,
                                                            const uint32_t *__restrict__ ranges,
                                                            const uint32_t *__restrict__ lists, Params prm,
                                                            float *__restrict__ out_lo, float *__restrict__ out_hi,
                                                            unsigned long long *__restrict__ counters) {
  using R = Rec<P>;
  extern __shared__ double smem[];
  const int G = prm.groups, C = prm.chunk;
  double *tch = smem;                                   // [2][G][64][2]
  double *red = smem + 2 * G * 64 * 2;                  // [64][6(P+1)+4] final reduction
  const int lane = threadIdx.x & 63;
  const int g = threadIdx.x >> 6;
  const int tile = blockIdx.x;
  const int tx = tile % prm.ntx, ty = tile / prm.ntx;
  const int col = tx * kTile + (lane & 7), row = ty * kTile + (lane >> 3);
  const bool inimg = col < prm.width && row < prm.height;
  const double uxd = (double)col + 0.5 - prm.cx, uyd = (double)row + 0.5 - prm.cy;
  const float ux = (float)uxd, uy = (float)uyd;
  const int beg = (int)ranges[2 * tile];
  const int n = (int)ranges[2 * tile + 1] - beg;
  const uint32_t *list = lists + beg;

  Acc<P> acc;
  acc_zero<P>(acc);
  double tt_lo = 1.0, tt_hi = 1.0;   // transmittance of everything processed so far
  bool early = false;
  unsigned long long npairs = 0;
  int parity = 0;
  for (int base = 0; base < n; base += G * C) {
    const int p0 = cut_at(list, keys, n, base + g * C);
    const int p1 = cut_at(list, keys, n, base + (g + 1) * C);
    Acc<P> loc;
    acc_zero<P>(loc);
    double tl_lo = 1.0, tl_hi = 1.0;     // local transmittance (chunk)
    double tg_lo = 1.0, tg_hi = 1.0;     // local transmittance at the current depth value
    uint64_t prev_key = ~0ull;
    for (int p = p0; p < p1; ++p) {
      const uint32_t gid = list[p];
      const float *rec = recs + (size_t)gid * R::STRIDE;
      const uint64_t key = keys[gid];
      if (key != prev_key) {
        tg_lo = tl_lo;
        tg_hi = tl_hi;
        prev_key = key;
      }
      const int type = __float_as_int(rec[R::SC + R::TYPE]);
      const bool kept = inimg && pair_kept<P>(rec, type, ux, uy);
      if (kept) {
        double alo, ahi;
        pair_contrib<P>(rec, type, uxd, uyd, tg_lo, tg_hi, loc, alo, ahi);
        tl_lo *= 1.0 - ahi;
        tl_hi *= 1.0 - alo;
        ++npairs;
      }
    }
    // exchange chunk transmittances, scale the local sums by the product in front
    double *tp = tch + parity * G * 128;
    tp[(g * 64 + lane) * 2 + 0] = tl_lo;
    tp[(g * 64 + lane) * 2 + 1] = tl_hi;
    __syncthreads();
    double pre_lo = tt_lo, pre_hi = tt_hi;
    for (int w = 0; w < G; ++w) {
      const double a = tp[(w * 64 + lane) * 2 + 0], b = tp[(w * 64 + lane) * 2 + 1];
      if (w == g) { pre_lo = tt_lo; pre_hi = tt_hi; acc_fma<P>(acc, loc, pre_lo, pre_hi); }
      tt_lo *= a;
      tt_hi *= b;
    }
    parity ^= 1;
    if (prm.t_min > 0.0) {
      const bool done = !inimg || tt_hi < prm.t_min;
      if (__all(done)) {
        early = cut_at(list, keys, n, base + G * C) < n;
        break;
      }
    }
  }

  acc_reduce<P>(acc, red, G, g, lane);
  // pair count
  unsigned long long cnt = npairs;
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
  if (lane == 0 && cnt) atomicAdd(&counters[0], cnt);
  if (g != 0 || !inimg) return;
  write_pixel<P>(acc, (double)n, prm.E, early ? tt_hi : 0.0, out_lo, out_hi, ((size_t)row * prm.width + col) * 3);
}

template <int P>
static hipError_t launch_trans_p(const Workspace &ws, const uint32_t *lists, const Params &prm, float *lo, float *hi,
                                 hipStream_t s) {
  const int ntiles = prm.ntx * prm.nty;
  const int G = prm.groups;
  constexpr int kRed = 6 * (P + 1) + 3 + 1;
  const size_t shm = sizeof(double) * (2 * G * 64 * 2 + 64 * kRed);
  hipLaunchKernelGGL(k_raster_translation<P>, dim3(ntiles), dim3(64 * G), shm, s, ws.rec, ws.key, ws.tile_range,
                     lists, prm, lo, hi, ws.counters);
  return hipGetLastError();
}

hipError_t launch_raster_translation(int P, const Workspace &ws, const uint32_t *lists, const SceneDev &,
                                     const Params &prm, float *lo, float *hi, hipStream_t s) {
  switch (P) {
    case 0: return launch_trans_p<0>(ws, lists, prm, lo, hi, s);
    case 1: return launch_trans_p<1>(ws, lists, prm, lo, hi, s);
    case 2: return launch_trans_p<2>(ws, lists, prm, lo, hi, s);
    case 3: return launch_trans_p<3>(ws, lists, prm, lo, hi, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ar
