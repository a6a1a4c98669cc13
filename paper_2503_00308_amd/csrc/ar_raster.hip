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
#include "ar_pair.h"

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
template <int P>
struct Acc {
  double lo[3][P + 1];
  double hi[3][P + 1];
  double ihi[3];
  float magl, magh;  // magnitude sums bounding the FP64 rounding of the sums
};

template <int P>
__device__ __forceinline__ void acc_zero(Acc<P> &a) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int j = 0; j <= P; ++j) { a.lo[c][j] = 0.0; a.hi[c][j] = 0.0; }
    a.ihi[c] = 0.0;
  }
  a.magl = 0.0f;
  a.magh = 0.0f;
}

// dst += (pre_lo, pre_hi) * src
template <int P>
__device__ __forceinline__ void acc_fma(Acc<P> &dst, const Acc<P> &src, double pre_lo, double pre_hi) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int j = 0; j <= P; ++j) {
      dst.lo[c][j] = fma(pre_lo, src.lo[c][j], dst.lo[c][j]);
      dst.hi[c][j] = fma(pre_hi, src.hi[c][j], dst.hi[c][j]);
    }
    dst.ihi[c] = fma(pre_hi, src.ihi[c], dst.ihi[c]);
  }
  dst.magl = fmaf((float)pre_lo, src.magl, dst.magl) * (1.0f + 4.0f * kU);
  dst.magh = fmaf((float)pre_hi, src.magh, dst.magh) * (1.0f + 4.0f * kU);
}

// One (pixel, Gaussian) pair: alpha bounds and its BlendInd contribution with the
// transmittances (tlo, thi) of the Gaussians in front.  Returns the alpha interval.
template <int P>
__device__ __forceinline__ void pair_contrib(const float *__restrict__ rec, int type, float ux, float uy, float dux,
                                             float duy, float d2, double tlo, double thi, Acc<P> &acc, float &a_lo,
                                             float &a_hi) {
  using R = Rec<P>;
  const float *sc = rec + R::SC;
  const float o = sc[R::O];
  const double c3[3] = {(double)sc[R::C0], (double)sc[R::C1], (double)sc[R::C2]};
  if (type == kNormal) {
    SForms<P> s;
    s_forms<P>(rec, ux, uy, dux, duy, s);
    ExpBounds b;
    exp_bounds(s.slo, s.shi, o, b);
    // lower alpha form  o e_dn (x_lower(e) - xlo + 1),  x_lower = -s_upper / 2
    // upper alpha form  o e_up + o k_up (x_upper(e) - xlo),  x_upper = -s_lower / 2
    const double wl = (double)o * (double)b.e_dn;
    const double wk = (double)o * (double)b.k_up;
    double gl[P + 1], gh[P + 1];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      gl[j] = wl * (-0.5 * (double)s.sh[j]);
      gh[j] = wk * (-0.5 * (double)s.sl[j]);
    }
    gl[P] = wl * ((-0.5 * (double)s.sh[P] - (double)b.xlo) + 1.0);
    gh[P] = (double)o * (double)b.e_up + wk * (-0.5 * (double)s.sl[P] - (double)b.xlo);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double wlo = c3[c] * tlo, whi = c3[c] * thi;
#pragma unroll
      for (int j = 0; j <= P; ++j) {
        acc.lo[c][j] = fma(wlo, gl[j], acc.lo[c][j]);
        acc.hi[c][j] = fma(whi, gh[j], acc.hi[c][j]);
      }
      acc.ihi[c] = fma(whi, (double)b.a_hi, acc.ihi[c]);
    }
    const float ml = (o * b.e_dn) * (0.5f * s.msh + fabsf(b.xlo) + 1.0f);
    const float mh = o * b.e_up + (o * b.k_up) * (0.5f * s.msl + fabsf(b.xlo)) + b.a_hi;
    acc.magl = fmaf((float)tlo, ml, acc.magl);
    acc.magh = fmaf((float)thi, mh, acc.magh);
    a_lo = b.a_lo;
    a_hi = b.a_hi;
  } else {
    // MatrixInv fallback: [0, o exp(-d2 / (2 lam))]; near-plane straddler: [0, o]
    float ah = o;
    if (type == kFallback) {
      const float lam = sc[R::LAM];
      ah = fminf(o, (o * expf(-0.5f * (d2 * (1.0f - 4.0f * kU)) / lam)) * (1.0f + 16.0f * kU));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double whi = c3[c] * thi;
      acc.hi[c][P] = fma(whi, (double)ah, acc.hi[c][P]);
      acc.ihi[c] = fma(whi, (double)ah, acc.ihi[c]);
    }
    acc.magh = fmaf((float)thi, 2.0f * ah, acc.magh);
    a_lo = 0.0f;
    a_hi = ah;
  }
}

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
  double *red = smem + 2 * G * 64 * 2;                  // [64][nred]
  constexpr int kRed = 6 * (P + 1) + 3 + 1;             // doubles exchanged in the final reduction
  const int lane = threadIdx.x & 63;
  const int g = threadIdx.x >> 6;
  const int tile = blockIdx.x;
  const int tx = tile % prm.ntx, ty = tile / prm.ntx;
  const int col = tx * kTile + (lane & 7), row = ty * kTile + (lane >> 3);
  const bool inimg = col < prm.width && row < prm.height;
  const double uxd = (double)col + 0.5 - prm.cx, uyd = (double)row + 0.5 - prm.cy;
  const float ux = (float)uxd, uy = (float)uyd;
  const float dux = 2.0f * (float)fabs((double)ux - uxd), duy = 2.0f * (float)fabs((double)uy - uyd);
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
      float d2 = 0.0f;
      bool kept = inimg;
      if (type != kWild) {
        d2 = dist2_box(rec[R::SC + R::MU0LO], rec[R::SC + R::MU0HI], rec[R::SC + R::MU1LO], rec[R::SC + R::MU1HI],
                       ux, uy);
        kept = kept && (d2 <= rec[R::SC + R::R2]);
      }
      if (kept) {
        float alo, ahi;
        pair_contrib<P>(rec, type, ux, uy, dux, duy, d2, tg_lo, tg_hi, loc, alo, ahi);
        tl_lo *= 1.0 - (double)ahi;
        tl_hi *= 1.0 - (double)alo;
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

  // reduce the G waves' sums into wave 0
  for (int w = 1; w < G; ++w) {
    __syncthreads();
    if (g == w) {
      double *dst = red + lane * kRed;
      int q = 0;
      for (int c = 0; c < 3; ++c) {
        for (int j = 0; j <= P; ++j) { dst[q++] = acc.lo[c][j]; dst[q++] = acc.hi[c][j]; }
        dst[q++] = acc.ihi[c];
      }
      float *fm = (float *)(dst + q);  // last slot: the two magnitude sums
      fm[0] = acc.magl;
      fm[1] = acc.magh;
    }
    __syncthreads();
    if (g == 0) {
      const double *src = red + lane * kRed;
      int q = 0;
      for (int c = 0; c < 3; ++c) {
        for (int j = 0; j <= P; ++j) { acc.lo[c][j] += src[q++]; acc.hi[c][j] += src[q++]; }
        acc.ihi[c] += src[q++];
      }
      acc.magl = (acc.magl + ((const float *)(src + q))[0]) * (1.0f + 4.0f * kU);
      acc.magh = (acc.magh + ((const float *)(src + q))[1]) * (1.0f + 4.0f * kU);
    }
  }
  // pair count
  unsigned long long cnt = npairs;
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
  if (lane == 0 && cnt) atomicAdd(&counters[0], cnt);
  if (g != 0 || !inimg) return;

  // bound on the FP64 rounding of all sums: (terms + 16) 2^-52 times the magnitudes
  const double nterm = (double)(n + 16);
  const double wlo = nterm * 0x1p-51 * (double)acc.magl;
  const double whi = nterm * 0x1p-51 * (double)acc.magh;
  const size_t pix = ((size_t)row * prm.width + col) * 3;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double sl = 0.0, sh = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) { sl += fabs(acc.lo[c][j]); sh += fabs(acc.hi[c][j]); }
    double lo = acc.lo[c][P] - sl - prm.E - wlo;
    double hi = fmin(acc.hi[c][P] + sh, acc.ihi[c]) + prm.E + whi;
    if (early) hi += tt_hi;
    lo = fmin(fmax(lo, 0.0), 1.0);
    hi = fmin(fmax(hi, 0.0), 1.0);
    out_lo[pix + c] = __double2float_rd(lo);
    out_hi[pix + c] = __double2float_ru(hi);
  }
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
