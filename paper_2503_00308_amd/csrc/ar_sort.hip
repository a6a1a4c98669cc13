// Stable LSD radix sort (8-bit digits) and exclusive scan for gfx950 (wave64).
//
// Used to order Gaussians by depth key (64-bit) and (tile, depth-rank) pairs by tile
// id (32-bit keys, stable so that each tile's list stays in depth order).
//
// Large inputs: one pass = histogram per block -> exclusive scan over the digit-major
// histogram -> stable scatter.  Small inputs: all passes in one workgroup.  Within a block the scatter ranks equal digits with 8 wave
// ballots, then across the block's waves through LDS, so equal keys keep input order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ar_internal.h"

namespace ar {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                       // per thread per block
constexpr int kSortTile = kSortThreads * kSortItems; // items per block
constexpr int kScanThreads = 1024;

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K *__restrict__ keys, int n, int shift,
                                                             uint32_t *__restrict__ hist, int nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortTile;
  for (int i = threadIdx.x; i < kSortTile; i += kSortThreads) {
    const int idx = base + i;
    if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                                K *__restrict__ kout, uint32_t *__restrict__ vout, int n,
                                                                int shift, const uint32_t *__restrict__ offs, int nblocks) {
  constexpr int kWaves = kSortThreads / 64;
  __shared__ uint32_t running[256];
  __shared__ uint32_t wcount[kWaves][256];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  running[threadIdx.x] = offs[threadIdx.x * nblocks + blockIdx.x];
  const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  const int base = blockIdx.x * kSortTile;
  for (int t = 0; t < kSortItems; ++t) {
    const int idx = base + t * kSortThreads + threadIdx.x;
    const bool valid = idx < n;
    K key = 0;
    uint32_t val = 0;
    uint32_t digit = 0;
    if (valid) {
      key = kin[idx];
      val = vin[idx];
      digit = (uint32_t)(key >> shift) & 255u;
    }
    for (int w = 0; w < kWaves; ++w) wcount[w][threadIdx.x] = 0;
    __syncthreads();
    // lanes of this wave holding the same digit
    uint64_t match = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((digit >> b) & 1u);
      match &= ((digit >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t rank = __popcll(match & below);
    if (valid && rank == 0) wcount[wave][digit] = __popcll(match);
    __syncthreads();
    if (valid) {
      uint32_t pos = running[digit] + rank;
      for (int w = 0; w < wave; ++w) pos += wcount[w][digit];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t tot = 0;
    for (int w = 0; w < kWaves; ++w) tot += wcount[w][threadIdx.x];
    running[threadIdx.x] += tot;
    __syncthreads();
  }
}

// Exclusive scan of n uint32 values in one workgroup (used for histograms and block sums).
__global__ __launch_bounds__(kScanThreads) void k_scan_single(uint32_t *data, int n) {
  __shared__ uint32_t part[kScanThreads];
  const int per = (n + kScanThreads - 1) / kScanThreads;
  const int b = threadIdx.x * per;
  const int e = min(n, b + per);
  uint32_t s = 0;
  for (int i = b; i < e; ++i) s += data[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;
  for (int i = b; i < e; ++i) {
    const uint32_t v = data[i];
    data[i] = run;
    run += v;
  }
}

constexpr int kScanBlock = 1024;  // elements per block of the large scan (256 threads x 4)

__global__ __launch_bounds__(256) void k_scan_blocks(const uint32_t *__restrict__ data, int n, uint32_t *__restrict__ sums) {
  __shared__ uint32_t red[256];
  const int base = blockIdx.x * kScanBlock + threadIdx.x * 4;
  uint32_t s = 0;
  for (int i = 0; i < 4; ++i)
    if (base + i < n) s += data[base + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_scan_apply(uint32_t *__restrict__ data, int n, const uint32_t *__restrict__ sums) {
  __shared__ uint32_t part[256];
  const int base = blockIdx.x * kScanBlock + threadIdx.x * 4;
  uint32_t v[4];
  uint32_t s = 0;
  for (int i = 0; i < 4; ++i) {
    v[i] = (base + i < n) ? data[base + i] : 0u;
    s += v[i];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t t = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  uint32_t run = sums[blockIdx.x] + part[threadIdx.x] - s;
  for (int i = 0; i < 4; ++i) {
    if (base + i < n) data[base + i] = run;
    run += v[i];
  }
}

hipError_t ensure_hist(Workspace &ws, size_t n_entries) {
  if (n_entries <= ws.cap_hist && ws.hist) return hipSuccess;
  const size_t cap = n_entries + n_entries / 2 + 1024;
  const hipError_t e = grow(ws, ws.hist, cap);
  if (e == hipSuccess) ws.cap_hist = cap;
  return e;
}

static hipError_t ensure_scan_tmp(Workspace &ws, size_t n_entries) {
  if (n_entries <= ws.cap_scan && ws.scan_tmp) return hipSuccess;
  const size_t cap = n_entries + n_entries / 2 + 1024;
  const hipError_t e = grow(ws, ws.scan_tmp, cap);
  if (e == hipSuccess) ws.cap_scan = cap;
  return e;
}

// Exclusive scan in place; block sums go to ws.scan_tmp (so data may be ws.hist).
hipError_t exclusive_scan_u32(uint32_t *data, int n, Workspace &ws, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n <= 32768) {
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kScanThreads), 0, s, data, n);
    return hipGetLastError();
  }
  const int nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb > 32768 * 16) return hipErrorInvalidValue;  // > 5e8 elements: beyond the supported sizes
  hipError_t e = ensure_scan_tmp(ws, (size_t)nb);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(256), 0, s, data, n, ws.scan_tmp);
  hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kScanThreads), 0, s, ws.scan_tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, s, data, n, ws.scan_tmp);
  return hipGetLastError();
}

// 64-bit total of n uint32 counts: a grid-stride sum per thread, a wave reduction and
// one atomic per wave.
__global__ __launch_bounds__(256) void k_sum_u32_u64(const uint32_t *__restrict__ data, size_t n,
                                                     unsigned long long *__restrict__ total) {
  unsigned long long s = 0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) s += data[i];
  for (int off = 32; off > 0; off >>= 1) s += (unsigned long long)__shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(total, s);
}

hipError_t sum_u32_u64(const uint32_t *data, size_t n, unsigned long long *total, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 1023) / 1024, 2048);
  hipLaunchKernelGGL(k_sum_u32_u64, dim3(blocks), dim3(256), 0, s, data, n, total);
  return hipGetLastError();
}

// Whole sort in one workgroup (small n): every pass histograms, scans and scatters
// through global memory (the data stay in L2) with block barriers in between, so a
// 64-bit sort is one launch instead of 24.  Passes whose digit is the same for every
// key are skipped.  The result is copied back to (keys, vals) if it ends in the
// alternate buffers.
constexpr int kBlockSortThreads = 1024;
constexpr int kBlockSortMax = 32768;

template <typename K>
__global__ __launch_bounds__(kBlockSortThreads) void k_radix_sort_block(K *__restrict__ keys, K *__restrict__ keys_alt,
                                                                        uint32_t *__restrict__ vals,
                                                                        uint32_t *__restrict__ vals_alt, int n,
                                                                        int begin_bit, int end_bit) {
  constexpr int kWaves = kBlockSortThreads / 64;
  __shared__ uint32_t hist[256];
  __shared__ uint32_t running[256];
  __shared__ uint32_t wcount[kWaves][256];
  __shared__ int skip;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  K *ki = keys, *ko = keys_alt;
  uint32_t *vi = vals, *vo = vals_alt;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    if (tid < 256) hist[tid] = 0u;
    __syncthreads();
    for (int i = tid; i < n; i += kBlockSortThreads) atomicAdd(&hist[(uint32_t)(ki[i] >> shift) & 255u], 1u);
    __syncthreads();
    if (tid == 0) {
      uint32_t run = 0;
      int full = 0;
      for (int d = 0; d < 256; ++d) {
        const uint32_t h = hist[d];
        running[d] = run;
        run += h;
        full |= (h == (uint32_t)n);
      }
      skip = full;
    }
    __syncthreads();
    if (skip) continue;   // every key has this digit: order unchanged
    for (int base = 0; base < n; base += kBlockSortThreads) {
      const int idx = base + tid;
      const bool valid = idx < n;
      K key = 0;
      uint32_t val = 0, digit = 0;
      if (valid) {
        key = ki[idx];
        val = vi[idx];
        digit = (uint32_t)(key >> shift) & 255u;
      }
      for (int w = 0; w < kWaves; w += 4) wcount[w + (tid >> 8)][tid & 255] = 0u;
      __syncthreads();
      uint64_t match = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint64_t bal = __ballot((digit >> b) & 1u);
        match &= ((digit >> b) & 1u) ? bal : ~bal;
      }
      const uint32_t rank = __popcll(match & below);
      if (valid && rank == 0) wcount[wave][digit] = __popcll(match);
      __syncthreads();
      if (valid) {
        uint32_t pos = running[digit] + rank;
        for (int w = 0; w < wave; ++w) pos += wcount[w][digit];
        ko[pos] = key;
        vo[pos] = val;
      }
      __syncthreads();
      if (tid < 256) {
        uint32_t tot = 0;
        for (int w = 0; w < kWaves; ++w) tot += wcount[w][tid];
        running[tid] += tot;
      }
      __syncthreads();
    }
    K *tk = ki; ki = ko; ko = tk;
    uint32_t *tv = vi; vi = vo; vo = tv;
  }
  if (ki != keys) {
    for (int i = tid; i < n; i += kBlockSortThreads) {
      keys[i] = ki[i];
      vals[i] = vi[i];
    }
  }
}

// Small depth sorts (n <= kRankMax): the rank of key i is the number of (key_j, j) below
// (key_i, i) -- a stable order by counting, no passes.  Block (kb, cb) counts the keys
// of chunk cb (staged in LDS) below the 256 keys of block kb and adds the counts; a
// second kernel scatters the values by rank.
constexpr int kRankMax = 16384;
constexpr int kRankChunk = 512;

__global__ __launch_bounds__(256) void k_rank_count(const uint64_t *__restrict__ keys, int n,
                                                    uint32_t *__restrict__ rank) {
  __shared__ uint64_t ck[kRankChunk];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int c0 = blockIdx.y * kRankChunk;
  const int cn = min(kRankChunk, n - c0);
  for (int t = threadIdx.x; t < cn; t += 256) ck[t] = keys[c0 + t];
  __syncthreads();
  if (i >= n) return;
  const uint64_t ki = keys[i];
  uint32_t below = 0;
  for (int t = 0; t < cn; ++t) {
    const uint64_t kj = ck[t];
    below += (kj < ki || (kj == ki && c0 + t < i)) ? 1u : 0u;
  }
  if (below) atomicAdd(&rank[i], below);
}

__global__ void k_rank_scatter(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                               const uint32_t *__restrict__ rank, int n, uint64_t *__restrict__ kout,
                               uint32_t *__restrict__ vout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t r = rank[i];
  kout[r] = keys[i];
  vout[r] = vals[i];
}

__global__ void k_zero_n(uint32_t *__restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_cell_keys(const uint32_t *__restrict__ items, int n_total, int n_cell,
                            uint32_t *__restrict__ keys, const uint32_t *__restrict__ item_off, int ncells) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_total) keys[i] = (uint32_t)item_cell(item_off, ncells, n_cell, items[i]);
}

hipError_t launch_cell_keys(const uint32_t *items, int n_total, int n_cell, uint32_t *keys, hipStream_t s,
                            const uint32_t *item_off, int ncells) {
  hipLaunchKernelGGL(k_cell_keys, dim3((n_total + 255) / 256), dim3(256), 0, s, items, n_total, n_cell, keys, item_off,
                     ncells);
  return hipGetLastError();
}

template <typename K>
static hipError_t radix_sort(K *keys, K *keys_alt, uint32_t *vals, uint32_t *vals_alt, int n, int begin_bit,
                             int end_bit, Workspace &ws, hipStream_t s, bool *in_alt) {
  *in_alt = false;
  if (n <= 1) return hipSuccess;
  if (n <= kBlockSortMax) {
    hipLaunchKernelGGL(k_radix_sort_block<K>, dim3(1), dim3(kBlockSortThreads), 0, s, keys, keys_alt, vals, vals_alt,
                       n, begin_bit, end_bit);
    return hipGetLastError();
  }
  const int nb = (n + kSortTile - 1) / kSortTile;
  hipError_t e = ensure_hist(ws, (size_t)256 * nb);
  if (e != hipSuccess) return e;
  K *ki = keys, *ko = keys_alt;
  uint32_t *vi = vals, *vo = vals_alt;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist<K>, dim3(nb), dim3(kSortThreads), 0, s, ki, n, shift, ws.hist, nb);
    e = exclusive_scan_u32(ws.hist, 256 * nb, ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter<K>, dim3(nb), dim3(kSortThreads), 0, s, ki, vi, ko, vo, n, shift, ws.hist, nb);
    K *tk = ki; ki = ko; ko = tk;
    uint32_t *tv = vi; vi = vo; vo = tv;
    *in_alt = !*in_alt;
  }
  return hipGetLastError();
}

hipError_t radix_sort_u64(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt, int n, int begin_bit,
                          int end_bit, Workspace &ws, hipStream_t s, bool *in_alt) {
  if (n > 1 && n <= kRankMax && begin_bit == 0 && end_bit == 64) {
    // stable order by counting; the sorted keys / values land in the alternate buffers
    hipError_t e = ensure_hist(ws, (size_t)n);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_n, dim3((n + 255) / 256), dim3(256), 0, s, ws.hist, n);
    hipLaunchKernelGGL(k_rank_count, dim3((n + 255) / 256, (n + kRankChunk - 1) / kRankChunk), dim3(256), 0, s, keys,
                       n, ws.hist);
    hipLaunchKernelGGL(k_rank_scatter, dim3((n + 255) / 256), dim3(256), 0, s, keys, vals, ws.hist, n, keys_alt,
                       vals_alt);
    *in_alt = true;
    return hipGetLastError();
  }
  return radix_sort<uint64_t>(keys, keys_alt, vals, vals_alt, n, begin_bit, end_bit, ws, s, in_alt);
}

hipError_t radix_sort_u32(uint32_t *keys, uint32_t *keys_alt, uint32_t *vals, uint32_t *vals_alt, int n, int begin_bit,
                          int end_bit, Workspace &ws, hipStream_t s, bool *in_alt) {
  return radix_sort<uint32_t>(keys, keys_alt, vals, vals_alt, n, begin_bit, end_bit, ws, s, in_alt);
}

}  // namespace ar
