// Stable LSD radix sort of (uint32 key, uint32 value) pairs.
//
// Used twice per frame: the visible surfels by FP32 depth bits (32 bits,
// 4 passes) and then the emitted (tile, surfel) pairs by tile id (ceil(log2
// tiles) bits, 2 passes).  Because the pairs are emitted in depth order and
// every pass is stable, the result is the pair list ordered by
// (tile, depth, surfel id) -- an LSD sort of the composite key in which the
// low 32 bits are sorted once per surfel instead of once per pair.
//
// Each pass is reduce-then-scan (no inter-block waiting):
//   upsweep   -- per-block digit histogram (LDS, one sub-histogram per wave);
//   scan      -- one block per digit scans that digit's row over blocks;
//   downsweep -- per block, stable ranks from wave ballots, scatter.
// The element count is read on the device, so the launch shape only depends
// on the capacity and no host synchronisation is needed.
#include "common.h"
#include "internal.h"

namespace psm {

__global__ __launch_bounds__(kSortThreads) void k_rs_upsweep(const uint32_t* __restrict__ keys,
                                                            const uint32_t* __restrict__ n_dev, int shift,
                                                            int bits, uint32_t* __restrict__ hist) {
  const uint32_t n = *n_dev;
  const uint32_t nb = (n + kSortTile - 1) / kSortTile;
  if (blockIdx.x >= nb) return;
  __shared__ uint32_t s_h[4][256];
  const int wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 4 * 256; i += kSortThreads) (&s_h[0][0])[i] = 0;
  __syncthreads();
  const uint32_t mask = (1u << bits) - 1u;
  const uint32_t base = blockIdx.x * kSortTile;
#pragma unroll 4
  for (int j = 0; j < kSortItems; ++j) {
    const uint32_t idx = base + j * kSortThreads + threadIdx.x;
    if (idx < n) atomicAdd(&s_h[wave][(keys[idx] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < (1 << bits); d += kSortThreads)
    hist[(size_t)d * nb + blockIdx.x] = s_h[0][d] + s_h[1][d] + s_h[2][d] + s_h[3][d];
}

// Block d: exclusive scan of digit d's counts over the blocks; the digit's
// total goes to hist[256 * nb_max + d].
__global__ __launch_bounds__(256) void k_rs_scan(const uint32_t* __restrict__ n_dev, uint32_t* __restrict__ hist,
                                                 int64_t nb_max) {
  const uint32_t n = *n_dev;
  const uint32_t nb = (n + kSortTile - 1) / kSortTile;
  const int d = blockIdx.x;
  const int t = threadIdx.x;
  uint32_t* row = hist + (size_t)d * nb;
  __shared__ uint32_t s[256];
  const uint32_t per = (nb + 255) / 256;
  const uint32_t b0 = t * per, b1 = min(nb, b0 + per);
  uint32_t acc = 0;
  for (uint32_t b = b0; b < b1; ++b) acc += row[b];
  s[t] = acc;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint32_t v = t >= o ? s[t - o] : 0u;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  uint32_t run = s[t] - acc;
  for (uint32_t b = b0; b < b1; ++b) {
    const uint32_t v = row[b];
    row[b] = run;
    run += v;
  }
  if (t == 255) hist[256 * nb_max + d] = s[255];
}

__global__ __launch_bounds__(kSortThreads) void k_rs_downsweep(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ n_dev, int shift, int bits,
    const uint32_t* __restrict__ hist, int64_t nb_max) {
  const uint32_t n = *n_dev;
  const uint32_t nb = (n + kSortTile - 1) / kSortTile;
  if (blockIdx.x >= nb) return;
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_wc[4][256];
  const int t = threadIdx.x;
  const int ndig = 1 << bits;
  const uint32_t mask = (uint32_t)ndig - 1u;
  // global start of each digit for this block: digits before it + earlier blocks
  const uint32_t tot = t < ndig ? hist[256 * nb_max + t] : 0u;
  s_base[t] = tot;
  for (int i = t; i < 4 * 256; i += kSortThreads) (&s_wc[0][0])[i] = 0;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint32_t v = t >= o ? s_base[t - o] : 0u;
    __syncthreads();
    s_base[t] += v;
    __syncthreads();
  }
  const uint32_t excl = s_base[t] - tot;
  __syncthreads();
  s_base[t] = excl + (t < ndig ? hist[(size_t)t * nb + blockIdx.x] : 0u);
  __syncthreads();

  const int lane = t & 63, wave = t >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t base = blockIdx.x * kSortTile;
  for (int j = 0; j < kSortItems; ++j) {
    const uint32_t idx = base + j * kSortThreads + t;
    const bool valid = idx < n;
    const uint32_t key = valid ? kin[idx] : 0u;
    const uint32_t val = valid ? vin[idx] : 0u;
    const uint32_t d = (key >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) s_wc[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = s_base[d] + rank;
      for (int w = 0; w < wave; ++w) pos += s_wc[w][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    if (t < ndig) {
      s_base[t] += s_wc[0][t] + s_wc[1][t] + s_wc[2][t] + s_wc[3][t];
      s_wc[0][t] = s_wc[1][t] = s_wc[2][t] = s_wc[3][t] = 0u;
    }
    __syncthreads();
  }
}

void radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* n_dev,
                      int64_t cap_n, int bits, uint32_t* hist, int64_t nb_max, hipStream_t st) {
  if (cap_n <= 0) return;
  int passes = std::max(2, (bits + 7) / 8);
  if (passes & 1) ++passes;
  const unsigned grid = (unsigned)cdiv(cap_n, kSortTile);
  uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int left = passes - p;
    const int b = (bits - shift + left - 1) / left;
    hipLaunchKernelGGL(k_rs_upsweep, dim3(grid), dim3(kSortThreads), 0, st, ki, n_dev, shift, b, hist);
    hipLaunchKernelGGL(k_rs_scan, dim3(1u << b), dim3(256), 0, st, n_dev, hist, nb_max);
    hipLaunchKernelGGL(k_rs_downsweep, dim3(grid), dim3(kSortThreads), 0, st, ki, vi, ko, vo, n_dev, shift, b,
                       hist, nb_max);
    std::swap(ki, ko);
    std::swap(vi, vo);
    shift += b;
  }
}

}  // namespace psm
