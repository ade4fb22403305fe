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
//   downsweep -- per block, stable ranks from wave ballots, the tile sorted
//                by digit in LDS, written out bucket by bucket.
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

// Block-wide (256 threads) exclusive prefix sum of one value per thread;
// red holds 4 words of scratch.  Ends with a barrier, so red can be reused.
__device__ __forceinline__ uint32_t sort_scan_excl(uint32_t v, uint32_t* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) red[wave] = x;
  __syncthreads();
  uint32_t pre = 0;
#pragma unroll
  for (int w = 0; w < 3; ++w) pre += w < wave ? red[w] : 0u;
  __syncthreads();
  return pre + x - v;
}

// One block per tile of kSortTile elements; wave w owns the elements
// [base + w kSortTile / 4, base + (w + 1) kSortTile / 4), kSortItems
// coalesced rows of 64.  (1) Each wave ranks its elements among equal digits
// in index order: wave ballots give the rank within a row, wave-private
// digit counters in LDS carry the count of the rows before (a wave's LDS
// operations complete in program order, so no barrier is needed).  (2) The
// counts are scanned over the waves and the digits, and every element is
// placed in LDS at its block-local position: the tile sorted stably by
// digit.  (3) The tile is written out in that order: consecutive threads
// write consecutive addresses of a digit's bucket.
__global__ __launch_bounds__(kSortThreads) void k_rs_downsweep(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ n_dev, int shift, int bits,
    const uint32_t* __restrict__ hist, int64_t nb_max) {
  static_assert(kSortThreads == 256, "one thread per digit of an 8-bit pass");
  const uint32_t n = *n_dev;
  const uint32_t nb = (n + kSortTile - 1) / kSortTile;
  if (blockIdx.x >= nb) return;
  __shared__ uint32_t s_cnt[4][256];  // per-wave digit counts, then the waves' offsets
  __shared__ uint32_t s_gbase[256];   // first global position of each digit for this block
  __shared__ uint32_t s_lbase[256];   // first block-local position of each digit
  __shared__ uint32_t s_red[4];
  __shared__ uint32_t s_k[kSortTile], s_v[kSortTile];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int ndig = 1 << bits;
  const uint32_t mask = (uint32_t)ndig - 1u;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t base = blockIdx.x * kSortTile;
  const uint32_t wbase = base + (uint32_t)wave * (64 * kSortItems);

  // global start of each digit for this block: all elements of smaller digits
  // plus this digit's elements in earlier blocks
  const uint32_t tot = t < ndig ? hist[256 * nb_max + t] : 0u;
  const uint32_t ex = sort_scan_excl(tot, s_red);
  s_gbase[t] = ex + (t < ndig ? hist[(size_t)t * nb + blockIdx.x] : 0u);
#pragma unroll
  for (int w = 0; w < 4; ++w) s_cnt[w][t] = 0u;
  __syncthreads();

  uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint32_t idx = wbase + j * 64 + lane;
    key[j] = idx < n ? kin[idx] : 0u;
    val[j] = idx < n ? vin[idx] : 0u;
  }
  uint32_t* cnt = s_cnt[wave];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const bool valid = wbase + j * 64 + lane < n;
    const uint32_t d = (key[j] >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t r = (uint32_t)__popcll(peers & lt);
    const uint32_t c = valid ? cnt[d] : 0u;
    rank[j] = c + r;
    if (valid && r == 0) cnt[d] = c + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // digit t: the waves' offsets (exclusive over waves) and the digit's
  // block-local start (exclusive over digits)
  const uint32_t c0 = s_cnt[0][t], c1 = s_cnt[1][t], c2 = s_cnt[2][t], c3 = s_cnt[3][t];
  s_cnt[0][t] = 0u;
  s_cnt[1][t] = c0;
  s_cnt[2][t] = c0 + c1;
  s_cnt[3][t] = c0 + c1 + c2;
  s_lbase[t] = sort_scan_excl(c0 + c1 + c2 + c3, s_red);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    if (wbase + j * 64 + lane < n) {
      const uint32_t d = (key[j] >> shift) & mask;
      const uint32_t lp = s_lbase[d] + cnt[d] + rank[j];
      s_k[lp] = key[j];
      s_v[lp] = val[j];
    }
  }
  __syncthreads();
  const uint32_t m = min((uint32_t)kSortTile, n - base);
  for (uint32_t i = t; i < m; i += kSortThreads) {
    const uint32_t k = s_k[i];
    const uint32_t d = (k >> shift) & mask;
    const uint32_t gp = s_gbase[d] + (i - s_lbase[d]);
    kout[gp] = k;
    vout[gp] = s_v[i];
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
