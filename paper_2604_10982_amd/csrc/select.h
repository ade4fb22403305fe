// Compact numbering of the surfels a tile's pixels selected for the feature
// channels (Sec. 5, eq. (18)).
//
// Every pixel of a tile keeps up to K list positions (ascending).  The
// distinct positions of the whole tile are few compared with the 256 K
// (pixel, selection) entries (a few dozen for K = 16 on plane-structured
// scenes), so the feature kernels stage each distinct feature row once per
// tile in LDS and address it by its slot: the rank of its list position among
// the tile's selected positions.  Positions are ranked with a bitmap over a
// window of list positions and a prefix count of its words; slots are taken
// in chunks of kSlotChunk rows.  Slot order follows list order, so a pixel's
// selections visit slots in ascending order across windows and chunks.
#pragma once

#include "common.h"

namespace psm {

constexpr int kWinWords = 512;           // bitmap words per window
constexpr int kWinPos = kWinWords * 32;  // list positions per window
constexpr int kSlotChunk = 128;          // feature rows staged at once

struct SelShared {
  uint32_t bits[kWinWords];  // selected positions of the window
  uint32_t pref[kWinWords];  // selected positions in the words before
  uint32_t red[8];           // block scan scratch
  uint32_t fid[kSlotChunk];  // surfel id of each slot of the chunk
  uint32_t lpos[kSlotChunk]; // list position of each slot of the chunk
};

// Block-wide (256 threads) exclusive prefix sum of one value per thread.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* red, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) red[wave] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t t = red[w];
    pre += w < wave ? t : 0u;
    tot += t;
  }
  total = tot;
  __syncthreads();
  return pre + x - v;
}

// Block-wide maximum of one value per thread.
__device__ __forceinline__ int block_max(int v, uint32_t* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  if (lane == 0) red[wave] = (uint32_t)v;
  __syncthreads();
  int m = (int)red[0];
#pragma unroll
  for (int w = 1; w < 4; ++w) m = max(m, (int)red[w]);
  __syncthreads();
  return m;
}

// Words of the window starting at list position w0 that can hold a position
// <= maxpos.
__device__ __forceinline__ int window_words(int maxpos, int w0) {
  return min(kWinWords, ((maxpos - w0) >> 5) + 1);
}

// Marks the selected positions of the window and ranks them; returns the
// number of distinct selected positions in the window.
template <int KMAX>
__device__ int build_window(SelShared& S, const int (&pos)[KMAX], int K, int w0, int nwords) {
  const int tid = threadIdx.x;
  for (int i = tid; i < nwords; i += 256) S.bits[i] = 0u;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const int r = pos[q] - w0;
    if (q < K && pos[q] >= 0 && r >= 0 && r < nwords * 32) atomicOr(&S.bits[r >> 5], 1u << (r & 31));
  }
  __syncthreads();
  const int w = 2 * tid;
  const uint32_t b0 = w < nwords ? S.bits[w] : 0u;
  const uint32_t b1 = w + 1 < nwords ? S.bits[w + 1] : 0u;
  uint32_t total;
  const uint32_t ex = block_scan_excl((uint32_t)(__popc(b0) + __popc(b1)), S.red, total);
  if (w < nwords) S.pref[w] = ex;
  if (w + 1 < nwords) S.pref[w + 1] = ex + (uint32_t)__popc(b0);
  __syncthreads();
  return (int)total;
}

// Window slot of list position pos, or -1 if it lies outside the window.
__device__ __forceinline__ int slot_of(const SelShared& S, int pos, int w0, int nwords) {
  const int r = pos - w0;
  if (pos < 0 || r < 0 || r >= nwords * 32) return -1;
  const uint32_t m = S.bits[r >> 5];
  return (int)(S.pref[r >> 5] + (uint32_t)__popc(m & ((1u << (r & 31)) - 1u)));
}

// LDS array of the tile's selection weights, one row of 256 pixels per
// selection index q (the feature kernels' matrix operand W[p][slot] is looked
// up here).  Row offsets are 288 q plus (q & 7) + 16 ((q >> 3) & 1), so the
// rows of the up to 16 selections of two pixels 8 apart fall in disjoint bank
// sets.
constexpr int kWRow = 288;  // floats per selection row
__device__ __forceinline__ int wsel_off(int q, int p) { return q * kWRow + (q & 7) + ((q & 8) << 1) + p; }

}  // namespace psm
