// Forward compositing (Sec. 3.1 eq. (1); Sec. 5 eq. (18)).
//
// k_walk: one 16x16 tile per 256-thread block (4 wave64), one pixel per lane.
//   Surfel records of the tile's depth-sorted list are staged in LDS in
//   batches of 256 and read by broadcast.  Each lane walks front to back:
//   ray/surfel intersection, alpha, transmittance, dense RGB/depth/normal/
//   alpha blend, stop before T would fall below 1e-4, and (Top-K mode) a
//   per-pixel register heap of the K largest weights with their list
//   positions.  A block stops when all of its pixels are done.
// k_blend_topk: eq. (18) blend of the selected feature rows, thread per pixel.
//   The tile's distinct selected rows are staged in LDS per pass of 16 or 32
//   channels and read by slot; each pixel accumulates in ascending list
//   position (front to back).
// k_full_feat: the dense feature blend of eq. (1) (the baseline the paper
//   accelerates), channel-chunked re-walks with feature rows staged in LDS.
#include "common.h"
#include "internal.h"
#include "select.h"

namespace psm {

constexpr int kWalkBatch = 256;

template <int N>
__device__ __forceinline__ void sort_by_position(int (&p)[N], float (&w)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const bool sw = up ? (p[i] > p[l]) : (p[i] < p[l]);
          const int tp = p[i];
          const float tw = w[i];
          p[i] = sw ? p[l] : p[i];
          w[i] = sw ? w[l] : w[i];
          p[l] = sw ? tp : p[l];
          w[l] = sw ? tw : w[l];
        }
      }
    }
  }
}

constexpr int kWalkChunk = 64;  // list entries a wave examines at once

// Each wave walks its 64 pixels (a 16x4 band of the tile) on its own, with no
// block barriers: per chunk of 64 list entries every lane tests one entry's
// footprint against the band (one vector gather of the extent records and a
// ballot), the kept entries' records are staged, compacted, in the wave's LDS
// slice by parallel vector loads, and the wave then evaluates them in list
// order with broadcast reads.
// KFULL: K == KMAX, known at compile time, so no per-entry "q < K" masks are
// held across the tile loop (they cost the persistent form 60 registers).
template <int KMAX, bool TOPK, bool PERSIST, bool LP, bool KFULL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_walk(const WalkRec* __restrict__ rec, const float4* __restrict__ ext,
                                              const uint32_t* __restrict__ pid,
                                              const uint2* __restrict__ ranges, CamTable ct, TileQueue tq,
                                              int K_, float* __restrict__ o_rgb, float* __restrict__ o_depth,
                                              float* __restrict__ o_normal, float* __restrict__ o_alpha,
                                              uint32_t* __restrict__ nlast, float* __restrict__ tfinal,
                                              int32_t* __restrict__ selpos, float* __restrict__ selw,
                                              uint32_t* __restrict__ status, int feat_only) {
  const int K = KFULL ? KMAX : K_;
  __shared__ Staged<kWalkChunk> s_rec[4];
  __shared__ int s_pos[4][kWalkChunk];
  __shared__ int s_item;
  for_tiles<PERSIST>(tq, &s_item, [&](const int tile) {
  const TileLoc tl = locate(ct, tile);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tx = tl.tx, ty = tl.ty, W = tl.W, H = tl.H;
  const int qx = tile_lx(ct, tid), qy = tile_ly(ct, tid), rpw = 64 >> ct.tsh;  // rows per wave
  const int px = tx * ct.tw + qx, py = ty * ct.th + qy;
  const bool inside = px < W && py < H;
  const float lx = (float)qx + 0.5f, ly = (float)qy + 0.5f;
  const float tx0 = (float)(tx * ct.tw), ty0 = (float)(ty * ct.th);
  const float yb0 = ty0 + (float)(rpw * wave) + 0.5f, yb1 = yb0 + (float)(rpw - 1);  // this wave's rows
  const uint2 rg = ranges[tile];
  const int L = (int)(rg.y - rg.x);
  const uint32_t* ids = pid + rg.x;
  Staged<kWalkChunk>& S = s_rec[wave];
  int* spos = s_pos[wave];

  float T = 1.0f, cr = 0.f, cg = 0.f, cb = 0.f, dep = 0.f, nx = 0.f, ny = 0.f, nz = 0.f;
  int last = 0, blended = 0, stop = -1;
  bool done = !inside;
  // Top-K heap: one 64-bit key per entry, weight bits above the complemented
  // list position.  Weights are positive, so unsigned key order is the order
  // (weight, then earlier position) of eq. (18); an empty entry is key 0 and
  // entries beyond K can never be the minimum.
  uint64_t hk[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) hk[q] = q < K ? 0ull : ~0ull;
  uint64_t kmin = 0ull;
  int imin = 0;

  for (int base = 0; base < L; base += kWalkChunk) {
    if (__all(done)) break;
    const int j = base + lane;
    uint32_t id = 0;
    bool keep = false;
    if (j < L) {
      id = ids[j];
      const float4 x = ext[id];
      keep = band_meets(x.y, x.w, yb0, yb1);
    }
    const uint64_t mask = __ballot(keep);
    const int nk = __popcll(mask);
    wave_lds_sync();  // the previous chunk's reads are done
    if (keep) {
      const int slot = __popcll(mask & ((1ull << lane) - 1ull));
      S.put(slot, rec[id], tx0, ty0);
      spos[slot] = j;
    }
    wave_lds_sync();
    for (int k = 0; k < nk; ++k) {
      if (__all(done)) break;
      if (done) continue;
      const int pos = spos[k];
      const LRec s = S.get(k);
      PixEval e;
      if (!eval_pixel<LP>(s, lx, ly, e)) continue;
      const float Tn = T * (1.0f - e.alpha);
      if (Tn < kTMin) {
        done = true;
        stop = pos;
        continue;
      }
      const float w = e.alpha * T;
      cr = fmaf(w, s.r, cr);
      cg = fmaf(w, s.g, cg);
      cb = fmaf(w, s.b, cb);
      dep = fmaf(w, s.mz * e.iw, dep);
      nx = fmaf(w, s.n0, nx);
      ny = fmaf(w, s.n1, ny);
      nz = fmaf(w, s.n2, nz);
      T = Tn;
      ++blended;
      last = pos + 1;
      if (TOPK) {
        // a later position loses ties, so the new entry enters iff its key
        // exceeds the minimum key; it replaces the minimum, then the new
        // minimum is found (branch-free selects)
        const uint64_t key = ((uint64_t)__float_as_uint(w) << 32) | (uint32_t)~(uint32_t)pos;
        if (key > kmin) {
#pragma unroll
          for (int q = 0; q < KMAX; ++q) hk[q] = q == imin ? key : hk[q];
          kmin = hk[0];
          imin = 0;
#pragma unroll
          for (int q = 1; q < KMAX; ++q) {
            const bool lt = hk[q] < kmin;
            kmin = lt ? hk[q] : kmin;
            imin = lt ? q : imin;
          }
        }
        // feature-only rendering: with K weights held, a later weight is
        // alpha T' <= fl(0.99 T) (alpha <= 0.99, T' <= T, rounding is
        // monotone) and loses a tie, so once fl(0.99 T) <= the smallest held
        // weight the selection is final and the pixel stops
        if (feat_only && kmin != 0ull && kAlphaMax * T <= __uint_as_float((uint32_t)(kmin >> 32))) {
          done = true;
          stop = pos;
        }
      }
    }
  }
  // list entries this pixel walked: up to and including its stop, or all
  const int walked = !inside ? 0 : (stop >= 0 ? stop + 1 : L);

  const int sp = tile * kTilePix + tid;
  nlast[sp] = (uint32_t)last;
  tfinal[sp] = T;
  {
    int wsum = walked, bsum = blended, lsum = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      wsum += __shfl_xor(wsum, o, 64);
      bsum += __shfl_xor(bsum, o, 64);
      lsum += __shfl_xor(lsum, o, 64);
    }
    if ((tid & 63) == 0) {
      atomicAdd(reinterpret_cast<unsigned long long*>(status + kStWalked), (unsigned long long)wsum);
      atomicAdd(reinterpret_cast<unsigned long long*>(status + kStBlended), (unsigned long long)bsum);
      atomicAdd(reinterpret_cast<unsigned long long*>(status + kStBwdEntries), (unsigned long long)lsum);
    }
  }
  if (inside) {
    const int64_t pix = tl.pix0 + (int64_t)py * W + px;
    if (o_rgb) {
      o_rgb[3 * pix] = cr;
      o_rgb[3 * pix + 1] = cg;
      o_rgb[3 * pix + 2] = cb;
    }
    if (o_depth) o_depth[pix] = dep;
    if (o_normal) {
      o_normal[3 * pix] = nx;
      o_normal[3 * pix + 1] = ny;
      o_normal[3 * pix + 2] = nz;
    }
    if (o_alpha) o_alpha[pix] = 1.0f - T;
  }
  if (TOPK) {
    float hw[KMAX];
    int hp[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      const bool used = q < K && hk[q] != 0ull;
      hw[q] = __uint_as_float((uint32_t)(hk[q] >> 32));
      hp[q] = used ? (int)~(uint32_t)hk[q] : 0x7FFFFFFF;
    }
    sort_by_position<KMAX>(hp, hw);
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      if (q < K) {
        const size_t o = ((size_t)tile * K + q) * kTilePix + tid;
        const bool ok = hp[q] != 0x7FFFFFFF;
        selpos[o] = ok ? hp[q] : -1;
        selw[o] = ok ? hw[q] : 0.0f;
      }
    }
  }
  });
}

// ---------------------------------------------------------------- features
// Stages channels [cc, cc + BC) of the chunk's ns slot rows into s_F (row
// stride BC + 4 floats).
template <typename FT, int BC>
__device__ __forceinline__ void stage_rows(float* s_F, const uint32_t* fid, int ns, const FeatSrc<FT>& feat,
                                           int C, int cc) {
  for (int item = threadIdx.x; item < ns * (BC / 4); item += 256) {
    const int s = item / (BC / 4), j = item % (BC / 4), c = cc + 4 * j;
    const float4 f = c < C ? feat.load4(fid[s], c) : make_float4(0.f, 0.f, 0.f, 0.f);
    *reinterpret_cast<float4*>(s_F + s * (BC + 4) + 4 * j) = f;
  }
}

// Adds the selections of this thread's pixel that fall in the staged chunk
// (sl[q] = chunk slot or -1), in ascending list position.
template <int KMAX, int BC>
__device__ __forceinline__ void blend_chunk(const float* s_F, const int (&sl)[KMAX], const float (&w)[KMAX], int K,
                                            float (&acc)[BC]) {
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    if (q < K && sl[q] >= 0) {
      const float* fr = s_F + sl[q] * (BC + 4);
#pragma unroll
      for (int c = 0; c < BC; c += 4) {
        const float4 f = *reinterpret_cast<const float4*>(fr + c);
        acc[c] = fmaf(w[q], f.x, acc[c]);
        acc[c + 1] = fmaf(w[q], f.y, acc[c + 1]);
        acc[c + 2] = fmaf(w[q], f.z, acc[c + 2]);
        acc[c + 3] = fmaf(w[q], f.w, acc[c + 3]);
      }
    }
  }
}

// Thread per pixel; the tile's distinct selected rows are staged in LDS once
// per pass of BC channels and read by slot.  Two passes over the tiles:
//   WIDE = false: tiles whose selected positions fit one ranking window and
//     whose distinct rows fit one staged chunk (the common case): rank once,
//     stage and blend per channel pass.  Other tiles are appended to a list.
//   WIDE = false leaves out the windowed code, which keeps its registers (and
//     so its occupancy) to what the common case needs.
//   WIDE = true: the listed tiles, window by window and chunk by chunk.
// Both take a pixel's selections in ascending list position, so a tile's
// result does not depend on the pass that blends it.
template <typename FT, int KMAX, int BC, bool PERSIST, bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WIDE || KMAX > 16 ? 1 : 4))) void k_blend_topk(const uint32_t* __restrict__ pid, const uint2* __restrict__ ranges,
                                                    const int32_t* __restrict__ selpos,
                                                    const float* __restrict__ selw, const FeatSrc<FT> feat,
                                                    int C, int K, CamTable ct, TileQueue tq,
                                                    float* __restrict__ o_feat, int renorm,
                                                    uint32_t* __restrict__ wide, uint32_t* __restrict__ status) {
  __shared__ SelShared S;
  constexpr int kBRow = BC + 4;
  __shared__ __align__(16) float s_F[kSlotChunk * kBRow];
  __shared__ int s_item;
  auto body = [&](const int tile) {
  const TileLoc tl = locate(ct, tile);
  const int tid = threadIdx.x;
  const int px = tl.tx * ct.tw + tile_lx(ct, tid), py = tl.ty * ct.th + tile_ly(ct, tid);
  const bool inside = px < tl.W && py < tl.H;
  const uint32_t start = ranges[tile].x;
  const size_t tbase = (size_t)tile * K * kTilePix;
  float* out = o_feat + (tl.pix0 + (int64_t)py * tl.W + px) * C;

  int pos[KMAX];
  float w[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    pos[q] = q < K ? selpos[tbase + (size_t)q * kTilePix + tid] : -1;
    w[q] = q < K ? selw[tbase + (size_t)q * kTilePix + tid] : 0.0f;
  }
  // list positions are below the tile's list length, which bounds the
  // windows (no block-wide maximum of the selections needed)
  const int maxpos = (int)(ranges[tile].y - start) - 1;
  float wsum = 0.0f;
#pragma unroll
  for (int q = 0; q < KMAX; ++q) wsum += pos[q] >= 0 ? w[q] : 0.0f;
  const float rw = wsum > 0.0f ? 1.0f / wsum : 0.0f;
  // writes channels [cc, cc + BC) of this pixel's feature row
  auto put = [&](int cc, float (&acc)[BC]) {
    if (inside) {
      if (renorm) {  // renormalised Top-K: the selected weights scaled to sum 1
#pragma unroll
        for (int c = 0; c < BC; ++c) acc[c] *= rw;
      }
#pragma unroll
      for (int c = 0; c < BC; c += 4)
        if (cc + c < C)
          *reinterpret_cast<float4*>(out + cc + c) = make_float4(acc[c], acc[c + 1], acc[c + 2], acc[c + 3]);
    }
  };
  // the same write after an in-register transpose among groups of BC / 4
  // lanes (pixels adjacent in x): lane g of a group then holds channel quad g
  // of each of the group's pixels, so every store instruction writes whole
  // BC-channel segments of consecutive pixels' rows instead of 16 bytes of 64
  // rows; every lane takes part in the exchanges
  auto put_rows = [&](int cc, float (&acc)[BC]) {
    constexpr int NQ = BC / 4;
    if (renorm) {
#pragma unroll
      for (int c = 0; c < BC; ++c) acc[c] *= rw;
    }
    float4 a[NQ];
#pragma unroll
    for (int e = 0; e < NQ; ++e) a[e] = make_float4(acc[4 * e], acc[4 * e + 1], acc[4 * e + 2], acc[4 * e + 3]);
    const int gi = tid & (NQ - 1);
#pragma unroll
    for (int st = 1; st < NQ; st <<= 1) {
      const bool hi = (gi & st) != 0;
#pragma unroll
      for (int e = 0; e < NQ; ++e) {
        if (e & st) continue;
        const float4 x = hi ? a[e] : a[e | st];
        const float4 y = make_float4(__shfl_xor(x.x, st, 64), __shfl_xor(x.y, st, 64), __shfl_xor(x.z, st, 64),
                                     __shfl_xor(x.w, st, 64));
        if (hi) a[e] = y;
        else a[e | st] = y;
      }
    }
    const int base = tid & ~(NQ - 1);
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int p = base + k;
      const int qx = tl.tx * ct.tw + tile_lx(ct, p), qy = tl.ty * ct.th + tile_ly(ct, p);
      if (qx < tl.W && qy < tl.H && cc + 4 * gi < C)
        *reinterpret_cast<float4*>(o_feat + (tl.pix0 + (int64_t)qy * tl.W + qx) * C + cc + 4 * gi) = a[k];
    }
  };

  if constexpr (!WIDE) {
    // one window whose slots fit one chunk: rank once, stage per channel pass
    int sl[KMAX];
    int U = 0;
    const bool one_window = maxpos < kWinPos;
    if (maxpos >= 0 && one_window) {
      U = build_window(S, pos, K, 0, window_words(maxpos, 0));
#pragma unroll
      for (int q = 0; q < KMAX; ++q) sl[q] = q < K ? slot_of(S, pos[q], 0, window_words(maxpos, 0)) : -1;
    }
    const bool cached = maxpos < 0 || (one_window && U <= kSlotChunk);  // block-uniform
    if (!cached) {
      if (tid == 0) wide[atomicAdd(&status[kStWide], 1u)] = (uint32_t)tile;
      return;
    }
    if (maxpos >= 0) {
#pragma unroll
      for (int q = 0; q < KMAX; ++q)
        if (sl[q] >= 0) S.fid[sl[q]] = (uint32_t)(pid[start + pos[q]] - tl.v0);
    }
    __syncthreads();
    for (int cc = 0; cc < C; cc += BC) {
      float acc[BC];
#pragma unroll
      for (int c = 0; c < BC; ++c) acc[c] = 0.0f;
      if (maxpos >= 0) {
        stage_rows<FT, BC>(s_F, S.fid, U, feat, C, cc);
        __syncthreads();
        blend_chunk<KMAX, BC>(s_F, sl, w, K, acc);
        __syncthreads();
      }
      put_rows(cc, acc);
    }
  } else {
    for (int cc = 0; cc < C; cc += BC) {
      float acc[BC];
#pragma unroll
      for (int c = 0; c < BC; ++c) acc[c] = 0.0f;
      for (int w0 = 0; w0 <= maxpos; w0 += kWinPos) {
        const int nw = window_words(maxpos, w0);
        const int Uw = build_window(S, pos, K, w0, nw);
        for (int c0 = 0; c0 < Uw; c0 += kSlotChunk) {
          const int ns = min(kSlotChunk, Uw - c0);
          int sq[KMAX];
#pragma unroll
          for (int q = 0; q < KMAX; ++q) {
            const int s = q < K ? slot_of(S, pos[q], w0, nw) : -1;
            sq[q] = (s >= c0 && s < c0 + ns) ? s - c0 : -1;
            if (sq[q] >= 0) S.fid[sq[q]] = (uint32_t)(pid[start + pos[q]] - tl.v0);
          }
          __syncthreads();
          stage_rows<FT, BC>(s_F, S.fid, ns, feat, C, cc);
          __syncthreads();
          blend_chunk<KMAX, BC>(s_F, sq, w, K, acc);
          __syncthreads();
        }
      }
      put(cc, acc);
    }
  }
  };
  if constexpr (WIDE) {
    const uint32_t nwide = status[kStWide];
    for (uint32_t i = blockIdx.x; i < nwide; i += gridDim.x) {
      __syncthreads();  // the previous tile's LDS reads are done
      body((int)wide[i]);
    }
  } else {
    for_tiles<PERSIST>(tq, &s_item, body);
  }
}

constexpr int kFullBatch = 64;

template <typename FT, int CH, bool PERSIST, bool LP>
__global__ __launch_bounds__(256) void k_full_feat(const WalkRec* __restrict__ rec, const uint32_t* __restrict__ pid,
                                                   const uint2* __restrict__ ranges, const FeatSrc<FT> feat,
                                                   int C, CamTable ct, TileQueue tq,
                                                   const uint32_t* __restrict__ nlast, float* __restrict__ o_feat) {
  __shared__ Staged<kFullBatch> s_r;
  __shared__ float s_f[kFullBatch][CH];
  __shared__ uint32_t s_id[kFullBatch];
  __shared__ int s_lmax;
  __shared__ int s_item;
  for_tiles<PERSIST>(tq, &s_item, [&](const int tile) {
  const TileLoc tl = locate(ct, tile);
  const int tid = threadIdx.x;
  const int tx = tl.tx, ty = tl.ty;
  const int qx = tile_lx(ct, tid), qy = tile_ly(ct, tid);
  const int px = tx * ct.tw + qx, py = ty * ct.th + qy;
  const bool inside = px < tl.W && py < tl.H;
  const float lx = (float)qx + 0.5f, ly = (float)qy + 0.5f;
  const uint32_t start = ranges[tile].x;
  const int my_last = (int)nlast[tile * kTilePix + tid];
  __syncthreads();
  if (tid == 0) s_lmax = 0;
  __syncthreads();
  atomicMax(&s_lmax, my_last);
  __syncthreads();
  const int Lw = s_lmax;
  for (int c0 = 0; c0 < C; c0 += CH) {
    float acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = 0.0f;
    float T = 1.0f;
    for (int base = 0; base < Lw; base += kFullBatch) {
      const int nb = min(kFullBatch, Lw - base);
      __syncthreads();
      if (tid < nb) {
        const uint32_t id = pid[start + base + tid];
        s_id[tid] = (uint32_t)(id - tl.v0);
        s_r.put(tid, rec[id], (float)(tx * ct.tw), (float)(ty * ct.th));
      }
      __syncthreads();
      for (int e = tid; e < nb * CH; e += 256) {
        const int k = e / CH, c = e % CH;
        float v = 0.0f;
        if (c0 + c < C) {
          v = feat.load1(s_id[k], c0 + c);
        }
        s_f[k][c] = v;
      }
      __syncthreads();
      for (int k = 0; k < nb; ++k) {
        if (base + k >= my_last) break;
        const LRec s = s_r.get(k);
        PixEval ev;
        if (!eval_pixel<LP>(s, lx, ly, ev)) continue;
        const float w = ev.alpha * T;
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] = fmaf(w, s_f[k][c], acc[c]);
        T = T * (1.0f - ev.alpha);
      }
    }
    if (inside) {
      float* out = o_feat + (tl.pix0 + (int64_t)py * tl.W + px) * C + c0;
      const int cn = min(CH, C - c0);
#pragma unroll
      for (int c = 0; c < CH; c += 4)
        if (c < cn) *reinterpret_cast<float4*>(out + c) = make_float4(acc[c], acc[c + 1], acc[c + 2], acc[c + 3]);
    }
  }
  });
}

__global__ __launch_bounds__(256) void k_export_sel(const uint32_t* __restrict__ pid, const uint2* __restrict__ ranges,
                                                    const int32_t* __restrict__ selpos,
                                                    const float* __restrict__ selw,
                                                    const uint32_t* __restrict__ nlast,
                                                    const float* __restrict__ tfinal, int K, CamTable ct,
                                                    int32_t* __restrict__ o_id, float* __restrict__ o_w,
                                                    int32_t* __restrict__ o_nlast, float* __restrict__ o_tf) {
  const int tile = blockIdx.x;
  const int tid = threadIdx.x;
  const TileLoc tl = locate(ct, tile);
  const int px = tl.tx * ct.tw + tile_lx(ct, tid), py = tl.ty * ct.th + tile_ly(ct, tid);
  if (px >= tl.W || py >= tl.H) return;
  const int64_t pix = tl.pix0 + (int64_t)py * tl.W + px;
  const uint32_t start = ranges[tile].x;
  for (int q = 0; q < K; ++q) {
    const size_t o = ((size_t)tile * K + q) * kTilePix + tid;
    const int pos = selpos ? selpos[o] : -1;
    if (o_id) o_id[pix * K + q] = pos >= 0 ? (int32_t)(pid[start + pos] - tl.v0) : -1;
    if (o_w) o_w[pix * K + q] = pos >= 0 ? selw[o] : 0.0f;
  }
  if (o_nlast) o_nlast[pix] = (int32_t)nlast[tile * kTilePix + tid];
  if (o_tf) o_tf[pix] = tfinal[tile * kTilePix + tid];
}

// Marks the virtual surfel of every held selection in a bitmap (block per
// tile, thread per pixel), counts the selections and the tile's distinct
// selected list positions (its (tile, surfel) pairs with a selection: the
// feature rows the Top-K backward writes per tile); k_count_bits then counts
// the marked surfels.  Stats read-back only, not part of a render.
__global__ __launch_bounds__(256) void k_mark_selected(const uint32_t* __restrict__ pid,
                                                       const uint2* __restrict__ ranges,
                                                       const int32_t* __restrict__ selpos, int K,
                                                       uint32_t* __restrict__ bits, uint32_t* __restrict__ status) {
  __shared__ SelShared S;
  const int tile = blockIdx.x;
  const int tid = threadIdx.x;
  const uint2 rg = ranges[tile];
  const uint32_t start = rg.x;
  const int len = (int)(rg.y - rg.x);
  int held = 0, maxpos = -1;
  int pos[kMaxK];
#pragma unroll
  for (int q = 0; q < kMaxK; ++q) {
    const int p = q < K ? selpos[((size_t)tile * K + q) * kTilePix + tid] : -1;
    pos[q] = p >= 0 && p < len ? p : -1;  // a position outside the list (no Top-K forward ran) is not followed
    if (pos[q] >= 0) {
      const uint32_t v = pid[start + pos[q]];
      atomicOr(bits + (v >> 5), 1u << (v & 31u));
      ++held;
      maxpos = max(maxpos, pos[q]);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) held += __shfl_xor(held, o, 64);
  if ((tid & 63) == 0 && held)
    atomicAdd(reinterpret_cast<unsigned long long*>(status + kStSelected), (unsigned long long)held);
  // distinct selected positions, window by window (the bound is block-uniform)
  const int mp = block_max(maxpos, S.red);
  int distinct = 0;
  for (int w0 = 0; w0 <= mp; w0 += kWinPos) distinct += build_window<kMaxK>(S, pos, K, w0, window_words(mp, w0));
  if (tid == 0 && distinct)
    atomicAdd(reinterpret_cast<unsigned long long*>(status + kStSelPairs), (unsigned long long)distinct);
}

__global__ __launch_bounds__(256) void k_count_bits(const uint32_t* __restrict__ bits, int64_t words,
                                                    uint32_t* __restrict__ status) {
  int cnt = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256)
    cnt += __popc(bits[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0 && cnt)
    atomicAdd(reinterpret_cast<unsigned long long*>(status + kStUnique), (unsigned long long)cnt);
}

// ------------------------------------------------------------- host wrappers
template <int KMAX, bool TOPK, bool PERSIST, bool LP, bool KFULL>
static void walk_launch_k(const Layout& L, const CamTable& ct, const Tuning& tu, const ImageArgs& out,
                          bool feat_only, char* ws, hipStream_t st) {
  const void* k = reinterpret_cast<const void*>(&k_walk<KMAX, TOPK, PERSIST, LP, KFULL>);
  hipLaunchKernelGGL((k_walk<KMAX, TOPK, PERSIST, LP, KFULL>), dim3(tile_grid(L, tu.sched, k, 0)), dim3(256), 0, st,
                     (const WalkRec*)(ws + L.rec), (const float4*)(ws + L.ext), (const uint32_t*)(ws + L.pid),
                     (const uint2*)(ws + L.ranges), ct, tile_queue(L, tu.sched, ws, kQWalk), L.k, out.rgb, out.depth,
                     out.normal, out.alpha,
                     (uint32_t*)(ws + L.nlast), (float*)(ws + L.tfinal), (int32_t*)(ws + L.selpos),
                     (float*)(ws + L.selw), (uint32_t*)(ws + L.status), feat_only ? 1 : 0);
}

template <int KMAX, bool TOPK, bool PERSIST, bool LP>
static void walk_launch_t(const Layout& L, const CamTable& ct, const Tuning& tu, const ImageArgs& out,
                          bool feat_only, char* ws, hipStream_t st) {
  if constexpr (TOPK) {
    if (L.k == KMAX) {
      walk_launch_k<KMAX, TOPK, PERSIST, LP, true>(L, ct, tu, out, feat_only, ws, st);
      return;
    }
  }
  walk_launch_k<KMAX, TOPK, PERSIST, LP, false>(L, ct, tu, out, feat_only, ws, st);
}

template <int KMAX, bool TOPK>
static void walk_launch(const Layout& L, const CamTable& ct, const Tuning& tu, const ImageArgs& out, bool feat_only,
                        bool lp, char* ws, hipStream_t st) {
  const bool p = tu.sched == kSchedPersistent;
  if (lp)
    (p ? walk_launch_t<KMAX, TOPK, true, true> : walk_launch_t<KMAX, TOPK, false, true>)(L, ct, tu, out, feat_only, ws,
                                                                                       st);
  else
    (p ? walk_launch_t<KMAX, TOPK, true, false> : walk_launch_t<KMAX, TOPK, false, false>)(L, ct, tu, out, feat_only,
                                                                                         ws, st);
}

void launch_walk(const Layout& L, const CamTable& ct, int blend, const Tuning& tu, const ImageArgs& out,
                 bool feat_only, bool lowpass, char* ws, hipStream_t st) {
  if (L.tiles == 0) return;
  if (blend == kFull) {
    walk_launch<1, false>(L, ct, tu, out, false, lowpass, ws, st);
  } else if (L.k <= 8) {
    walk_launch<8, true>(L, ct, tu, out, feat_only, lowpass, ws, st);
  } else if (L.k <= 16) {
    walk_launch<16, true>(L, ct, tu, out, feat_only, lowpass, ws, st);
  } else {
    walk_launch<32, true>(L, ct, tu, out, feat_only, lowpass, ws, st);
  }
}

template <typename FT, int KMAX, int BC, bool PERSIST>
static void blend_topk_launch(const SurfelArgs& s, const Layout& L, const CamTable& ct, const Tuning& tu,
                              float* out_feat, bool renorm, char* ws, hipStream_t st) {
  uint32_t* status = (uint32_t*)(ws + L.status);
  uint32_t* wide = (uint32_t*)(ws + L.wide);
  launch_fill_u32(status + kStWide, 0u, 1, st);
  const void* k = reinterpret_cast<const void*>(&k_blend_topk<FT, KMAX, BC, PERSIST, false>);
  const int sched = PERSIST ? kSchedPersistent : kSchedGrid;
  hipLaunchKernelGGL((k_blend_topk<FT, KMAX, BC, PERSIST, false>), dim3(tile_grid(L, sched, k, 0)), dim3(256), 0,
                     st, (const uint32_t*)(ws + L.pid), (const uint2*)(ws + L.ranges), (const int32_t*)(ws + L.selpos),
                     (const float*)(ws + L.selw), feat_src<FT>(s), s.c, L.k, ct, tile_queue(L, sched, ws, kQBlend),
                     out_feat, renorm ? 1 : 0, wide, status);
  // the listed tiles (usually none): a fixed grid strides over the list,
  // whose length it reads on the device
  const unsigned gw = (unsigned)std::min<int64_t>(L.tiles, 1024);
  hipLaunchKernelGGL((k_blend_topk<FT, KMAX, BC, false, true>), dim3(gw), dim3(256), 0, st,
                     (const uint32_t*)(ws + L.pid), (const uint2*)(ws + L.ranges), (const int32_t*)(ws + L.selpos),
                     (const float*)(ws + L.selw), feat_src<FT>(s), s.c, L.k, ct, TileQueue{nullptr, nullptr, 0},
                     out_feat, renorm ? 1 : 0, wide, status);
}

template <typename FT, int BC>
static void blend_topk_k(const SurfelArgs& s, const Layout& L, const CamTable& ct, const Tuning& tu, float* out_feat,
                         bool rn, char* ws, hipStream_t st) {
  // always grid-scheduled: with the long tiles moved to the windowed pass the
  // common pass's tiles cost about the same, and the grid form keeps fewer
  // registers live across tiles (more waves per SIMD)
  if (L.k <= 8) blend_topk_launch<FT, 8, BC, false>(s, L, ct, tu, out_feat, rn, ws, st);
  else if (L.k <= 16) blend_topk_launch<FT, 16, BC, false>(s, L, ct, tu, out_feat, rn, ws, st);
  else blend_topk_launch<FT, 32, BC, false>(s, L, ct, tu, out_feat, rn, ws, st);
}

template <typename FT, bool PERSIST, bool LP>
static void full_feat_launch(const SurfelArgs& s, const Layout& L, const CamTable& ct, const Tuning& tu,
                             float* out_feat, char* ws, hipStream_t st) {
  const void* k = reinterpret_cast<const void*>(&k_full_feat<FT, 64, PERSIST, LP>);
  hipLaunchKernelGGL((k_full_feat<FT, 64, PERSIST, LP>), dim3(tile_grid(L, tu.sched, k, 0)), dim3(256), 0, st,
                     (const WalkRec*)(ws + L.rec), (const uint32_t*)(ws + L.pid), (const uint2*)(ws + L.ranges),
                     feat_src<FT>(s), s.c, ct, tile_queue(L, tu.sched, ws, kQBlend), (const uint32_t*)(ws + L.nlast),
                     out_feat);
}

template <typename FT>
static void blend_launch(const SurfelArgs& s, const Layout& L, const CamTable& ct, int blend, const Tuning& tu,
                         float* out_feat, bool renorm, bool lp, char* ws, hipStream_t st) {
  const bool p = tu.sched == kSchedPersistent;
  if (blend == kTopK) {
    if (tu.blend_pass == 16) blend_topk_k<FT, 16>(s, L, ct, tu, out_feat, renorm, ws, st);
    else blend_topk_k<FT, 32>(s, L, ct, tu, out_feat, renorm, ws, st);
  } else if (lp) {
    (p ? full_feat_launch<FT, true, true> : full_feat_launch<FT, false, true>)(s, L, ct, tu, out_feat, ws, st);
  } else {
    (p ? full_feat_launch<FT, true, false> : full_feat_launch<FT, false, false>)(s, L, ct, tu, out_feat, ws, st);
  }
}

void launch_feature_blend(const SurfelArgs& s, const Layout& L, const CamTable& ct, int blend, const Tuning& tu,
                          float* out_feat, bool renorm, bool lowpass, char* ws, hipStream_t st) {
  if (!out_feat || s.c <= 0 || L.tiles == 0) return;
  if (s.dtype == kF32) blend_launch<float>(s, L, ct, blend, tu, out_feat, renorm, lowpass, ws, st);
  else if (s.dtype == kF16) blend_launch<__half>(s, L, ct, blend, tu, out_feat, renorm, lowpass, ws, st);
  else blend_launch<uint16_t>(s, L, ct, blend, tu, out_feat, renorm, lowpass, ws, st);
}

void launch_count_selected(const Layout& L, char* ws, hipStream_t st) {
  uint32_t* status = (uint32_t*)(ws + L.status);
  const int64_t words = cdiv(L.n > 0 ? L.n : 1, 32);
  launch_fill_u32(ws + L.ubits, 0u, words, st);
  launch_fill_u32(status + kStUnique, 0u, 6, st);
  if (L.tiles == 0) return;
  hipLaunchKernelGGL(k_mark_selected, dim3((unsigned)L.tiles), dim3(256), 0, st, (const uint32_t*)(ws + L.pid),
                     (const uint2*)(ws + L.ranges), (const int32_t*)(ws + L.selpos), L.k, (uint32_t*)(ws + L.ubits),
                     status);
  const int64_t blocks = std::min<int64_t>(1024, cdiv(words, 256));
  hipLaunchKernelGGL(k_count_bits, dim3((unsigned)blocks), dim3(256), 0, st, (const uint32_t*)(ws + L.ubits), words,
                     status);
}

void launch_export_selection(const Layout& L, const CamTable& ct, char* ws, int32_t* sel_id, float* sel_w,
                             int32_t* n_last, float* t_final, hipStream_t st) {
  if (L.tiles == 0) return;
  hipLaunchKernelGGL(k_export_sel, dim3((unsigned)L.tiles), dim3(256), 0, st, (const uint32_t*)(ws + L.pid),
                     (const uint2*)(ws + L.ranges), (const int32_t*)(ws + L.selpos), (const float*)(ws + L.selw),
                     (const uint32_t*)(ws + L.nlast), (const float*)(ws + L.tfinal), L.k, ct, sel_id, sel_w, n_last,
                     t_final);
}

}  // namespace psm
