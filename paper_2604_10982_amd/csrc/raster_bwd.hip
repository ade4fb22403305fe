// Backward of the renderer: gradients of L = <upstream, outputs> with respect
// to every surfel parameter.  The selection (eq. (18)), the contributor set,
// the stop point and the alpha clamp are held fixed.
//
// Deterministic and free of floating-point atomics: every (tile, surfel) pair
// of the sorted list owns a slot at its sorted index for its partial sums,
// and a per-surfel pass later adds its own slots in a fixed order (the pair
// sort recorded where each surfel's pairs went).
//
// k_feat_bwd_topk: per tile, for every (pixel, selected surfel): the dot
//   product of the pixel's feature gradient with the surfel's feature row
//   (needed by the alpha adjoint); and, per distinct selected surfel of the
//   tile, the row sum_p w_p g_F(p) over the pixels that selected it, in pixel
//   order (per-slot pixel masks give each entry its rank without atomics on
//   floats).
// k_walk_bwd: per tile, back to front from each pixel's last contributor,
//   recovering T_i = T_{i+1} / (1 - alpha_i).  Per surfel the per-pixel terms
//   are reduced over the wave, then over the 4 waves through LDS, and written
//   as the pair's 16 partial sums.  In dense-blend mode each batch also forms
//   the feature dot products and feature-gradient rows tile-wide.
// k_reduce_geo / k_reduce_feat: per surfel, sum of its pairs' partials, then
//   the chain rule to mu, s, q (FP64, as the forward's walk record).
#include "common.h"
#include "internal.h"

namespace psm {

constexpr int kBB = 32;          // surfels per backward batch
constexpr int kNV = 17;          // per-pixel values reduced per surfel
constexpr int kWinWords = 1024;  // selected-position window: 32768 positions

// ------------------------------------------------------------ Top-K feature
constexpr int kSlotChunk = 256;  // distinct selected surfels handled per pass

// Position (within the window) of the s-th set bit of the window bitmap.
__device__ __forceinline__ int slot_position(const uint32_t* bits, const uint32_t* pref, int s) {
  int lo = 0, hi = kWinWords - 1;  // largest word w with pref[w] <= s
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int)pref[mid] <= s) lo = mid;
    else hi = mid - 1;
  }
  uint32_t w = bits[lo];
  for (int r = s - (int)pref[lo]; r > 0; --r) w &= w - 1u;
  return lo * 32 + (__ffs(w) - 1);
}

template <typename FT>
__global__ __launch_bounds__(256) void k_feat_bwd_topk(
    const uint32_t* __restrict__ pid, const uint2* __restrict__ ranges, const int32_t* __restrict__ selpos,
    const float* __restrict__ selw, const FT* __restrict__ feat, const float* __restrict__ gfeat, int C, int K,
    int W, int H, int ntx, int tiles, float* __restrict__ seldot, float* __restrict__ fpart,
    uint8_t* __restrict__ fflag) {
  extern __shared__ char smem[];
  uint32_t* s_bits = reinterpret_cast<uint32_t*>(smem);  // selected positions of the window
  uint32_t* s_pref = s_bits + kWinWords;                   // exclusive popcount prefix per word
  uint32_t* s_mask = s_pref + kWinWords;                   // [kSlotChunk][8] pixels selecting a slot
  uint32_t* s_off = s_mask + kSlotChunk * 8;               // [kSlotChunk + 1] entry offsets
  uint32_t* s_list = s_off + kSlotChunk + 1;               // [256 K] entries (pixel | k << 8)
  __shared__ int s_maxpos;
  __shared__ uint32_t s_wsum[256];

  const int tile = xcd_tile(blockIdx.x, tiles);
  if (tile >= tiles) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tx = tile % ntx, ty = tile / ntx;
  const uint32_t start = ranges[tile].x;
  constexpr int V = VecN<FT>::N;
  const int lpp = C / V;
  const int lpp2 = lpp >= 64 ? 64 : pow2_ge(lpp);
  const int ppw = 64 / lpp2;
  const int sub = lane / lpp2, cl = lane % lpp2;
  const size_t tbase = (size_t)tile * K * kTilePix;

  // --- dot products g_F(p) . f_j for the selected j (front-to-back slots)
  for (int p0 = 0; p0 < 64; p0 += ppw) {
    const int p = wave * 64 + p0 + sub;
    const int px = tx * kTile + (p & 15), py = ty * kTile + (p >> 4);
    const bool in = px < W && py < H;
    const float* grow = gfeat + ((int64_t)py * W + px) * C;
    for (int q = 0; q < K; ++q) {
      const int pos = in ? selpos[tbase + (size_t)q * kTilePix + p] : -1;
      float part = 0.0f;
      if (pos >= 0) {
        const uint32_t id = pid[start + pos];
        for (int cg = cl; cg < lpp; cg += lpp2) {
          float f[V];
          load_vec<FT>(feat + (size_t)id * C + cg * V, f);
#pragma unroll
          for (int v = 0; v < V; v += 4) {
            const float4 x = *reinterpret_cast<const float4*>(grow + cg * V + v);
            part = fmaf(x.x, f[v], part);
            part = fmaf(x.y, f[v + 1], part);
            part = fmaf(x.z, f[v + 2], part);
            part = fmaf(x.w, f[v + 3], part);
          }
        }
      }
      for (int o = lpp2 >> 1; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
      if (cl == 0) seldot[tbase + (size_t)q * kTilePix + p] = pos >= 0 ? part : 0.0f;
    }
  }

  // --- dL/df rows, one per distinct selected (tile, surfel) pair
  if (tid == 0) s_maxpos = -1;
  __syncthreads();
  int mymax = -1;
  for (int q = 0; q < K; ++q) mymax = max(mymax, selpos[tbase + (size_t)q * kTilePix + tid]);
  atomicMax(&s_maxpos, mymax);
  __syncthreads();
  const int maxpos = s_maxpos;
  for (int w0 = 0; w0 <= maxpos; w0 += kWinWords * 32) {
    for (int i = tid; i < kWinWords; i += 256) s_bits[i] = 0u;
    __syncthreads();
    for (int q = 0; q < K; ++q) {
      const int pos = selpos[tbase + (size_t)q * kTilePix + tid] - w0;
      if (pos >= 0 && pos < kWinWords * 32) atomicOr(&s_bits[pos >> 5], 1u << (pos & 31));
    }
    __syncthreads();
    uint32_t c4 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) c4 += __popc(s_bits[tid * 4 + i]);
    s_wsum[tid] = c4;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const uint32_t v = tid >= o ? s_wsum[tid - o] : 0u;
      __syncthreads();
      s_wsum[tid] += v;
      __syncthreads();
    }
    uint32_t run = s_wsum[tid] - c4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s_pref[tid * 4 + i] = run;
      run += __popc(s_bits[tid * 4 + i]);
    }
    const int U = (int)s_wsum[255];
    __syncthreads();
    for (int c0 = 0; c0 < U; c0 += kSlotChunk) {
      const int ns = min(kSlotChunk, U - c0);
      for (int i = tid; i < ns * 8; i += 256) s_mask[i] = 0u;
      __syncthreads();
      // which pixels selected each slot of this chunk
      for (int q = 0; q < K; ++q) {
        const int pos = selpos[tbase + (size_t)q * kTilePix + tid] - w0;
        if (pos < 0 || pos >= kWinWords * 32) continue;
        const int slot = (int)(s_pref[pos >> 5] + __popc(s_bits[pos >> 5] & ((1u << (pos & 31)) - 1u))) - c0;
        if (slot >= 0 && slot < ns) atomicOr(&s_mask[slot * 8 + (tid >> 5)], 1u << (tid & 31));
      }
      __syncthreads();
      // entry offsets: exclusive scan of the slot populations
      uint32_t cnt = 0;
      if (tid < ns)
        for (int w = 0; w < 8; ++w) cnt += __popc(s_mask[tid * 8 + w]);
      s_wsum[tid] = cnt;
      __syncthreads();
      for (int o = 1; o < 256; o <<= 1) {
        const uint32_t v = tid >= o ? s_wsum[tid - o] : 0u;
        __syncthreads();
        s_wsum[tid] += v;
        __syncthreads();
      }
      if (tid < ns) s_off[tid] = s_wsum[tid] - cnt;
      if (tid == 0) s_off[ns] = s_wsum[ns - 1];
      __syncthreads();
      // entries in pixel order within each slot
      for (int q = 0; q < K; ++q) {
        const int pos = selpos[tbase + (size_t)q * kTilePix + tid] - w0;
        if (pos < 0 || pos >= kWinWords * 32) continue;
        const int slot = (int)(s_pref[pos >> 5] + __popc(s_bits[pos >> 5] & ((1u << (pos & 31)) - 1u))) - c0;
        if (slot < 0 || slot >= ns) continue;
        const uint32_t* m = s_mask + slot * 8;
        uint32_t rank = __popc(m[tid >> 5] & ((1u << (tid & 31)) - 1u));
        for (int w = 0; w < (tid >> 5); ++w) rank += __popc(m[w]);
        s_list[s_off[slot] + rank] = (uint32_t)tid | ((uint32_t)q << 8);
      }
      __syncthreads();
      // one lane group per slot: sum_p w_p g_F(p)
      for (int sb = wave * ppw; sb < ns; sb += 4 * ppw) {
        const int sl = sb + sub;
        if (sl < ns) {
          const int pos = w0 + slot_position(s_bits, s_pref, c0 + sl);
          const uint32_t e0 = s_off[sl], e1 = s_off[sl + 1];
          float* out = fpart + ((size_t)start + pos) * C;
          for (int cg = cl; cg < lpp; cg += lpp2) {
            float acc[V];
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = 0.0f;
            for (uint32_t e = e0; e < e1; ++e) {
              const uint32_t ent = s_list[e];
              const int p = (int)(ent & 255u), q = (int)(ent >> 8);
              const float w = selw[tbase + (size_t)q * kTilePix + p];
              const int px = tx * kTile + (p & 15), py = ty * kTile + (p >> 4);
              const float* grow = gfeat + ((int64_t)py * W + px) * C + cg * V;
#pragma unroll
              for (int v = 0; v < V; v += 4) {
                const float4 x = *reinterpret_cast<const float4*>(grow + v);
                acc[v] = fmaf(w, x.x, acc[v]);
                acc[v + 1] = fmaf(w, x.y, acc[v + 1]);
                acc[v + 2] = fmaf(w, x.z, acc[v + 2]);
                acc[v + 3] = fmaf(w, x.w, acc[v + 3]);
              }
            }
#pragma unroll
            for (int v = 0; v < V; v += 4)
              *reinterpret_cast<float4*>(out + cg * V + v) = make_float4(acc[v], acc[v + 1], acc[v + 2], acc[v + 3]);
          }
          if (cl == 0) fflag[start + pos] = 1;
        }
      }
      __syncthreads();
    }
    __syncthreads();  // the next window rewrites the bitmap
  }
}

// ------------------------------------------------------------- walk backward
template <int MODE, typename FT>
__global__ __launch_bounds__(256) void k_walk_bwd(
    const WalkRec* __restrict__ rec, const uint32_t* __restrict__ pid, const uint2* __restrict__ ranges, int W,
    int H, int ntx, int tiles, int K, const uint32_t* __restrict__ nlast, const float* __restrict__ tfinal,
    const int32_t* __restrict__ selpos, const float* __restrict__ seldot, const float* __restrict__ g_rgb,
    const float* __restrict__ g_depth, const float* __restrict__ g_normal, const float* __restrict__ g_alpha,
    const float* __restrict__ g_feat, const FT* __restrict__ feat, int C, float* __restrict__ gpart,
    uint8_t* __restrict__ gflag, float* __restrict__ fpart, uint8_t* __restrict__ fflag) {
  __shared__ Staged<kBB> s_r;
  __shared__ uint32_t s_id[kBB];
  __shared__ float s_part[4][kBB][kNV];
  __shared__ uint32_t s_has[4][kBB];
  __shared__ int s_lmax;
  // dense-blend mode only: feature chunk of the batch and the batch weights
  __shared__ float s_fc[MODE == kFull ? kBB : 1][64];
  __shared__ float s_om[MODE == kFull ? kBB : 1][kTilePix];

  const int tile = xcd_tile(blockIdx.x, tiles);
  if (tile >= tiles) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tx = tile % ntx, ty = tile / ntx;
  const int px = tx * kTile + (tid & 15), py = ty * kTile + (tid >> 4);
  const bool inside = px < W && py < H;
  const float lx = (float)(tid & 15) + 0.5f, ly = (float)(tid >> 4) + 0.5f;
  const float tx0 = (float)(tx * kTile), ty0 = (float)(ty * kTile);
  const uint32_t start = ranges[tile].x;
  const int sp = tile * kTilePix + tid;
  const int my_last = (int)nlast[sp];
  float T = tfinal[sp];
  const float Tfin = T;
  const int64_t pix = (int64_t)py * W + px;
  float gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gN0 = 0.f, gN1 = 0.f, gN2 = 0.f, gA = 0.f;
  if (inside) {
    if (g_rgb) { gC0 = g_rgb[3 * pix]; gC1 = g_rgb[3 * pix + 1]; gC2 = g_rgb[3 * pix + 2]; }
    if (g_depth) gD = g_depth[pix];
    if (g_normal) { gN0 = g_normal[3 * pix]; gN1 = g_normal[3 * pix + 1]; gN2 = g_normal[3 * pix + 2]; }
    if (g_alpha) gA = g_alpha[pix];
  }
  // Top-K: walk the saved selection from its back end
  int kp = -1, nextsel = -1;
  float nextdot = 0.0f;
  const size_t tbase = (size_t)tile * K * kTilePix;
  if (MODE == kTopK) {
    for (int q = 0; q < K; ++q)
      if (selpos[tbase + (size_t)q * kTilePix + tid] >= 0) kp = q;
    if (kp >= 0) {
      nextsel = selpos[tbase + (size_t)kp * kTilePix + tid];
      nextdot = seldot[tbase + (size_t)kp * kTilePix + tid];
    }
  }
  const bool has_gf = MODE == kFull && g_feat != nullptr && inside;
  const float* grow = g_feat + pix * C;

  if (tid == 0) s_lmax = 0;
  __syncthreads();
  atomicMax(&s_lmax, my_last);
  __syncthreads();
  const int Lmax = s_lmax;
  float suffix = 0.0f;

  for (int hi = Lmax; hi > 0; hi -= kBB) {
    const int lo = max(0, hi - kBB), nb = hi - lo;
    __syncthreads();
    if (tid < nb) {
      const uint32_t id = pid[start + lo + tid];
      s_id[tid] = id;
      s_r.put(tid, rec[id], tx0, ty0);
    }
    __syncthreads();

    // dense mode: phi[k] = g_F(p) . f_k for the batch (tile-wide product)
    float phi[MODE == kFull ? kBB : 1];
    if constexpr (MODE == kFull) {
#pragma unroll
      for (int k = 0; k < kBB; ++k) phi[k] = 0.0f;
      if (g_feat) {
        for (int c0 = 0; c0 < C; c0 += 64) {
          for (int e = tid; e < nb * 64; e += 256) {
            const int k = e >> 6, c = e & 63;
            s_fc[k][c] = (c0 + c < C) ? load_one<FT>(feat + (size_t)s_id[k] * C + c0 + c) : 0.0f;
          }
          __syncthreads();
          if (has_gf) {
            const int cn = min(64, C - c0);
            for (int c = 0; c < cn; c += 4) {
              const float4 g = *reinterpret_cast<const float4*>(grow + c0 + c);
#pragma unroll
              for (int k = 0; k < kBB; ++k)
                phi[k] = fmaf(g.x, s_fc[k][c], fmaf(g.y, s_fc[k][c + 1], fmaf(g.z, s_fc[k][c + 2], fmaf(g.w, s_fc[k][c + 3], phi[k]))));
            }
          }
          __syncthreads();
        }
      }
    }

#pragma unroll 1
    for (int k = nb - 1; k >= 0; --k) {
      const int pos = lo + k;
      float v[kNV];
#pragma unroll
      for (int i = 0; i < kNV; ++i) v[i] = 0.0f;
      bool contrib = false;
      float wgt = 0.0f;
      if (pos < my_last) {
        const LRec s = s_r.get(k);
        PixEval e;
        if (eval_pixel(s, lx, ly, e)) {
          contrib = true;
          const float one_m = 1.0f - e.alpha;
          const float Tb = T / one_m;
          const float w = e.alpha * Tb;
          wgt = w;
          const float u = e.u, vv = e.v, z = s.mz * e.iw;
          float eF = 0.0f;
          if (MODE == kTopK) {
            if (pos == nextsel) {
              eF = nextdot;
              --kp;
              nextsel = kp >= 0 ? selpos[tbase + (size_t)kp * kTilePix + tid] : -1;
              nextdot = kp >= 0 ? seldot[tbase + (size_t)kp * kTilePix + tid] : 0.0f;
            }
          } else {
#pragma unroll
            for (int q = 0; q < kBB; ++q)
              if (q == k) eF = phi[q];
          }
          const float ei = gC0 * s.r + gC1 * s.g + gC2 * s.b + gD * z + gN0 * s.n0 + gN1 * s.n1 + gN2 * s.n2 + eF;
          const float da = Tb * ei - (suffix - gA * Tfin) / one_m;
          suffix = fmaf(w, ei, suffix);
          T = Tb;
          const float dop = e.clamped ? 0.0f : da * e.G;
          const float drho = e.clamped ? 0.0f : -0.5f * da * e.alpha;
          const float du = 2.0f * u * drho, dv = 2.0f * vv * drho;
          const float dz = w * gD;
          const float du1 = du * e.iw, dv1 = dv * e.iw;
          const float dw1 = -(du * u + dv * vv + dz * z) * e.iw;
          v[0] = du1 * e.dx; v[1] = du1 * e.dy; v[2] = du1;
          v[3] = dv1 * e.dx; v[4] = dv1 * e.dy; v[5] = dv1;
          v[6] = dw1 * e.dx; v[7] = dw1 * e.dy; v[8] = dw1;
          v[9] = dz * e.iw;
          v[10] = dop;
          v[11] = w * gC0; v[12] = w * gC1; v[13] = w * gC2;
          v[14] = w * gN0; v[15] = w * gN1; v[16] = w * gN2;
        }
      }
      if constexpr (MODE == kFull) s_om[k][tid] = wgt;
      const bool any = __any(contrib);
      if (any) {
        float v16[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v16[i] = v[i];
        const float tot = wave_reduce16(v16);
        const float last = wave_sum(v[16]);
        if ((lane & 3) == 0) s_part[wave][k][(lane >> 2) & 15] = tot;
        if (lane == 0) s_part[wave][k][16] = last;
      }
      if (lane == 0) s_has[wave][k] = any ? 1u : 0u;
    }
    __syncthreads();

    // combine the 4 waves, convert to the 16 per-surfel accumulators
    if (tid < nb) {
      const int k = tid;
      if (s_has[0][k] | s_has[1][k] | s_has[2][k] | s_has[3][k]) {
        float t[kNV];
#pragma unroll
        for (int i = 0; i < kNV; ++i) {
          float a = 0.0f;
#pragma unroll
          for (int w = 0; w < 4; ++w) a += s_has[w][k] ? s_part[w][k][i] : 0.0f;
          t[i] = a;
        }
        const uint32_t id = s_id[k];
        const WalkRec& rr = rec[id];
        const float a00 = (float)rr.d0.x, a01 = (float)rr.d0.y, a10 = (float)rr.d1.x, a11 = (float)rr.d1.y;
        const float e0 = (float)rr.d2.x, e1 = (float)rr.d2.y;
        const size_t slot = (size_t)start + lo + k;
        float4* g = reinterpret_cast<float4*>(gpart + slot * 16);
        // u' = A^-1 d, w' = 1 - e.d with d = pixel - centre; d depends on the
        // centre with slope -1
        g[0] = make_float4(t[0], t[1], t[3], t[4]);
        g[1] = make_float4(-t[6], -t[7], -(a00 * t[2] + a10 * t[5] - e0 * t[8]),
                           -(a01 * t[2] + a11 * t[5] - e1 * t[8]));
        g[2] = make_float4(t[9], t[10], t[11], t[12]);
        g[3] = make_float4(t[13], t[14], t[15], t[16]);
        gflag[slot] = 1;
      }
    }

    // dense mode: dL/df_k = sum_p w_k(p) g_F(p) for the batch
    if constexpr (MODE == kFull) {
      if (g_feat) {
        __syncthreads();
        const int kg = wave;  // 4 groups of kBB/4 surfels
        constexpr int PER = kBB / 4;
        for (int c0 = 0; c0 < C; c0 += 64) {
          const int c = c0 + lane;
          float acc[PER];
#pragma unroll
          for (int j = 0; j < PER; ++j) acc[j] = 0.0f;
          if (c < C) {
            for (int p = 0; p < kTilePix; ++p) {
              const int qx = tx * kTile + (p & 15), qy = ty * kTile + (p >> 4);
              if (qx >= W || qy >= H) continue;
              const float g = g_feat[((int64_t)qy * W + qx) * C + c];
#pragma unroll
              for (int j = 0; j < PER; ++j) acc[j] = fmaf(s_om[kg * PER + j][p], g, acc[j]);
            }
#pragma unroll
            for (int j = 0; j < PER; ++j) {
              const int k = kg * PER + j;
              if (k < nb) {
                const size_t slot = (size_t)start + lo + k;
                fpart[slot * C + c] = acc[j];
                if (c == 0) fflag[slot] = 1;
              }
            }
          }
        }
      }
    }
  }
}

// ------------------------------------------------------- per-surfel reduction
struct CamB {
  float R[9], t[3], fx, fy, cx, cy;
};

// Thread per surfel, visited in depth order so its pairs are the emitted
// range [offs[r], offs[r] + count): their sorted slots come from `inv`.
__global__ __launch_bounds__(256) void k_reduce_geo(int64_t n, const uint32_t* __restrict__ order,
                                                    const uint32_t* __restrict__ count,
                                                    const uint32_t* __restrict__ offs,
                                                    const uint32_t* __restrict__ inv, int64_t cap,
                                                    const float* __restrict__ gpart,
                                                    const uint8_t* __restrict__ gflag,
                                                    const float* __restrict__ means, const float* __restrict__ scales,
                                                    const float* __restrict__ quats, const int32_t* __restrict__ cull,
                                                    CamB k, float* __restrict__ d_means, float* __restrict__ d_scales,
                                                    float* __restrict__ d_quats, float* __restrict__ d_opacity,
                                                    float* __restrict__ d_rgb) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t i = order[r];
  if ((cull[i] & 0xFF) != 0) {
    for (int j = 0; j < 3; ++j) { d_means[3 * i + j] = 0.f; d_rgb[3 * i + j] = 0.f; }
    d_scales[2 * i] = d_scales[2 * i + 1] = 0.f;
    for (int j = 0; j < 4; ++j) d_quats[4 * i + j] = 0.f;
    d_opacity[i] = 0.f;
    return;
  }
  double G[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) G[j] = 0.0;
  const int64_t base = offs[r], cnt = count[i];
  for (int64_t j = 0; j < cnt && base + j < cap; ++j) {
    const uint32_t slot = inv[base + j];
    if (!gflag[slot]) continue;
    const float4* g = reinterpret_cast<const float4*>(gpart + (size_t)slot * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 v = g[q];
      G[4 * q] += v.x; G[4 * q + 1] += v.y; G[4 * q + 2] += v.z; G[4 * q + 3] += v.w;
    }
  }
  // The walk record was evaluated in FP64 from the FP32 inputs; its chain
  // rule is evaluated the same way.
  const double mu[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
  const double su = scales[2 * i], sv = scales[2 * i + 1];
  const double q0 = quats[4 * i], q1 = quats[4 * i + 1], q2 = quats[4 * i + 2], q3 = quats[4 * i + 3];
  const double rn = 1.0 / sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const double w = q0 * rn, x = q1 * rn, y = q2 * rn, z = q3 * rn;
  const double Rq[3][3] = {{1. - 2. * (y * y + z * z), 2. * (x * y - w * z), 2. * (x * z + w * y)},
                           {2. * (x * y + w * z), 1. - 2. * (x * x + z * z), 2. * (y * z - w * x)},
                           {2. * (x * z - w * y), 2. * (y * z + w * x), 1. - 2. * (x * x + y * y)}};
  double mc[3], ra[3], rb[3], a[3], b[3];
  for (int r = 0; r < 3; ++r) {
    const float* Rr = k.R + 3 * r;
    mc[r] = Rr[0] * mu[0] + Rr[1] * mu[1] + Rr[2] * mu[2] + (double)k.t[r];
    ra[r] = Rr[0] * Rq[0][0] + Rr[1] * Rq[1][0] + Rr[2] * Rq[2][0];
    rb[r] = Rr[0] * Rq[0][1] + Rr[1] * Rq[1][1] + Rr[2] * Rq[2][1];
    a[r] = su * ra[r];
    b[r] = sv * rb[r];
  }
  const double sgn = (cull[i] >> 8) & 1 ? -1.0 : 1.0;  // orientation chosen by the key stage
  const double fx = k.fx, fy = k.fy;
  const double iz = 1.0 / mc[2];
  const double p = a[2] * iz, q = b[2] * iz;
  const double mx = mc[0] * iz, my = mc[1] * iz;
  const double B00 = fx * (a[0] - mx * a[2]), B01 = fx * (b[0] - mx * b[2]);
  const double B10 = fy * (a[1] - my * a[2]), B11 = fy * (b[1] - my * b[2]);
  const double A00 = B00 * iz, A01 = B01 * iz, A10 = B10 * iz, A11 = B11 * iz;
  const double idA = 1.0 / (A00 * A11 - A01 * A10);
  const double Ai[2][2] = {{A11 * idA, -A01 * idA}, {-A10 * idA, A00 * idA}};
  // accumulators: d/dA^-1 (4), d/de (2), d/dxc, d/dyc, d/dz_centre, d/do, d/dc (3), d/dn_c (3)
  const double dAi[2][2] = {{G[0], G[1]}, {G[2], G[3]}};
  const double de[2] = {G[4], G[5]};
  const double dxc = G[6], dyc = G[7], dmz = G[8];
  const double gv[2] = {p, q};
  // e = g^T A^-1
  double dAt[2][2];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) dAt[r][c] = dAi[r][c] + gv[r] * de[c];
  const double dp = de[0] * Ai[0][0] + de[1] * Ai[0][1];
  const double dq = de[0] * Ai[1][0] + de[1] * Ai[1][1];
  // A^-1: dA = -A^-T dAt A^-T
  double M1[2][2], dA[2][2];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) M1[r][c] = dAt[r][0] * Ai[c][0] + dAt[r][1] * Ai[c][1];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) dA[r][c] = -(Ai[0][r] * M1[0][c] + Ai[1][r] * M1[1][c]);
  // A = diag(fx, fy) [a_xy - m a_z | b_xy - m b_z] / z,  p = a_z / z, q = b_z / z
  double d_a[3], d_b[3], d_mc[3];
  d_a[0] = fx * iz * dA[0][0];
  d_b[0] = fx * iz * dA[0][1];
  d_a[1] = fy * iz * dA[1][0];
  d_b[1] = fy * iz * dA[1][1];
  d_a[2] = -(fx * mx * dA[0][0] + fy * my * dA[1][0]) * iz + iz * dp;
  d_b[2] = -(fx * mx * dA[0][1] + fy * my * dA[1][1]) * iz + iz * dq;
  const double d_mx = -fx * iz * (a[2] * dA[0][0] + b[2] * dA[0][1]) + fx * dxc;
  const double d_my = -fy * iz * (a[2] * dA[1][0] + b[2] * dA[1][1]) + fy * dyc;
  const double d_iz = dA[0][0] * B00 + dA[0][1] * B01 + dA[1][0] * B10 + dA[1][1] * B11 + dp * a[2] + dq * b[2] +
                      d_mx * mc[0] + d_my * mc[1];
  d_mc[0] = d_mx * iz;
  d_mc[1] = d_my * iz;
  d_mc[2] = -d_iz * iz * iz + dmz;
  const double dn[3] = {sgn * G[13], sgn * G[14], sgn * G[15]};
  // back through the world -> camera rotation
  double dtu[3], dtv[3], dnn[3], dmu[3];
  for (int c = 0; c < 3; ++c) {
    const double R0 = k.R[c], R1 = k.R[3 + c], R2 = k.R[6 + c];
    dtu[c] = su * (R0 * d_a[0] + R1 * d_a[1] + R2 * d_a[2]);
    dtv[c] = sv * (R0 * d_b[0] + R1 * d_b[1] + R2 * d_b[2]);
    dnn[c] = R0 * dn[0] + R1 * dn[1] + R2 * dn[2];
    dmu[c] = R0 * d_mc[0] + R1 * d_mc[1] + R2 * d_mc[2];
  }
  const double dsu = d_a[0] * ra[0] + d_a[1] * ra[1] + d_a[2] * ra[2];
  const double dsv = d_b[0] * rb[0] + d_b[1] * rb[1] + d_b[2] * rb[2];
  // Rq columns are t_u, t_v, n;  Gm[r][c] = dL/dRq[r][c]
  const double Gm[3][3] = {{dtu[0], dtv[0], dnn[0]}, {dtu[1], dtv[1], dnn[1]}, {dtu[2], dtv[2], dnn[2]}};
  const double dw = 2. * (-z * Gm[0][1] + y * Gm[0][2] + z * Gm[1][0] - x * Gm[1][2] - y * Gm[2][0] + x * Gm[2][1]);
  const double dx = 2. * (y * Gm[0][1] + z * Gm[0][2] + y * Gm[1][0] - 2. * x * Gm[1][1] - w * Gm[1][2] +
                          z * Gm[2][0] + w * Gm[2][1] - 2. * x * Gm[2][2]);
  const double dy = 2. * (-2. * y * Gm[0][0] + x * Gm[0][1] + w * Gm[0][2] + x * Gm[1][0] + z * Gm[1][2] -
                          w * Gm[2][0] + z * Gm[2][1] - 2. * y * Gm[2][2]);
  const double dz = 2. * (-2. * z * Gm[0][0] - w * Gm[0][1] + x * Gm[0][2] + w * Gm[1][0] - 2. * z * Gm[1][1] +
                          y * Gm[1][2] + x * Gm[2][0] + y * Gm[2][1]);
  // unit quaternion: project out the radial component
  const double dot = w * dw + x * dx + y * dy + z * dz;
  d_quats[4 * i + 0] = (float)((dw - w * dot) * rn);
  d_quats[4 * i + 1] = (float)((dx - x * dot) * rn);
  d_quats[4 * i + 2] = (float)((dy - y * dot) * rn);
  d_quats[4 * i + 3] = (float)((dz - z * dot) * rn);
  for (int j = 0; j < 3; ++j) d_means[3 * i + j] = (float)dmu[j];
  d_scales[2 * i] = (float)dsu;
  d_scales[2 * i + 1] = (float)dsv;
  d_opacity[i] = (float)G[9];
  d_rgb[3 * i] = (float)G[10];
  d_rgb[3 * i + 1] = (float)G[11];
  d_rgb[3 * i + 2] = (float)G[12];
}

// Lane group per surfel (in depth order): dL/df = sum of its pairs' rows.
__global__ __launch_bounds__(256) void k_reduce_feat(int64_t n, const uint32_t* __restrict__ order,
                                                     const uint32_t* __restrict__ count,
                                                     const uint32_t* __restrict__ offs,
                                                     const uint32_t* __restrict__ inv, int64_t cap,
                                                     const float* __restrict__ fpart,
                                                     const uint8_t* __restrict__ fflag, int C,
                                                     float* __restrict__ dfeat) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lpp = C / 4;
  const int lpp2 = lpp >= 64 ? 64 : pow2_ge(lpp);
  const int spw = 64 / lpp2;
  const int sub = lane / lpp2, cl = lane % lpp2;
  const int64_t r = ((int64_t)blockIdx.x * 4 + wave) * spw + sub;
  if (r >= n) return;
  const uint32_t i = order[r];
  const int64_t base = offs[r], cnt = count[i];
  for (int cg = cl; cg < lpp; cg += lpp2) {
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t j = 0; j < cnt && base + j < cap; ++j) {
      const uint32_t slot = inv[base + j];
      if (!fflag[slot]) continue;
      const float4 v = *reinterpret_cast<const float4*>(fpart + (size_t)slot * C + cg * 4);
      acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    }
    *reinterpret_cast<float4*>(dfeat + (size_t)i * C + cg * 4) = acc;
  }
}

// ------------------------------------------------------------- host wrappers
template <typename FT>
static void backward_typed(const SurfelArgs& s, const CamArgs& c, int blend, const Layout& L, const ImageGradArgs& g,
                           const GradArgs& gr, char* ws, hipStream_t st, const ProfHook& prof) {
  const WalkRec* rec = (const WalkRec*)(ws + L.rec);
  const uint32_t* pid = (const uint32_t*)(ws + L.pid);
  const uint2* ranges = (const uint2*)(ws + L.ranges);
  float* gpart = (float*)(ws + L.gpart);
  float* fpart = (float*)(ws + L.fpart);
  uint8_t* gflag = (uint8_t*)(ws + L.gflag);
  uint8_t* fflag = (uint8_t*)(ws + L.fflag);
  const dim3 grid(xcd_grid(L.tiles));
  const bool want_f = g.feat != nullptr && s.c > 0;
  if (blend == kTopK) {
    prof.begin(kStageBwdFeature, st);
    if (want_f) {
      const size_t shm = (size_t)(2 * kWinWords + kSlotChunk * 8 + kSlotChunk + 1 + kTilePix * L.k) * 4;
      hipLaunchKernelGGL((k_feat_bwd_topk<FT>), grid, dim3(256), shm, st, pid, ranges,
                         (const int32_t*)(ws + L.selpos), (const float*)(ws + L.selw), (const FT*)s.feat, g.feat, s.c,
                         L.k, c.W, c.H, (int)L.ntx, (int)L.tiles, (float*)(ws + L.seldot), fpart, fflag);
    } else {
      launch_fill_u32(ws + L.seldot, 0u, L.spix * (int64_t)L.k, st);
    }
    prof.end(kStageBwdFeature, st);
    prof.begin(kStageBwdWalk, st);
    hipLaunchKernelGGL((k_walk_bwd<kTopK, FT>), grid, dim3(256), 0, st, rec, pid, ranges, c.W, c.H, (int)L.ntx,
                       (int)L.tiles, L.k, (const uint32_t*)(ws + L.nlast), (const float*)(ws + L.tfinal),
                       (const int32_t*)(ws + L.selpos), (const float*)(ws + L.seldot), g.rgb, g.depth, g.normal,
                       g.alpha, g.feat, (const FT*)s.feat, s.c, gpart, gflag, fpart, fflag);
    prof.end(kStageBwdWalk, st);
  } else {
    prof.begin(kStageBwdWalk, st);
    hipLaunchKernelGGL((k_walk_bwd<kFull, FT>), grid, dim3(256), 0, st, rec, pid, ranges, c.W, c.H, (int)L.ntx,
                       (int)L.tiles, L.k, (const uint32_t*)(ws + L.nlast), (const float*)(ws + L.tfinal),
                       (const int32_t*)(ws + L.selpos), (const float*)(ws + L.seldot), g.rgb, g.depth, g.normal,
                       g.alpha, want_f ? g.feat : nullptr, (const FT*)s.feat, s.c, gpart, gflag, fpart, fflag);
    prof.end(kStageBwdWalk, st);
  }
  CamB cb;
  for (int i = 0; i < 9; ++i) cb.R[i] = c.R[i];
  for (int i = 0; i < 3; ++i) cb.t[i] = c.t[i];
  cb.fx = c.fx; cb.fy = c.fy; cb.cx = c.cx; cb.cy = c.cy;
  prof.begin(kStageBwdPreprocess, st);
  const uint32_t* order = (const uint32_t*)(ws + L.id0);
  const uint32_t* count = (const uint32_t*)(ws + L.count);
  const uint32_t* offs = (const uint32_t*)(ws + L.offs);
  const uint32_t* inv = (const uint32_t*)(ws + L.inv);
  if (s.n > 0) {
    hipLaunchKernelGGL(k_reduce_geo, dim3((unsigned)cdiv(s.n, 256)), dim3(256), 0, st, s.n, order, count, offs, inv,
                       L.cap, (const float*)gpart, (const uint8_t*)gflag, s.means, s.scales, s.quats,
                       (const int32_t*)(ws + L.cull), cb, gr.means, gr.scales, gr.quats, gr.opacity, gr.rgb);
    if (s.c > 0 && gr.feat) {
      const int lpp = s.c / 4;
      int lpp2 = 1;
      while (lpp2 < lpp && lpp2 < 64) lpp2 <<= 1;
      const int per_block = 4 * (64 / lpp2);
      hipLaunchKernelGGL(k_reduce_feat, dim3((unsigned)cdiv(s.n, per_block)), dim3(256), 0, st, s.n, order, count,
                         offs, inv, L.cap, (const float*)fpart, (const uint8_t*)fflag, s.c, gr.feat);
    }
  }
  prof.end(kStageBwdPreprocess, st);
}

void launch_backward(const SurfelArgs& s, const CamArgs& c, int blend, const Layout& L, const ImageGradArgs& g,
                     const GradArgs& grads, char* ws, hipStream_t st, const ProfHook& prof) {
  prof.begin(kStageFill, st);
  launch_fill_u32(ws + L.gflag, 0u, cdiv(std::max<int64_t>(L.cap, 1), 4), st);
  launch_fill_u32(ws + L.fflag, 0u, cdiv(std::max<int64_t>(L.cap, 1), 4), st);
  prof.end(kStageFill, st);
  if (s.dtype == kF32) backward_typed<float>(s, c, blend, L, g, grads, ws, st, prof);
  else if (s.dtype == kF16) backward_typed<__half>(s, c, blend, L, g, grads, ws, st, prof);
  else backward_typed<uint16_t>(s, c, blend, L, g, grads, ws, st, prof);
}

}  // namespace psm
