// Backward of the renderer: gradients of L = <upstream, outputs> with respect
// to every surfel parameter.  The selection (eq. (18)), the contributor set,
// the stop point and the alpha clamp are held fixed.
//
// k_feat_bwd_topk: per tile, for every (pixel, selected surfel): the dot
//   product of the pixel's feature gradient with the surfel's feature row
//   (needed by the alpha adjoint), and dL/df accumulated first in LDS per
//   distinct selected surfel of the tile, then with one global atomic per
//   (surfel, channel).
// k_walk_bwd: per tile, back to front from each pixel's last contributor,
//   recovering T_i = T_{i+1} / (1 - alpha_i).  Per surfel the per-pixel
//   terms are reduced over the wave, then over the 4 waves through LDS, and
//   added to 16 per-surfel accumulators with global atomics.  In dense-blend
//   mode each batch also computes the feature dot products (batch x C x
//   pixels) and the feature gradients (pixels x batch x C) tile-wide.
// k_preprocess_bwd: chain rule from the accumulators to mu, s, q, o, rgb.
#include "common.h"
#include "internal.h"

namespace psm {

constexpr int kBB = 32;          // surfels per backward batch
constexpr int kNV = 17;          // per-pixel values reduced per surfel
constexpr int kWinWords = 1024;  // selected-position window: 32768 positions

// ------------------------------------------------------------ Top-K feature
template <typename FT>
__global__ __launch_bounds__(256) void k_feat_bwd_topk(
    const uint32_t* __restrict__ pid, const uint2* __restrict__ ranges, const int32_t* __restrict__ selpos,
    const float* __restrict__ selw, const FT* __restrict__ feat, const float* __restrict__ gfeat, int C, int K,
    int W, int H, int ntx, int tiles, int sch, float* __restrict__ seldot, float* __restrict__ dfeat) {
  extern __shared__ char smem[];
  uint32_t* s_bits = reinterpret_cast<uint32_t*>(smem);
  uint32_t* s_pref = s_bits + kWinWords;
  uint32_t* s_sid = s_pref + kWinWords;            // slot -> surfel id (256*K)
  float* s_acc = reinterpret_cast<float*>(s_sid + kTilePix * K);  // [sch][C]
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
          float f[V], g[V];
          load_vec<FT>(feat + (size_t)id * C + cg * V, f);
#pragma unroll
          for (int v = 0; v < V; v += 4) {
            const float4 x = *reinterpret_cast<const float4*>(grow + cg * V + v);
            g[v] = x.x; g[v + 1] = x.y; g[v + 2] = x.z; g[v + 3] = x.w;
          }
#pragma unroll
          for (int v = 0; v < V; ++v) part = fmaf(g[v], f[v], part);
        }
      }
      for (int o = lpp2 >> 1; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
      if (cl == 0 && p < kTilePix) seldot[tbase + (size_t)q * kTilePix + p] = pos >= 0 ? part : 0.0f;
    }
  }

  // --- dL/df: distinct selected positions of the tile -> LDS slots
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
    // exclusive scan of the popcounts (4 words per thread)
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
    for (int q = 0; q < K; ++q) {
      const int pos = selpos[tbase + (size_t)q * kTilePix + tid] - w0;
      if (pos >= 0 && pos < kWinWords * 32) {
        const uint32_t wd = s_bits[pos >> 5];
        const int slot = (int)(s_pref[pos >> 5] + __popc(wd & ((1u << (pos & 31)) - 1u)));
        s_sid[slot] = pid[start + w0 + pos];
      }
    }
    for (int c0 = 0; c0 < U; c0 += sch) {
      for (int i = tid; i < sch * C; i += 256) s_acc[i] = 0.0f;
      __syncthreads();
      for (int p0 = 0; p0 < 64; p0 += ppw) {
        const int p = wave * 64 + p0 + sub;
        const int px = tx * kTile + (p & 15), py = ty * kTile + (p >> 4);
        if (px >= W || py >= H) continue;
        const float* grow = gfeat + ((int64_t)py * W + px) * C;
        for (int q = 0; q < K; ++q) {
          const size_t o = tbase + (size_t)q * kTilePix + p;
          const int pos = selpos[o] - w0;
          if (pos < 0 || pos >= kWinWords * 32) continue;
          const int slot = (int)(s_pref[pos >> 5] + __popc(s_bits[pos >> 5] & ((1u << (pos & 31)) - 1u))) - c0;
          if (slot < 0 || slot >= sch) continue;
          const float w = selw[o];
          for (int cg = cl; cg < lpp; cg += lpp2) {
#pragma unroll
            for (int v = 0; v < V; v += 4) {
              const float4 x = *reinterpret_cast<const float4*>(grow + cg * V + v);
              float* a = s_acc + (size_t)slot * C + cg * V + v;
              atomicAdd(a + 0, w * x.x);
              atomicAdd(a + 1, w * x.y);
              atomicAdd(a + 2, w * x.z);
              atomicAdd(a + 3, w * x.w);
            }
          }
        }
      }
      __syncthreads();
      const int ns = min(sch, U - c0);
      for (int i = tid; i < ns * C; i += 256) {
        const float v = s_acc[i];
        if (v != 0.0f) atomicAdd(dfeat + (size_t)s_sid[c0 + i / C] * C + (i % C), v);
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
    const float* __restrict__ g_feat, const FT* __restrict__ feat, int C, float* __restrict__ dfeat,
    float* __restrict__ gacc) {
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
#pragma unroll
        for (int i = 0; i < kNV; ++i) v[i] = wave_sum(v[i]);
        if (lane == 0) {
#pragma unroll
          for (int i = 0; i < kNV; ++i) s_part[wave][k][i] = v[i];
        }
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
        float* g = gacc + (size_t)id * 16;
        // u' = A^-1 d, w' = 1 - e.d with d = pixel - centre
        atomicAdd(g + 0, t[0]);
        atomicAdd(g + 1, t[1]);
        atomicAdd(g + 2, t[3]);
        atomicAdd(g + 3, t[4]);
        atomicAdd(g + 4, -t[6]);
        atomicAdd(g + 5, -t[7]);
        // d depends on the centre with slope -1
        atomicAdd(g + 6, -(a00 * t[2] + a10 * t[5] - e0 * t[8]));
        atomicAdd(g + 7, -(a01 * t[2] + a11 * t[5] - e1 * t[8]));
        atomicAdd(g + 8, t[9]);
        atomicAdd(g + 9, t[10]);
        atomicAdd(g + 10, t[11]);
        atomicAdd(g + 11, t[12]);
        atomicAdd(g + 12, t[13]);
        atomicAdd(g + 13, t[14]);
        atomicAdd(g + 14, t[15]);
        atomicAdd(g + 15, t[16]);
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
              if (k < nb && acc[j] != 0.0f) atomicAdd(dfeat + (size_t)s_id[k] * C + c, acc[j]);
            }
          }
        }
      }
    }
  }
}

// ------------------------------------------------------- preprocess backward
struct CamB {
  float R[9], t[3], fx, fy, cx, cy;
};

__global__ __launch_bounds__(256) void k_preprocess_bwd(int64_t n, const float* __restrict__ means,
                                                        const float* __restrict__ scales,
                                                        const float* __restrict__ quats,
                                                        const int32_t* __restrict__ cull, CamB k,
                                                        const float* __restrict__ gacc, float* __restrict__ d_means,
                                                        float* __restrict__ d_scales, float* __restrict__ d_quats,
                                                        float* __restrict__ d_opacity, float* __restrict__ d_rgb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if ((cull[i] & 0xFF) != 0) {
    for (int j = 0; j < 3; ++j) { d_means[3 * i + j] = 0.f; d_rgb[3 * i + j] = 0.f; }
    d_scales[2 * i] = d_scales[2 * i + 1] = 0.f;
    for (int j = 0; j < 4; ++j) d_quats[4 * i + j] = 0.f;
    d_opacity[i] = 0.f;
    return;
  }
  // The walk record was evaluated in FP64 from the FP32 inputs; its chain
  // rule is evaluated the same way.
  double G[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) G[j] = gacc[16 * i + j];
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

// ------------------------------------------------------------- host wrappers
template <typename FT>
static void backward_typed(const SurfelArgs& s, const CamArgs& c, int blend, const Layout& L, const ImageGradArgs& g,
                           const GradArgs& gr, char* ws, hipStream_t st, const ProfHook& prof) {
  const WalkRec* rec = (const WalkRec*)(ws + L.rec);
  const uint32_t* pid = (const uint32_t*)(ws + L.pid0);
  const uint2* ranges = (const uint2*)(ws + L.ranges);
  float* gacc = (float*)(ws + L.gacc);
  const dim3 grid(xcd_grid(L.tiles));
  if (blend == kTopK) {
    prof.begin(kStageBwdFeature, st);
    if (g.feat && s.c > 0) {
      const size_t fixed = (size_t)(2 * kWinWords + kTilePix * L.k) * 4;
      const size_t budget = 60 * 1024;  // dynamic part; about 1 KB of static LDS comes on top
      int sch = (int)((budget - fixed) / ((size_t)s.c * 4));
      sch = std::max(1, std::min(sch, kTilePix * L.k));
      const size_t shm = fixed + (size_t)sch * s.c * 4;
      hipLaunchKernelGGL((k_feat_bwd_topk<FT>), grid, dim3(256), shm, st, pid, ranges,
                         (const int32_t*)(ws + L.selpos), (const float*)(ws + L.selw), (const FT*)s.feat, g.feat, s.c,
                         L.k, c.W, c.H, (int)L.ntx, (int)L.tiles, sch, (float*)(ws + L.seldot), gr.feat);
    } else {
      launch_fill_u32(ws + L.seldot, 0u, L.spix * (int64_t)L.k, st);
    }
    prof.end(kStageBwdFeature, st);
    prof.begin(kStageBwdWalk, st);
    hipLaunchKernelGGL((k_walk_bwd<kTopK, FT>), grid, dim3(256), 0, st, rec, pid, ranges, c.W, c.H, (int)L.ntx,
                       (int)L.tiles, L.k, (const uint32_t*)(ws + L.nlast), (const float*)(ws + L.tfinal),
                       (const int32_t*)(ws + L.selpos), (const float*)(ws + L.seldot), g.rgb, g.depth, g.normal,
                       g.alpha, g.feat, (const FT*)s.feat, s.c, gr.feat, gacc);
    prof.end(kStageBwdWalk, st);
  } else {
    prof.begin(kStageBwdWalk, st);
    hipLaunchKernelGGL((k_walk_bwd<kFull, FT>), grid, dim3(256), 0, st, rec, pid, ranges, c.W, c.H, (int)L.ntx,
                       (int)L.tiles, L.k, (const uint32_t*)(ws + L.nlast), (const float*)(ws + L.tfinal),
                       (const int32_t*)(ws + L.selpos), (const float*)(ws + L.seldot), g.rgb, g.depth, g.normal,
                       g.alpha, (s.c > 0 ? g.feat : nullptr), (const FT*)s.feat, s.c, gr.feat, gacc);
    prof.end(kStageBwdWalk, st);
  }
  CamB cb;
  for (int i = 0; i < 9; ++i) cb.R[i] = c.R[i];
  for (int i = 0; i < 3; ++i) cb.t[i] = c.t[i];
  cb.fx = c.fx; cb.fy = c.fy; cb.cx = c.cx; cb.cy = c.cy;
  prof.begin(kStageBwdPreprocess, st);
  if (s.n > 0)
    hipLaunchKernelGGL(k_preprocess_bwd, dim3((unsigned)cdiv(s.n, 256)), dim3(256), 0, st, s.n, s.means, s.scales,
                       s.quats, (const int32_t*)(ws + L.cull), cb, (const float*)gacc, gr.means, gr.scales, gr.quats,
                       gr.opacity, gr.rgb);
  prof.end(kStageBwdPreprocess, st);
}

void launch_backward(const SurfelArgs& s, const CamArgs& c, int blend, const Layout& L, const ImageGradArgs& g,
                     const GradArgs& grads, char* ws, hipStream_t st, const ProfHook& prof) {
  prof.begin(kStageFill, st);
  launch_fill_u32(ws + L.gacc, 0u, L.n * 16, st);
  if (grads.feat && s.c > 0) launch_fill_u32(grads.feat, 0u, L.n * (int64_t)s.c, st);
  prof.end(kStageFill, st);
  if (s.dtype == kF32) backward_typed<float>(s, c, blend, L, g, grads, ws, st, prof);
  else if (s.dtype == kF16) backward_typed<__half>(s, c, blend, L, g, grads, ws, st, prof);
  else backward_typed<uint16_t>(s, c, blend, L, g, grads, ws, st, prof);
}

}  // namespace psm
