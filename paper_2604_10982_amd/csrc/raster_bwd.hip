// Backward of the renderer: gradients of L = <upstream, outputs> with respect
// to every surfel parameter.  The selection (eq. (18)), the contributor set,
// the stop point and the alpha clamp are held fixed.
//
// Deterministic and free of floating-point atomics: every (tile, surfel) pair
// owns a slot for its partial sums at the index where the key stage emitted
// it, so a surfel's pairs are contiguous and a per-surfel pass adds them in
// a fixed order (emission order).
//
// k_feat_bwd_topk: per tile, for every (pixel, selected surfel): the dot
//   product of the pixel's feature gradient with the surfel's feature row
//   (needed by the alpha adjoint); and, per distinct selected surfel of the
//   tile, the row sum_p w_p g_F(p) over the pixels that selected it, in pixel
//   order.
// k_walk_bwd: per tile, back to front from each pixel's last contributor,
//   recovering T_i = T_{i+1} / (1 - alpha_i).  Per surfel the per-pixel terms
//   are reduced over the wave, then over the 4 waves through LDS, and written
//   as the pair's 16 partial sums.  In dense-blend mode each batch also forms
//   the feature dot products and feature-gradient rows tile-wide.
// k_reduce_geo / k_reduce_feat: per surfel, sum of its pairs' partials, then
//   the chain rule to mu, s, q (FP64, as the forward's walk record).
#include <type_traits>

#include "common.h"
#include "internal.h"
#include "select.h"

namespace psm {

constexpr int kBB = 32;          // surfels per backward batch
// per-pixel values reduced per surfel: 17, and 2 more (the low-pass filter
// term's centre gradient) with the filter
constexpr int nv_of(bool lp) { return lp ? 19 : 17; }

// ------------------------------------------------------------ Top-K feature
// Per tile, the distinct selected surfels of the tile (a few dozen: each is
// chosen by about a hundred of the 256 pixels for K = 16) get slots in list
// order, 64 per chunk.  With G = the pixels' feature gradients (256 x C),
// F = the slots' feature rows and W = the selection weights (pixel x slot,
// zero where the pixel did not select the slot), the adjoint needs
//   dots = G F^T  at the selected (pixel, slot) entries   (alpha adjoint)
//   rows = W^T G                                           (feature gradient)
// and the weight matrix of a tile is dense enough (about half its entries)
// that both run as dense FP32 matrix-core products.  Wave w owns pixels
// [64 w, 64 w + 64): its dots tiles, and its share of the rows (a sum over
// its pixels), added across the 4 waves in wave order.  The number of
// 16-slot blocks of a chunk is a compile-time parameter of the product
// loops (one instantiation per count), so they carry no branches.  Per pass
// of GC channels G and F are staged in LDS; every layout below keeps the
// operand reads free of bank conflicts (see the strides).  Every sum has a
// fixed order: results do not depend on the pass width or the tile
// schedule.
constexpr int kFbSlots = 64;   // slots per chunk: 4 blocks of 16
constexpr int kQStride = 72;   // bytes per pixel row of the selection map

// Selection map: the byte of (pixel p, slot s) holds the index q of the
// pixel's selection of s (0xFF = none); the 4 slots s = li + 16 sb share one
// dword, so a lane reads its 4 slot blocks at once.
__device__ __forceinline__ int qmap_off(int p, int s) { return p * kQStride + (s & 15) * 4 + (s >> 4); }

template <typename FT, int KMAX, int GC, bool PERSIST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KMAX <= 16 ? 2 : 1))) void k_feat_bwd_topk(
    const uint32_t* __restrict__ pid, const uint32_t* __restrict__ eid, const uint2* __restrict__ ranges,
    const int32_t* __restrict__ selpos, const float* __restrict__ selw, const FeatSrc<FT> feat,
    const float* __restrict__ gfeat, int C, int K, CamTable ct, TileQueue tq, float* __restrict__ seldot,
    float* __restrict__ fpart, uint8_t* __restrict__ fflag, int renorm) {
  static_assert(GC % 16 == 0, "pass width is a multiple of the MFMA tile");
  // Row stride of the staged G and F: = 2 mod 4, so a 16-row x 2-column read
  // (lanes 0-31 of an operand fetch) touches 32 distinct banks, and 8 rows
  // apart is 16 banks apart.
  constexpr int GS = GC + 2;
  constexpr int NCB = GC / 16;              // channel blocks per pass
  constexpr int FPT = kFbSlots * GC / 256;  // staged F values per thread
  __shared__ SelShared S;
  __shared__ __align__(16) float s_G[kTilePix * GS];  // G rows of the pass; then the waves' partial rows
  __shared__ float s_F[kFbSlots * GS];
  __shared__ __align__(16) uint8_t s_q[kTilePix * kQStride];
  __shared__ uint32_t s_fe[kFbSlots];  // emitted pair index per slot
  extern __shared__ float s_w[];       // selection weights, replaced by dots
  __shared__ int s_item;

  for_tiles<PERSIST>(tq, &s_item, [&](const int tile) {
  const TileLoc tl = locate(ct, tile);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int px = tl.tx * ct.tw + tile_lx(ct, tid), py = tl.ty * ct.th + tile_ly(ct, tid);
  const bool inside = px < tl.W && py < tl.H;
  const uint32_t start = ranges[tile].x;
  const size_t tbase = (size_t)tile * K * kTilePix;
  const float* grow = gfeat + (tl.pix0 + (int64_t)py * tl.W + px) * C;
  const int p0 = wave * 64;  // first pixel of this wave

  // the selection positions are re-read where needed (an L2 hit) rather
  // than held in registers through the products
  auto load_pos = [&](int (&pos)[KMAX]) {
#pragma unroll
    for (int q = 0; q < KMAX; ++q) pos[q] = q < K ? selpos[tbase + (size_t)q * kTilePix + tid] : -1;
  };
  // list positions are below the tile's list length, which bounds the
  // windows (no block-wide maximum of the selections needed)
  const int lastpos = (int)(ranges[tile].y - start) - 1;
  int Uw0 = 0;
  float rw = 1.0f;  // renormalised Top-K: 1 / (sum of the pixel's selected weights)
  {
    int pos[KMAX];
    load_pos(pos);
    float wsum = 0.0f;
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {  // unselected entries keep weight 0 and report dot 0
      const float wq = q < K && pos[q] >= 0 ? selw[tbase + (size_t)q * kTilePix + tid] : 0.0f;
      if (q < K) s_w[wsel_off(q, tid)] = wq;
      wsum += wq;
    }
    if (renorm) rw = wsum > 0.0f ? 1.0f / wsum : 0.0f;
    if (lastpos >= 0) Uw0 = build_window(S, pos, K, 0, window_words(lastpos, 0));
  }

  for (int w0 = 0; w0 <= lastpos; w0 += kWinPos) {
    const int nw = window_words(lastpos, w0);
    int Uw = Uw0;
    if (w0 > 0) {
      int pos[KMAX];
      load_pos(pos);
      Uw = build_window(S, pos, K, w0, nw);
    }
    for (int c0 = 0; c0 < Uw; c0 += kFbSlots) {
      const int ns = min(kFbSlots, Uw - c0), nb = (ns + 15) >> 4;
      for (int i = tid; i < kTilePix * kQStride / 16; i += 256)
        reinterpret_cast<uint4*>(s_q)[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
      __syncthreads();
      {
        int pos[KMAX];
        load_pos(pos);
#pragma unroll
        for (int q = 0; q < KMAX; ++q) {
          const int sl = q < K ? slot_of(S, pos[q], w0, nw) - c0 : -1;
          if (sl >= 0 && sl < ns) {
            s_q[qmap_off(tid, sl)] = (uint8_t)q;
            S.lpos[sl] = (uint32_t)pos[q];  // same value from every selecting pixel
          }
        }
      }
      __syncthreads();
      if (tid < ns) {
        const uint32_t j = start + S.lpos[tid];
        s_fe[tid] = eid[j];
        S.fid[tid] = (uint32_t)(pid[j] - tl.v0);
      }
      __syncthreads();

      auto chunk = [&](auto nb_c) {
        constexpr int NB = decltype(nb_c)::value;
        f4v dacc[4][NB];
#pragma unroll
        for (int pb = 0; pb < 4; ++pb)
#pragma unroll
          for (int sb = 0; sb < NB; ++sb) dacc[pb][sb] = f4v{0.f, 0.f, 0.f, 0.f};
        // rows A operand for the whole chunk: W[p][s] at lane (s, p) of step
        // ks, whose 4 pixels are base + 8 k (k = lane group)
        float wa[NB][16];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
          const int p = p0 + (ks & 7) + 32 * (ks >> 3) + 8 * lk;
          const uint32_t qd = *reinterpret_cast<const uint32_t*>(s_q + p * kQStride + 4 * li);
#pragma unroll
          for (int sb = 0; sb < NB; ++sb) {
            const int q = (int)((qd >> (8 * sb)) & 0xFFu);
            const float x = s_w[wsel_off(min(q, K - 1), p)];  // always in range
            wa[sb][ks] = q != 0xFF ? x : 0.0f;
          }
        }
        float gv[GC], fv[FPT];
        auto load_pass = [&](int cc) {
#pragma unroll
          for (int j = 0; j < GC / 4; ++j) {
            const int c = cc + 4 * j;
            const float4 g =
                inside && c < C ? *reinterpret_cast<const float4*>(grow + c) : make_float4(0.f, 0.f, 0.f, 0.f);
            // renormalised Top-K: the rows and dots see g / W (rw = 1 otherwise)
            gv[4 * j] = g.x * rw;
            gv[4 * j + 1] = g.y * rw;
            gv[4 * j + 2] = g.z * rw;
            gv[4 * j + 3] = g.w * rw;
          }
#pragma unroll
          for (int u = 0; u < FPT; ++u) {
            const int item = tid + 256 * u, sidx = item / GC, c = cc + item % GC;
            fv[u] = sidx < ns && c < C ? feat.load1(S.fid[sidx], c) : 0.0f;
          }
        };
        load_pass(0);
        for (int cc = 0; cc < C; cc += GC) {
#pragma unroll
          for (int c = 0; c < GC; c += 2)
            *reinterpret_cast<float2*>(s_G + tid * GS + c) = make_float2(gv[c], gv[c + 1]);
#pragma unroll
          for (int u = 0; u < FPT; ++u) {
            const int item = tid + 256 * u;
            s_F[(item / GC) * GS + item % GC] = fv[u];
          }
          __syncthreads();
          if (cc + GC < C) load_pass(cc + GC);
          // dots: D[p][s] += G[p][c] F[s][c], 4 channels per step
#pragma unroll 2
          for (int ks = 0; ks < GC / 4; ++ks) {
            float fb[NB], ga[4];
#pragma unroll
            for (int sb = 0; sb < NB; ++sb) fb[sb] = s_F[(16 * sb + li) * GS + 4 * ks + lk];
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) ga[pb] = s_G[(p0 + 16 * pb + li) * GS + 4 * ks + lk];
#pragma unroll
            for (int pb = 0; pb < 4; ++pb)
#pragma unroll
              for (int sb = 0; sb < NB; ++sb) dacc[pb][sb] = mfma_16x16x4(ga[pb], fb[sb], dacc[pb][sb]);
          }
          // rows: R[s][c] += W[p][s] G[p][c] over this wave's pixels; step ks
          // takes the 4 pixels base + 8 k (k = lane group)
          f4v racc[NB][NCB];
#pragma unroll
          for (int sb = 0; sb < NB; ++sb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) racc[sb][cb] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int ks = 0; ks < 16; ++ks) {
            const int p = p0 + (ks & 7) + 32 * (ks >> 3) + 8 * lk;
            float gb[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) gb[cb] = s_G[p * GS + 16 * cb + li];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
              for (int sb = 0; sb < NB; ++sb) racc[sb][cb] = mfma_16x16x4(wa[sb][ks], gb[cb], racc[sb][cb]);
          }
          __syncthreads();  // every wave is done with the staged G
          // partial row of slot s of wave w at row 64 w + perm(s), perm
          // swapping bits 2 and 3 of s (lanes 0-31 then write 16 banks apart)
#pragma unroll
          for (int sb = 0; sb < NB; ++sb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                s_G[(p0 + 16 * sb + 8 * (lk & 1) + 4 * (lk >> 1) + r) * GS + 16 * cb + li] = racc[sb][cb][r];
          __syncthreads();
          for (int item = tid; item < ns * GC; item += 256) {
            const int sidx = item / GC, c = item % GC;
            const int row = (sidx & ~12) | ((sidx & 4) << 1) | ((sidx & 8) >> 1);
            const float* r = s_G + row * GS + c;
            const float v = ((r[0] + r[64 * GS]) + r[128 * GS]) + r[192 * GS];
            if (cc + c < C) fpart[(size_t)s_fe[sidx] * C + cc + c] = v;
          }
          __syncthreads();
        }
        // dots of the selected entries replace their (already consumed) weights
#pragma unroll
        for (int pb = 0; pb < 4; ++pb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int p = p0 + 16 * pb + 4 * lk + r;
            const uint32_t qd = *reinterpret_cast<const uint32_t*>(s_q + p * kQStride + 4 * li);
#pragma unroll
            for (int sb = 0; sb < NB; ++sb) {
              const int q = (int)((qd >> (8 * sb)) & 0xFFu);
              if (q != 0xFF) s_w[wsel_off(q, p)] = dacc[pb][sb][r];
            }
          }
      };
      switch (nb) {
        case 1: chunk(std::integral_constant<int, 1>{}); break;
        case 2: chunk(std::integral_constant<int, 2>{}); break;
        case 3: chunk(std::integral_constant<int, 3>{}); break;
        default: chunk(std::integral_constant<int, 4>{}); break;
      }
      if (tid < ns) fflag[s_fe[tid]] = 1;
      __syncthreads();
    }
  }
  __syncthreads();
  // renormalised Top-K: d/dw_q of F = sum w f / W is g.(f_q - F) / W, i.e.
  // dot'_q - sum_j (w_j / W) dot'_j with dot' = (g / W) . f
  float cshift = 0.0f;
  if (renorm) {
#pragma unroll
    for (int q = 0; q < KMAX; ++q)
      if (q < K) {
        const float wq = selpos[tbase + (size_t)q * kTilePix + tid] >= 0 ? selw[tbase + (size_t)q * kTilePix + tid] : 0.0f;
        cshift = fmaf(wq, s_w[wsel_off(q, tid)], cshift);
      }
    cshift *= rw;
  }
#pragma unroll
  for (int q = 0; q < KMAX; ++q)
    if (q < K) seldot[tbase + (size_t)q * kTilePix + tid] = s_w[wsel_off(q, tid)] - cshift;
  __syncthreads();
  });
}

// ------------------------------------------------------------- walk backward
// DM (dense mode only): the batch's feature contractions on the matrix cores
// (true) or in vector FMAs (false); a launch choice, whichever is faster for
// the workload (the autotuner times both).
template <int MODE, typename FT, bool PERSIST, bool LP, bool DM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == kTopK ? 4 : 1))) void k_walk_bwd(
    const WalkRec* __restrict__ rec, const float4* __restrict__ ext, const uint32_t* __restrict__ pid, const uint32_t* __restrict__ eid,
    const uint2* __restrict__ ranges, CamTable ct, TileQueue tq, int K, const uint32_t* __restrict__ nlast,
    const float* __restrict__ tfinal,
    const int32_t* __restrict__ selpos, const float* __restrict__ seldot, const float* __restrict__ g_rgb,
    const float* __restrict__ g_depth, const float* __restrict__ g_normal, const float* __restrict__ g_alpha,
    const float* __restrict__ g_feat, const FeatSrc<FT> feat, int C, float* __restrict__ gpart,
    uint8_t* __restrict__ gflag, float* __restrict__ fpart, uint8_t* __restrict__ fflag) {
#pragma clang fp contract(fast)
  // (products and sums written in this kernel may fuse into FMAs: its outputs
  // are gradients, which no decision depends on; the hit test, alpha and the
  // weights come from eval_pixel, written outside this scope and evaluated
  // exactly as in the forward)
  __shared__ Staged<kBB> s_r;
  __shared__ float2 s_band[kBB];  // (ecy, ey) of the batch, for band culling
  __shared__ uint32_t s_id[kBB];
  constexpr int kNV = nv_of(LP);
  __shared__ float s_part[4][kBB][kNV];
  __shared__ uint32_t s_has[4][kBB];
  __shared__ int s_lmax;
  // dense-blend mode only: each wave's dots tile (16 pixels x the batch) and
  // the batch weights (rows padded to 260 floats: the matrix-core operand
  // reads of 16 entries x 4 pixels fall in distinct banks)
  constexpr int kPhS = kBB + 4, kOmS = kTilePix + 4;
  __shared__ float s_ph[MODE == kFull && DM ? 4 : 1][16 * kPhS];
  __shared__ float s_fc[MODE == kFull && !DM ? kBB : 1][64];  // vector form: the batch's feature chunk
  __shared__ __align__(16) float s_om[MODE == kFull ? kBB : 1][kOmS];
  // Top-K mode: every pixel's selected list positions ([K][256]), read back
  // to front by the pixel's own lane; the feature dots stay in global memory,
  // each loaded when the previous one is used (16 KB of LDS instead of 32 KB
  // for K = 16 lets four blocks share a CU, with the kernel's registers held
  // to 128 for four waves per SIMD)
  extern __shared__ int s_sel[];
  __shared__ int s_item;

  for_tiles<PERSIST>(tq, &s_item, [&](const int tile) {
  const TileLoc tl = locate(ct, tile);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tx = tl.tx, ty = tl.ty, W = tl.W, H = tl.H;
  const int qx0 = tile_lx(ct, tid), qy0 = tile_ly(ct, tid), rpw = 64 >> ct.tsh;  // rows per wave
  const int px = tx * ct.tw + qx0, py = ty * ct.th + qy0;
  const bool inside = px < W && py < H;
  const float lx = (float)qx0 + 0.5f, ly = (float)qy0 + 0.5f;
  const float tx0 = (float)(tx * ct.tw), ty0 = (float)(ty * ct.th);
  const float yb0 = ty0 + (float)(rpw * wave) + 0.5f, yb1 = yb0 + (float)(rpw - 1);  // this wave's rows
  const uint32_t start = ranges[tile].x;
  const int sp = tile * kTilePix + tid;
  const int my_last = (int)nlast[sp];
  float T = tfinal[sp];
  const float Tfin = T;
  const int64_t pix = tl.pix0 + (int64_t)py * W + px;
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
  int* s_sp = s_sel;
  const float* g_sd = seldot + tbase + tid;  // this pixel's dots, read one ahead of their use
  if (MODE == kTopK) {
    for (int q = 0; q < K; ++q) {
      const int sq = selpos[tbase + (size_t)q * kTilePix + tid];
      s_sp[q * kTilePix + tid] = sq;
      if (sq >= 0) kp = q;
    }
    if (kp >= 0) {
      nextsel = s_sp[kp * kTilePix + tid];
      nextdot = g_sd[(size_t)kp * kTilePix];
    }
  }

  __syncthreads();
  if (tid == 0) s_lmax = 0;
  __syncthreads();
  atomicMax(&s_lmax, my_last);
  __syncthreads();
  const int Lmax = __builtin_amdgcn_readfirstlane(s_lmax);  // block-uniform: a scalar loop bound
  float suffix = 0.0f;
  // the wave starts each batch at its own last contributor: the entries past
  // it change nothing of its pixels (no selection lies there; in dense mode
  // their weights are zero)
  int wmax = my_last;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, __shfl_xor(wmax, o, 64));
  wmax = __builtin_amdgcn_readfirstlane(wmax);  // the same in every lane: keeps the loop bound scalar

  for (int hi = Lmax; hi > 0; hi -= kBB) {
    const int lo = max(0, hi - kBB), nb = hi - lo;
    __syncthreads();
    if (tid < nb) {
      const uint32_t id = pid[start + lo + tid];
      s_id[tid] = id;  // virtual surfel id
      s_r.put(tid, rec[id], tx0, ty0);
      const float4 x = ext[id];
      s_band[tid] = make_float2(x.y, x.w);
    }
    __syncthreads();

    // dense mode: phi[k] = g_F(p) . f_k for the batch, the product
    // PHI = G F^T on the matrix cores: wave w takes its 4 pixel blocks of 16
    // x the 2 entry blocks of 16, k = 4 channels per step (lane (li, lk)
    // loads channels 4 lk .. 4 lk + 3 of a 16-channel group as one vector,
    // component i feeding step i); the tile goes through the wave's LDS
    // region to the lanes of its pixels
    float phi[MODE == kFull ? kBB : 1];
    if constexpr (MODE == kFull && !DM) {
      // vector form: feature chunks of 64 channels staged in LDS, each pixel
      // its 32 dots (LDS reads by broadcast)
#pragma unroll
      for (int k = 0; k < kBB; ++k) phi[k] = 0.0f;
      if (g_feat) {
        const float* grow = g_feat + pix * C;
        const bool has_gf = inside;
        for (int c0 = 0; c0 < C; c0 += 64) {
          for (int e = tid; e < nb * 64; e += 256) {
            const int k = e >> 6, c = e & 63;
            s_fc[k][c] = (c0 + c < C) ? feat.load1(s_id[k] - tl.v0, c0 + c) : 0.0f;
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
    if constexpr (MODE == kFull && DM) {
#pragma unroll
      for (int k = 0; k < kBB; ++k) phi[k] = 0.0f;
      if (g_feat) {
        const int li = lane & 15, lk = lane >> 4;
        int fr[2];  // feature row of the lane's entry of each block, -1 past the batch
#pragma unroll
        for (int eb = 0; eb < 2; ++eb) {
          const int e = 16 * eb + li;
          fr[eb] = e < nb ? (int)(s_id[e] - tl.v0) : -1;
        }
        float* ph = s_ph[wave];
        for (int pb = 0; pb < 4; ++pb) {
          const int q = 64 * wave + 16 * pb + li;  // pixel of lane li
          const int qx = tx * ct.tw + tile_lx(ct, q), qy = ty * ct.th + tile_ly(ct, q);
          const float* gq = qx < W && qy < H ? g_feat + (tl.pix0 + (int64_t)qy * W + qx) * C : nullptr;
          f4v acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
          // 128 channels at a time: every operand of the segment is loaded
          // before its products, so the loads are in flight together
          for (int cs = 0; cs < C; cs += 128) {
            float4 a[8], b[2][8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int c = cs + 16 * j + 4 * lk;  // C % 4 == 0: a group of 4 is whole or absent
              a[j] = gq && c < C ? *reinterpret_cast<const float4*>(gq + c) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
              for (int eb = 0; eb < 2; ++eb)
                b[eb][j] = fr[eb] >= 0 && c < C ? feat.load4(fr[eb], c) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
#pragma unroll
              for (int eb = 0; eb < 2; ++eb) {
                acc[eb] = mfma_16x16x4(a[j].x, b[eb][j].x, acc[eb]);
                acc[eb] = mfma_16x16x4(a[j].y, b[eb][j].y, acc[eb]);
                acc[eb] = mfma_16x16x4(a[j].z, b[eb][j].z, acc[eb]);
                acc[eb] = mfma_16x16x4(a[j].w, b[eb][j].w, acc[eb]);
              }
          }
#pragma unroll
          for (int eb = 0; eb < 2; ++eb)
#pragma unroll
            for (int r = 0; r < 4; ++r) ph[(4 * lk + r) * kPhS + 16 * eb + li] = acc[eb][r];
          wave_lds_sync();
          if (lk == pb) {
#pragma unroll
            for (int k = 0; k < kBB; ++k) phi[k] = ph[li * kPhS + k];
          }
          wave_lds_sync();
        }
      }
    }

    // surfels of the batch whose footprint meets this wave's 4 rows
    const uint64_t band = __ballot(lane < nb && band_meets(s_band[lane < kBB ? lane : 0].x,
                                                           s_band[lane < kBB ? lane : 0].y, yb0, yb1));
    const int ktop = min(nb - 1, wmax - 1 - lo);
    if (lane > ktop && lane < nb) s_has[wave][lane] = 0u;  // skipped entries: nothing to add
    if constexpr (MODE == kFull)
      for (int k = max(ktop + 1, 0); k < nb; ++k) s_om[k][tid] = 0.0f;  // and zero weight
#pragma unroll 1
    for (int k = ktop; k >= 0; --k) {
      const int pos = lo + k;
      // the pixel's terms are products of these scalars, all zero where the
      // pixel does not take part
      float w = 0.0f, du1 = 0.0f, dv1 = 0.0f, dw1 = 0.0f, dzi = 0.0f, dop = 0.0f, ex = 0.0f, ey = 0.0f;
      float gcx = 0.0f, gcy = 0.0f;  // low-pass term: direct gradient of the projected centre
      bool contrib = false;
      if (pos < my_last && ((band >> k) & 1u)) {
        const LRec s = s_r.get(k);
        PixEval e;
        if (eval_pixel<LP>(s, lx, ly, e)) {
          contrib = true;
          // 1 / (1 - alpha) once for both quotients: alpha <= 0.99, so the
          // reciprocal's relative error (about 1 ulp) stays that small
          const float r1m = __builtin_amdgcn_rcpf(1.0f - e.alpha);
          const float Tb = T * r1m;
          w = e.alpha * Tb;
          const float u = e.u, vv = e.v, z = s.mz * e.iw;
          float eF = 0.0f;
          if (MODE == kTopK) {
            if (pos == nextsel) {
              eF = nextdot;
              --kp;
              nextsel = kp >= 0 ? s_sp[kp * kTilePix + tid] : -1;
              nextdot = kp >= 0 ? g_sd[(size_t)kp * kTilePix] : 0.0f;
            }
          } else {
#pragma unroll
            for (int q = 0; q < kBB; ++q)
              if (q == k) eF = phi[q];
          }
          const float ei = gC0 * s.r + gC1 * s.g + gC2 * s.b + gD * z + gN0 * s.n0 + gN1 * s.n1 + gN2 * s.n2 + eF;
          const float da = Tb * ei - (suffix - gA * Tfin) * r1m;
          suffix = fmaf(w, ei, suffix);
          T = Tb;
          dop = e.clamped ? 0.0f : da * e.G;
          const float drho = e.clamped ? 0.0f : -0.5f * da * e.alpha;
          const float dz = w * gD;
          if (LP && e.filt) {
            // rho = 2 |d|^2 with d = pixel - centre, depth = centre depth
            gcx = -4.0f * drho * e.dx;
            gcy = -4.0f * drho * e.dy;
            dzi = dz;
          } else {
            const float du = 2.0f * u * drho, dv = 2.0f * vv * drho;
            du1 = du * e.iw;
            dv1 = dv * e.iw;
            dw1 = -(du * u + dv * vv + dz * z) * e.iw;
            dzi = dz * e.iw;
            ex = e.dx;
            ey = e.dy;
          }
        }
      }
      if constexpr (MODE == kFull) s_om[k][tid] = w;
      const bool any = __any(contrib);
      if (any) {
        float v16[16] = {du1 * ex, du1 * ey, du1, dv1 * ex, dv1 * ey, dv1, dw1 * ex, dw1 * ey,
                         dw1,      dzi,      dop, w * gC0,  w * gC1,  w * gC2, w * gN0,  w * gN1};
        const float tot = wave_reduce16(v16);
        const float last = wave_sum(w * gN2);
        if ((lane & 3) == 0) s_part[wave][k][(lane >> 2) & 15] = tot;
        if (lane == 0) s_part[wave][k][16] = last;
        if constexpr (LP) {
          const float c0 = wave_sum(gcx), c1 = wave_sum(gcy);
          if (lane == 0) {
            s_part[wave][k][17] = c0;
            s_part[wave][k][18] = c1;
          }
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
        const size_t slot = eid[start + lo + k];
        float4* g = reinterpret_cast<float4*>(gpart + slot * 16);
        // u' = A^-1 d, w' = 1 - e.d with d = pixel - centre; d depends on the
        // centre with slope -1
        g[0] = make_float4(t[0], t[1], t[3], t[4]);
        float gxc = -(a00 * t[2] + a10 * t[5] - e0 * t[8]), gyc = -(a01 * t[2] + a11 * t[5] - e1 * t[8]);
        if constexpr (LP) {
          gxc += t[17];
          gyc += t[18];
        }
        g[1] = make_float4(-t[6], -t[7], gxc, gyc);
        g[2] = make_float4(t[9], t[10], t[11], t[12]);
        g[3] = make_float4(t[13], t[14], t[15], t[16]);
        gflag[slot] = 1;
      }
    }

    // dense mode: dL/df_k = sum_p w_k(p) g_F(p) for the batch, the product
    // R = W^T G on the matrix cores: units (entry block of 16, channel block
    // of 16) dealt to the waves, each a sum over the 256 pixels in 64 steps
    // of 4 (pixels 16 y + 4 u + lk of tile row y), written at the pair's
    // emission index
    if constexpr (MODE == kFull && !DM) {
      // vector form: wave w takes 8 surfels of the batch, lane = channel, the
      // 256 pixels 8 at a time (8 independent upstream loads in flight;
      // pixels outside the image have zero weight and read as zero)
      if (g_feat) {
        __syncthreads();
        constexpr int PER = kBB / 4;
        // the tile's pixels inside the image: wl columns, hl rows; pixel
        // offsets from the tile's first one are below 2^29 (W, C and the tile
        // height are bounded)
        const int wl = min(ct.tw, W - tx * ct.tw), hl = min(ct.th, H - ty * ct.th), wc = W * C;
        for (int c0 = 0; c0 < C; c0 += 64) {
          const int c = c0 + lane;
          float acc[PER];
#pragma unroll
          for (int j = 0; j < PER; ++j) acc[j] = 0.0f;
          if (c < C) {
            const float* gt = g_feat + (tl.pix0 + (int64_t)(ty * ct.th) * W + tx * ct.tw) * C + c;
            for (int p0 = 0; p0 < kTilePix; p0 += 8) {
              float g[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                const int p = p0 + u, lx = tile_lx(ct, p), ly = tile_ly(ct, p);
                g[u] = lx < wl && ly < hl ? gt[ly * wc + lx * C] : 0.0f;
              }
#pragma unroll
              for (int j = 0; j < PER; ++j) {
                const float4 w0 = *reinterpret_cast<const float4*>(&s_om[wave * PER + j][p0]);
                const float4 w1 = *reinterpret_cast<const float4*>(&s_om[wave * PER + j][p0 + 4]);
                float a = acc[j];
                a = fmaf(w0.x, g[0], a);
                a = fmaf(w0.y, g[1], a);
                a = fmaf(w0.z, g[2], a);
                a = fmaf(w0.w, g[3], a);
                a = fmaf(w1.x, g[4], a);
                a = fmaf(w1.y, g[5], a);
                a = fmaf(w1.z, g[6], a);
                a = fmaf(w1.w, g[7], a);
                acc[j] = a;
              }
            }
#pragma unroll
            for (int j = 0; j < PER; ++j) {
              const int k = wave * PER + j;
              if (k < nb) {
                const size_t slot = eid[start + lo + k];
                fpart[slot * C + c] = acc[j];
                if (c == 0) fflag[slot] = 1;
              }
            }
          }
        }
      }
    }
    if constexpr (MODE == kFull && DM) {
      if (g_feat) {
        __syncthreads();
        const int li = lane & 15, lk = lane >> 4;
        const int ncb = (C + 15) >> 4;
        // the tile's pixels inside the image: wl columns, hl rows
        const int wl = min(ct.tw, W - tx * ct.tw), hl = min(ct.th, H - ty * ct.th);
        for (int unit = wave; unit < 2 * ncb; unit += 4) {
          const int eb = unit & 1, cb = unit >> 1;
          const int c = 16 * cb + li;
          f4v racc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
          const float* wrow = s_om[16 * eb + li];
          // G of the lane's first pixel (tile column lk, row 0); step t covers
          // pixels 4 t + lk (row-major in the tile, tw a multiple of 4), whose
          // offsets from it are the same for all lanes and below 2^29 (W, C
          // and the tile height are bounded)
          const float* gt = g_feat + (tl.pix0 + (int64_t)(ty * ct.th) * W + tx * ct.tw + lk) * C + c;
          // 128 pixels (32 steps) at a time: their 32 G values are loaded
          // together, so enough of them are in flight to cover the memory
          // latency
          for (int t0 = 0; t0 < kTilePix / 4; t0 += 32) {
            // the shape values go through an empty asm statement so that the
            // step offsets and bounds are formed here and not kept live
            // across units (64 of them would not fit in the registers)
            int wc = W * C, cs = C, tm = ct.tw - 1, sh = ct.tsh, wlim = wl - lk, hlim = hl;
            asm volatile("" : "+s"(wc), "+s"(cs), "+s"(tm), "+s"(sh), "+v"(wlim), "+s"(hlim));
            float b[32];
#pragma unroll
            for (int t = 0; t < 32; ++t) {
              const int q4 = 4 * (t0 + t), lx = q4 & tm, ly = q4 >> sh;
              b[t] = lx < wlim && ly < hlim && c < C ? gt[ly * wc + lx * cs] : 0.0f;
            }
#pragma unroll
            for (int t = 0; t < 32; ++t) racc[t & 1] = mfma_16x16x4(wrow[4 * (t0 + t) + lk], b[t], racc[t & 1]);
          }
          const f4v rs = racc[0] + racc[1];
          if (c < C) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int k = 16 * eb + 4 * lk + r;
              if (k < nb) {
                const size_t slot = eid[start + lo + k];
                fpart[slot * C + c] = rs[r];
                if (c == 0) fflag[slot] = 1;
              }
            }
          }
        }
      }
    }
  }
  });
}

// ------------------------------------------------------- per-surfel reduction

// Chain rule of one camera's view of a surfel: from the 16 pair sums G (dL/d
// of A^-1 (4), e (2), projected centre (2), centre depth, o, c (3), n_c (3))
// to the surfel parameters.  The walk record was evaluated in FP64 from the
// FP32 inputs; its chain rule is evaluated the same way.
struct SurfelGrad {
  double mu[3], su, sv, q[4], o, rgb[3];
};

__device__ __forceinline__ void chain_rule(const double (&G)[16], const CamArgs& k, bool flip, const double (&mu)[3],
                                           double su, double sv, const double (&qn)[4], const double (&Rq)[3][3],
                                           SurfelGrad& acc) {
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  double mc[3], ra[3], rb[3], a[3], b[3];
  for (int r = 0; r < 3; ++r) {
    const float* Rr = k.R + 3 * r;
    mc[r] = Rr[0] * mu[0] + Rr[1] * mu[1] + Rr[2] * mu[2] + (double)k.t[r];
    ra[r] = Rr[0] * Rq[0][0] + Rr[1] * Rq[1][0] + Rr[2] * Rq[2][0];
    rb[r] = Rr[0] * Rq[0][1] + Rr[1] * Rq[1][1] + Rr[2] * Rq[2][1];
    a[r] = su * ra[r];
    b[r] = sv * rb[r];
  }
  const double sgn = flip ? -1.0 : 1.0;  // orientation chosen by the key stage
  const double fx = k.fx, fy = k.fy;
  const double iz = 1.0 / mc[2];
  const double p = a[2] * iz, q = b[2] * iz;
  const double mx = mc[0] * iz, my = mc[1] * iz;
  const double B00 = fx * (a[0] - mx * a[2]), B01 = fx * (b[0] - mx * b[2]);
  const double B10 = fy * (a[1] - my * a[2]), B11 = fy * (b[1] - my * b[2]);
  const double A00 = B00 * iz, A01 = B01 * iz, A10 = B10 * iz, A11 = B11 * iz;
  const double idA = 1.0 / (A00 * A11 - A01 * A10);
  const double Ai[2][2] = {{A11 * idA, -A01 * idA}, {-A10 * idA, A00 * idA}};
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
  double dtu[3], dtv[3], dnn[3];
  for (int c = 0; c < 3; ++c) {
    const double R0 = k.R[c], R1 = k.R[3 + c], R2 = k.R[6 + c];
    dtu[c] = su * (R0 * d_a[0] + R1 * d_a[1] + R2 * d_a[2]);
    dtv[c] = sv * (R0 * d_b[0] + R1 * d_b[1] + R2 * d_b[2]);
    dnn[c] = R0 * dn[0] + R1 * dn[1] + R2 * dn[2];
    acc.mu[c] += R0 * d_mc[0] + R1 * d_mc[1] + R2 * d_mc[2];
  }
  acc.su += d_a[0] * ra[0] + d_a[1] * ra[1] + d_a[2] * ra[2];
  acc.sv += d_b[0] * rb[0] + d_b[1] * rb[1] + d_b[2] * rb[2];
  // Rq columns are t_u, t_v, n;  Gm[r][c] = dL/dRq[r][c]
  const double Gm[3][3] = {{dtu[0], dtv[0], dnn[0]}, {dtu[1], dtv[1], dnn[1]}, {dtu[2], dtv[2], dnn[2]}};
  acc.q[0] += 2. * (-z * Gm[0][1] + y * Gm[0][2] + z * Gm[1][0] - x * Gm[1][2] - y * Gm[2][0] + x * Gm[2][1]);
  acc.q[1] += 2. * (y * Gm[0][1] + z * Gm[0][2] + y * Gm[1][0] - 2. * x * Gm[1][1] - w * Gm[1][2] + z * Gm[2][0] +
                    w * Gm[2][1] - 2. * x * Gm[2][2]);
  acc.q[2] += 2. * (-2. * y * Gm[0][0] + x * Gm[0][1] + w * Gm[0][2] + x * Gm[1][0] + z * Gm[1][2] - w * Gm[2][0] +
                    z * Gm[2][1] - 2. * y * Gm[2][2]);
  acc.q[3] += 2. * (-2. * z * Gm[0][0] - w * Gm[0][1] + x * Gm[0][2] + w * Gm[1][0] - 2. * z * Gm[1][1] +
                    y * Gm[1][2] + x * Gm[2][0] + y * Gm[2][1]);
  acc.o += G[9];
  acc.rgb[0] += G[10];
  acc.rgb[1] += G[11];
  acc.rgb[2] += G[12];
}

// Thread per surfel: for each camera in order, the sum of its pairs' partials
// (its emitted range [vbase, vbase + count), in emission order), then that
// camera's chain rule; the cameras' contributions are added in camera order.
// A surfel's pair count ranges from 0 to several hundred (a heavy tail), so
// the wave's 64 ranges are read as one flat sequence: lane l loads pair
// t0 + l of it (coalesced), the batch is staged in LDS, and each surfel's
// lane adds its own pairs of the batch.  The sums are the same, term by
// term, as a per-surfel loop over its range.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_reduce_geo(int64_t n, CamTable ct, const uint32_t* __restrict__ vbase,
                                                    const uint32_t* __restrict__ count, int64_t cap,
                                                    const float* __restrict__ gpart,
                                                    const uint8_t* __restrict__ gflag,
                                                    const float* __restrict__ means, const float* __restrict__ scales,
                                                    const float* __restrict__ quats, const int32_t* __restrict__ cull,
                                                    float* __restrict__ d_means, float* __restrict__ d_scales,
                                                    float* __restrict__ d_quats, float* __restrict__ d_opacity,
                                                    float* __restrict__ d_rgb) {
  constexpr int kPS = 17;  // LDS row stride of a staged pair (16 partials)
  __shared__ float s_part[4][64 * kPS];
  __shared__ uint32_t s_pre[4][64];
  __shared__ uint32_t s_vb[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = ((int64_t)blockIdx.x * 4 + wave) * 64 + lane;
  const bool valid = i < n;  // every lane stays: the wave shares the pair loads
  const int64_t ii = valid ? i : 0;
  SurfelGrad acc;
  for (int j = 0; j < 3; ++j) acc.mu[j] = acc.rgb[j] = 0.0;
  for (int j = 0; j < 4; ++j) acc.q[j] = 0.0;
  acc.su = acc.sv = acc.o = 0.0;
  // the surfel's parameters are re-read (an L1/L2 hit) where they are used
  // rather than held through the pair sums: it keeps the kernel's registers
  // to what the sums and the chain rule need
  struct Params {
    double mu[3], su, sv, rn, qn[4], Rq[3][3];
  };
  auto params = [&](Params& P) {
    P.mu[0] = means[3 * ii]; P.mu[1] = means[3 * ii + 1]; P.mu[2] = means[3 * ii + 2];
    P.su = scales[2 * ii]; P.sv = scales[2 * ii + 1];
    const double q0 = quats[4 * ii], q1 = quats[4 * ii + 1], q2 = quats[4 * ii + 2], q3 = quats[4 * ii + 3];
    const double qq = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
    P.rn = qq > 0.0 ? 1.0 / sqrt(qq) : 0.0;
    P.qn[0] = q0 * P.rn; P.qn[1] = q1 * P.rn; P.qn[2] = q2 * P.rn; P.qn[3] = q3 * P.rn;
    const double w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
    P.Rq[0][0] = 1. - 2. * (y * y + z * z); P.Rq[0][1] = 2. * (x * y - w * z); P.Rq[0][2] = 2. * (x * z + w * y);
    P.Rq[1][0] = 2. * (x * y + w * z); P.Rq[1][1] = 1. - 2. * (x * x + z * z); P.Rq[1][2] = 2. * (y * z - w * x);
    P.Rq[2][0] = 2. * (x * z - w * y); P.Rq[2][1] = 2. * (y * z + w * x); P.Rq[2][2] = 1. - 2. * (x * x + y * y);
  };
  float* part = s_part[wave];
  // the next camera's pair range is loaded while this camera's is summed
  int32_t ncv = valid ? cull[i] : 1;
  uint32_t nvb = valid ? vbase[i] : 0u, nvc = valid ? count[i] : 0u;
#pragma unroll 1
  for (int b = 0; b < ct.n; ++b) {
    const int32_t cv = ncv;
    const uint32_t vb = nvb;
    const int64_t end = min((int64_t)vb + (int64_t)nvc, cap);
    if (b + 1 < ct.n && valid) {
      const int64_t v = (int64_t)(b + 1) * n + i;
      ncv = cull[v];
      nvb = vbase[v];
      nvc = count[v];
    }
    const bool live = valid && (cv & 0xFF) == 0;
    const uint32_t cnt = live && end > (int64_t)vb ? (uint32_t)(end - (int64_t)vb) : 0u;
    // the wave's pairs as one flat sequence: surfel l owns [pre_l, pre_l + cnt_l)
    uint32_t xs = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(xs, o, 64);
      if (lane >= o) xs += t;
    }
    const uint32_t pre = xs - cnt, total = __shfl(xs, 63, 64);
    s_pre[wave][lane] = pre;
    s_vb[wave][lane] = vb;
    wave_lds_sync();
    double G[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) G[j] = 0.0;
    for (uint32_t t0 = 0; t0 < total; t0 += 64) {
      // 64 consecutive pairs of the sequence, one per lane; unflagged pairs
      // stage zeros (adding +0 leaves a sum unchanged)
      const uint32_t t = t0 + (uint32_t)lane;
      float4 r[4];
#pragma unroll
      for (int qd = 0; qd < 4; ++qd) r[qd] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (t < total) {
        int o = 0;  // owner: the last surfel whose range starts at or before t
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)
          if (s_pre[wave][o + step] <= t) o += step;
        const uint32_t pr = s_vb[wave][o] + (t - s_pre[wave][o]);
        if (gflag[pr]) {
          const float4* g = reinterpret_cast<const float4*>(gpart + (size_t)pr * 16);
#pragma unroll
          for (int qd = 0; qd < 4; ++qd) r[qd] = g[qd];
        }
      }
#pragma unroll
      for (int qd = 0; qd < 4; ++qd) {
        part[lane * kPS + 4 * qd] = r[qd].x;
        part[lane * kPS + 4 * qd + 1] = r[qd].y;
        part[lane * kPS + 4 * qd + 2] = r[qd].z;
        part[lane * kPS + 4 * qd + 3] = r[qd].w;
      }
      wave_lds_sync();
      // each surfel adds its pairs of this batch in emission order
      const uint32_t lo = max(pre, t0), hi = min(pre + cnt, t0 + 64u);
      for (uint32_t u = lo; u < hi; ++u) {
        const float* pp = part + (u - t0) * kPS;
#pragma unroll
        for (int j = 0; j < 16; ++j) G[j] += pp[j];
      }
      wave_lds_sync();
    }
    if (live) {
      Params P;
      params(P);
      chain_rule(G, ct.cam[b], ((cv >> 8) & 1) != 0, P.mu, P.su, P.sv, P.qn, P.Rq, acc);
    }
  }
  if (!valid) return;
  Params P;
  params(P);
  // unit quaternion: project out the radial component
  const double dot = P.qn[0] * acc.q[0] + P.qn[1] * acc.q[1] + P.qn[2] * acc.q[2] + P.qn[3] * acc.q[3];
  for (int j = 0; j < 4; ++j) d_quats[4 * i + j] = (float)((acc.q[j] - P.qn[j] * dot) * P.rn);
  for (int j = 0; j < 3; ++j) d_means[3 * i + j] = (float)acc.mu[j];
  d_scales[2 * i] = (float)acc.su;
  d_scales[2 * i + 1] = (float)acc.sv;
  d_opacity[i] = (float)acc.o;
  for (int j = 0; j < 3; ++j) d_rgb[3 * i + j] = (float)acc.rgb[j];
}

// Lane group per surfel: dL/df = sum over cameras (in order) of the sum of its
// pairs' rows (emission order), channels [0, ca) written to dfa (row stride
// ca), channels [ca, C) to dfb (row stride C - ca); either may be null.
// A surfel with more than kHeavyRows flagged rows is not summed here (its
// rows would follow one another, four per round trip, and hold the whole
// kernel): the group stops when its count passes the bound and puts the
// surfel on the heavy list for k_reduce_feat_heavy.  The choice depends only
// on the surfel's flagged rows, like each path's order of addition.
template <int NG>
__global__ __launch_bounds__(256) void k_reduce_feat(int64_t n, int ncam, const uint32_t* __restrict__ vbase,
                                                     const uint32_t* __restrict__ count, int64_t cap,
                                                     const float* __restrict__ fpart,
                                                     const uint8_t* __restrict__ fflag, int C, int lpp2,
                                                     float* __restrict__ dfa, float* __restrict__ dfb, int ca,
                                                     uint32_t* __restrict__ heavy, uint32_t* __restrict__ status) {
  // lpp2 lanes (a power of two) per surfel, each lane up to NG float4 channel
  // groups: a wave reduces 64 / lpp2 surfels at once
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lpp = C / 4;
  const int spw = 64 / lpp2;
  const int sub = lane / lpp2, cl = lane % lpp2;
  const int64_t i = ((int64_t)blockIdx.x * 4 + wave) * spw + sub;
  if (i >= n) return;
  constexpr int kMaxGroups = NG;  // channel groups of 4 per lane (the registers it needs)
  constexpr int kRowsInFlight = 4;
  uint32_t nf = 0;  // flagged rows met so far (the same in every lane of the group)
  float4 acc[kMaxGroups];
#pragma unroll
  for (int j = 0; j < kMaxGroups; ++j) acc[j] = make_float4(0.f, 0.f, 0.f, 0.f);
  const int ng = (lpp + lpp2 - 1) / lpp2;  // channel groups of this lane
  const uint64_t gmask = lpp2 == 64 ? ~0ull : ((1ull << lpp2) - 1ull);
  uint32_t nvb = vbase[i], nvc = count[i];
#pragma unroll 1
  for (int b = 0; b < ncam; ++b) {
    const int64_t base = nvb;
    const int64_t end = min(base + (int64_t)nvc, cap);
    if (b + 1 < ncam) {
      const int64_t v = (int64_t)(b + 1) * n + i;
      nvb = vbase[v];
      nvc = count[v];
    }
    // a scan tests `steps` strides of lpp2 flags at once (up to 64 slots, one
    // 64-bit mask: bit t = slot s0 + t), so a surfel with many pairs and few
    // flagged rows waits for one flag load per 64 slots, not per lpp2; the
    // flagged rows in emission order, up to kRowsInFlight rows loaded before
    // they are added
    const int steps = lpp2 >= 8 ? 64 / lpp2 : 8;
    for (int64_t s0 = base; s0 < end; s0 += (int64_t)steps * lpp2) {
      bool fl[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t sj = s0 + (int64_t)j * lpp2 + cl;
        fl[j] = j < steps && sj < end && fflag[sj];
      }
      uint64_t m = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < steps) m |= ((__ballot(fl[j]) >> (sub * lpp2)) & gmask) << (j * lpp2);
      nf += (uint32_t)__popcll(m);
      if (nf > (uint32_t)kHeavyRows) {
        if (cl == 0) heavy[atomicAdd(status + kStHeavy, 1u)] = (uint32_t)i;
        return;
      }
      while (m) {
        int us[kRowsInFlight];
#pragma unroll
        for (int r = 0; r < kRowsInFlight; ++r) {
          us[r] = m ? __ffsll((unsigned long long)m) - 1 : -1;
          m &= m - 1ull;
        }
        float4 t[kRowsInFlight][kMaxGroups];
#pragma unroll
        for (int r = 0; r < kRowsInFlight; ++r) {
          const float* row = fpart + (size_t)(s0 + max(us[r], 0)) * C;
#pragma unroll
          for (int j = 0; j < kMaxGroups; ++j)
            t[r][j] = us[r] >= 0 && j < ng && cl + j * lpp2 < lpp
                          ? *reinterpret_cast<const float4*>(row + (cl + j * lpp2) * 4)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int r = 0; r < kRowsInFlight; ++r)
#pragma unroll
          for (int j = 0; j < kMaxGroups; ++j)
            if (us[r] >= 0) {
              acc[j].x += t[r][j].x; acc[j].y += t[r][j].y; acc[j].z += t[r][j].z; acc[j].w += t[r][j].w;
            }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kMaxGroups; ++j)
    if (j < ng && cl + j * lpp2 < lpp) {
      const int c = (cl + j * lpp2) * 4;  // ca % 4 == 0: the group lies in one output
      float* dst = c < ca ? (dfa ? dfa + (size_t)i * ca + c : nullptr)
                          : (dfb ? dfb + (size_t)i * (C - ca) + (c - ca) : nullptr);
      if (dst) *reinterpret_cast<float4*>(dst) = acc[j];
    }
}

// Block per heavy surfel (a fixed grid strides over the heavy list, whose
// length it reads on the device): CL channel lanes (float4 groups) x R =
// 256 / CL row lanes.  The surfel's flagged slots are compacted in emission
// order (camera by camera, 256 slots a step, block prefix count) into an LDS
// list; row lane r adds, in rank order, the rows whose rank among the
// surfel's flagged rows is r mod R, four rows in flight, and the R partial
// rows are then added in row-lane order.  The partition depends only on the
// sequence of flagged rows: the result is deterministic, the same for every
// launch choice, and unchanged by pairs that carry no row.
constexpr int kHvList = 2048;
__global__ __launch_bounds__(256) void k_reduce_feat_heavy(int64_t n, int ncam, const uint32_t* __restrict__ vbase,
                                                           const uint32_t* __restrict__ count, int64_t cap,
                                                           const float* __restrict__ fpart,
                                                           const uint8_t* __restrict__ fflag, int C,
                                                           float* __restrict__ dfa, float* __restrict__ dfb, int ca,
                                                           const uint32_t* __restrict__ heavy,
                                                           const uint32_t* __restrict__ status) {
  __shared__ uint32_t s_slot[kHvList];
  __shared__ float4 s_acc[256];
  __shared__ uint32_t s_red[8];
  const int t = threadIdx.x;
  const int G = C / 4, CL = min(G, 64), R = 256 / CL;
  const int rl = t / CL, cl = t % CL;
  const uint32_t nh = status[kStHeavy];
  for (uint32_t h = blockIdx.x; h < nh; h += gridDim.x) {
    const int64_t i = heavy[h];
    for (int g0 = 0; g0 < G; g0 += CL) {
      const int g = g0 + cl;
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      uint32_t nl = 0, rank0 = 0;  // listed slots, rank of the first (block-uniform)
      // the listed rows added by their row lanes; the list is then empty
      auto drain = [&]() {
        __syncthreads();
        if (rl < R && g < G) {
          for (uint32_t j = (uint32_t)((rl + R - (int)(rank0 % (uint32_t)R)) % R); j < nl; j += 4u * R) {
            float4 x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const uint32_t jj = j + (uint32_t)(u * R);
              x[u] = jj < nl ? *reinterpret_cast<const float4*>(fpart + (size_t)s_slot[jj] * C + 4 * g)
                             : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              acc.x += x[u].x; acc.y += x[u].y; acc.z += x[u].z; acc.w += x[u].w;
            }
          }
        }
        rank0 += nl;
        nl = 0;
        __syncthreads();
      };
      for (int b = 0; b < ncam; ++b) {
        const int64_t v = (int64_t)b * n + i, base = vbase[v];
        const int64_t end = min(base + (int64_t)count[v], cap);
        for (int64_t c0 = base; c0 < end; c0 += 256) {
          const bool f = c0 + t < end && fflag[c0 + t];
          uint32_t total;
          const uint32_t pre = block_scan_excl(f ? 1u : 0u, s_red, total);
          if (f) s_slot[nl + pre] = (uint32_t)(c0 + t);  // nl <= kHvList - 256 here
          nl += total;
          if (nl > (uint32_t)(kHvList - 256)) drain();
        }
      }
      drain();
      s_acc[t] = acc;
      __syncthreads();
      if (rl == 0 && g < G) {
        float4 sum = s_acc[cl];
        for (int r = 1; r < R; ++r) {
          const float4 y = s_acc[r * CL + cl];
          sum.x += y.x; sum.y += y.y; sum.z += y.z; sum.w += y.w;
        }
        const int c = 4 * g;  // ca % 4 == 0: the group lies in one output
        float* dst = c < ca ? (dfa ? dfa + (size_t)i * ca + c : nullptr)
                            : (dfb ? dfb + (size_t)i * (C - ca) + (c - ca) : nullptr);
        if (dst) *reinterpret_cast<float4*>(dst) = sum;
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------- host wrappers
template <typename FT, int KMAX, int GC, bool PERSIST>
static void feat_bwd_launch(const SurfelArgs& s, const Layout& L, const CamTable& ct, const Tuning& tu,
                            const ImageGradArgs& g, bool renorm, char* ws, hipStream_t st) {
  const size_t shm = (size_t)kWRow * L.k * sizeof(float);  // weights, then dots
  const void* k = reinterpret_cast<const void*>(&k_feat_bwd_topk<FT, KMAX, GC, PERSIST>);
  hipLaunchKernelGGL((k_feat_bwd_topk<FT, KMAX, GC, PERSIST>), dim3(tile_grid(L, tu.sched_bwd, k, shm)), dim3(256), shm, st,
                     (const uint32_t*)(ws + L.pid), (const uint32_t*)(ws + L.eid0), (const uint2*)(ws + L.ranges),
                     (const int32_t*)(ws + L.selpos), (const float*)(ws + L.selw), feat_src<FT>(s), g.feat, s.c, L.k,
                     ct, tile_queue(L, tu.sched_bwd, ws, kQFeatBwd), (float*)(ws + L.seldot), (float*)(ws + L.fpart),
                     (uint8_t*)(ws + L.fflag), renorm ? 1 : 0);
}

template <typename FT, int GC>
static void feat_bwd_k(const SurfelArgs& s, const Layout& L, const CamTable& ct, const Tuning& tu,
                       const ImageGradArgs& g, bool rn, char* ws, hipStream_t st) {
  const bool p = tu.sched_bwd == kSchedPersistent;
  if (L.k <= 8) (p ? feat_bwd_launch<FT, 8, GC, true> : feat_bwd_launch<FT, 8, GC, false>)(s, L, ct, tu, g, rn, ws, st);
  else if (L.k <= 16)
    (p ? feat_bwd_launch<FT, 16, GC, true> : feat_bwd_launch<FT, 16, GC, false>)(s, L, ct, tu, g, rn, ws, st);
  else (p ? feat_bwd_launch<FT, 32, GC, true> : feat_bwd_launch<FT, 32, GC, false>)(s, L, ct, tu, g, rn, ws, st);
}

template <int MODE, typename FT, bool PERSIST, bool LP, bool DM>
static void walk_bwd_launch_d(const SurfelArgs& s, const Layout& L, const CamTable& ct, const Tuning& tu,
                              const ImageGradArgs& g, bool want_f, char* ws, hipStream_t st) {
  const void* k = reinterpret_cast<const void*>(&k_walk_bwd<MODE, FT, PERSIST, LP, DM>);
  const size_t shm = MODE == kTopK ? (size_t)L.k * kTilePix * 4 : 0;  // selection positions
  hipLaunchKernelGGL((k_walk_bwd<MODE, FT, PERSIST, LP, DM>), dim3(tile_grid(L, tu.sched_bwd, k, shm)), dim3(256), shm,
                     st, (const WalkRec*)(ws + L.rec), (const float4*)(ws + L.ext), (const uint32_t*)(ws + L.pid),
                     (const uint32_t*)(ws + L.eid0), (const uint2*)(ws + L.ranges), ct,
                     tile_queue(L, tu.sched_bwd, ws, kQWalkBwd), L.k,
                     (const uint32_t*)(ws + L.nlast), (const float*)(ws + L.tfinal), (const int32_t*)(ws + L.selpos),
                     (const float*)(ws + L.seldot), g.rgb, g.depth, g.normal, g.alpha, want_f ? g.feat : nullptr,
                     feat_src<FT>(s), s.c, (float*)(ws + L.gpart), (uint8_t*)(ws + L.gflag), (float*)(ws + L.fpart),
                     (uint8_t*)(ws + L.fflag));
}

// dense mode: the feature-backward pass width selects the contraction unit
// (16: vector FMAs, 32: matrix cores)
template <int MODE, typename FT, bool PERSIST, bool LP>
static void walk_bwd_launch_t(const SurfelArgs& s, const Layout& L, const CamTable& ct, const Tuning& tu,
                              const ImageGradArgs& g, bool want_f, char* ws, hipStream_t st) {
  if (MODE == kFull && tu.bwd_pass == 32) walk_bwd_launch_d<MODE, FT, PERSIST, LP, true>(s, L, ct, tu, g, want_f, ws, st);
  else walk_bwd_launch_d<MODE, FT, PERSIST, LP, false>(s, L, ct, tu, g, want_f, ws, st);
}

template <int MODE, typename FT>
static void walk_bwd_launch(const SurfelArgs& s, const Layout& L, const CamTable& ct, const Tuning& tu,
                            const ImageGradArgs& g, bool want_f, bool lp, char* ws, hipStream_t st) {
  const bool p = tu.sched_bwd == kSchedPersistent;
  if (lp)
    (p ? walk_bwd_launch_t<MODE, FT, true, true> : walk_bwd_launch_t<MODE, FT, false, true>)(s, L, ct, tu, g, want_f,
                                                                                           ws, st);
  else
    (p ? walk_bwd_launch_t<MODE, FT, true, false> : walk_bwd_launch_t<MODE, FT, false, false>)(s, L, ct, tu, g,
                                                                                             want_f, ws, st);
}

template <typename FT>
static void backward_typed(const SurfelArgs& s, const CamTable& ct, int blend, const Tuning& tu, const Layout& L,
                           const ImageGradArgs& g, const GradArgs& gr, bool renorm, bool lp, char* ws,
                           hipStream_t st, const ProfHook& prof) {
  const bool want_f = g.feat != nullptr && s.c > 0;
  if (L.tiles > 0) {
    if (blend == kTopK) {
      prof.begin(kStageBwdFeature, st);
      if (want_f) {
        if (tu.bwd_pass == 32) feat_bwd_k<FT, 32>(s, L, ct, tu, g, renorm, ws, st);
        else feat_bwd_k<FT, 16>(s, L, ct, tu, g, renorm, ws, st);
      } else {
        launch_fill_u32(ws + L.seldot, 0u, L.spix * (int64_t)L.k, st);
      }
      prof.end(kStageBwdFeature, st);
      prof.begin(kStageBwdWalk, st);
      walk_bwd_launch<kTopK, FT>(s, L, ct, tu, g, want_f, lp, ws, st);
      prof.end(kStageBwdWalk, st);
    } else {
      prof.begin(kStageBwdWalk, st);
      walk_bwd_launch<kFull, FT>(s, L, ct, tu, g, want_f, lp, ws, st);
      prof.end(kStageBwdWalk, st);
    }
  }
  prof.begin(kStageBwdPreprocess, st);
  const uint32_t* vbase = (const uint32_t*)(ws + L.vbase);
  const uint32_t* count = (const uint32_t*)(ws + L.count);
  if (s.n > 0) {
    hipLaunchKernelGGL(k_reduce_geo, dim3((unsigned)cdiv(s.n, 256)), dim3(256), 0, st, s.n, ct, vbase, count, L.cap,
                       (const float*)(ws + L.gpart), (const uint8_t*)(ws + L.gflag), s.means, s.scales, s.quats,
                       (const int32_t*)(ws + L.cull), gr.means, gr.scales, gr.quats, gr.opacity, gr.rgb);
    if (s.c > 0 && (gr.feat || gr.feat_ext)) {
      // two channel groups per lane (at most 4 for C = 1024): more surfels,
      // and so more independent row loads, in flight per wave
      const int lpp = s.c / 4;
      const int lpp2 = std::min(64, pow2_ge_host((lpp + 1) / 2));
      const int per_block = 4 * (64 / lpp2);
      const int ng = (lpp + lpp2 - 1) / lpp2;  // 1 or 2 up to C = 512, else at most 4
      auto k = ng <= 2 ? k_reduce_feat<2> : k_reduce_feat<4>;
      uint32_t* status = (uint32_t*)(ws + L.status);
      uint32_t* heavy = (uint32_t*)(ws + L.heavy);
      launch_fill_u32(status + kStHeavy, 0u, 1, st);
      hipLaunchKernelGGL(k, dim3((unsigned)cdiv(s.n, per_block)), dim3(256), 0, st, s.n, ct.n, vbase,
                         count, L.cap, (const float*)(ws + L.fpart), (const uint8_t*)(ws + L.fflag), s.c, lpp2,
                         gr.feat, gr.feat_ext, s.ca, heavy, status);
      const unsigned gh = (unsigned)std::min<int64_t>(L.cap / (kHeavyRows + 1) + 1, 1024);
      hipLaunchKernelGGL(k_reduce_feat_heavy, dim3(gh), dim3(256), 0, st, s.n, ct.n, vbase, count, L.cap,
                         (const float*)(ws + L.fpart), (const uint8_t*)(ws + L.fflag), s.c, gr.feat, gr.feat_ext, s.ca,
                         (const uint32_t*)heavy, (const uint32_t*)status);
    }
  }
  prof.end(kStageBwdPreprocess, st);
}

void launch_backward(const SurfelArgs& s, const CamTable& ct, int blend, const Tuning& tu, const Layout& L,
                     const ImageGradArgs& g, const GradArgs& grads, bool renorm, bool lowpass, char* ws,
                     hipStream_t st, const ProfHook& prof) {
  prof.begin(kStageFill, st);
  launch_fill_u32(ws + L.gflag, 0u, cdiv(std::max<int64_t>(L.cap, 1), 4), st);
  launch_fill_u32(ws + L.fflag, 0u, cdiv(std::max<int64_t>(L.cap, 1), 4), st);
  launch_fill_u32((uint32_t*)(ws + L.status) + kStQueue + kQFeatBwd, 0u, 2, st);
  prof.end(kStageFill, st);
  if (s.dtype == kF32) backward_typed<float>(s, ct, blend, tu, L, g, grads, renorm, lowpass, ws, st, prof);
  else if (s.dtype == kF16) backward_typed<__half>(s, ct, blend, tu, L, g, grads, renorm, lowpass, ws, st, prof);
  else backward_typed<uint16_t>(s, ct, blend, tu, L, g, grads, renorm, lowpass, ws, st, prof);
}

}  // namespace psm
