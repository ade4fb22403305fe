// Frustum-local cross-attention of instance queries over surfels (Sec. 4.1,
// eqs. (9)-(11)):
//   active set: surfels whose 99% confidence disk (rho <= -2 ln 0.01 in its
//     own plane) has a bounding sphere meeting the view frustum (near plane
//     and the four planes through the camera centre and the image borders);
//     an FP32 test in a prescribed operation order,
//   K_j = f_j + psi(mu_j), V_j = f_j,
//   e_ij = (Q_i W_Q) . (K_j W_K) / sqrt(d),  Q'_i = sum_j softmax_j(e_ij) V_j W_V.
//
// The active surfels are compacted in surfel order (per-block counts, one
// scan, an in-order scatter).  The attention is a dense contraction on the
// matrix cores (FP32 v_mfma_f32_16x16x4f32, exact products): a fixed grid of
// blocks splits the active list into contiguous ranges; a block stages 64
// keys at a time in LDS, projects them (K W_K, V W_V), and per wave and
// 16-query block forms the score tile S^T (16 keys x 16 queries), the online
// softmax (running maximum and sum per query) and O^T += (V W_V)^T P^T.  The
// k-step of the last product takes the keys 4 g + r of a 16-key block (g =
// lane group), which is exactly how the score tile's registers hold them, so
// P never leaves the registers.  Each block writes (maximum, sum, O) per
// query; a last kernel merges the blocks in block order, so the result does
// not depend on timing.
#include "common.h"
#include "internal.h"

namespace psm {

constexpr float kR99 = 3.03485425877029f;  // sqrt(-2 ln 0.01) rounded to FP32
constexpr int kAttKeys = 64;               // keys staged per step
constexpr int kAttCullBlock = 256;

// ------------------------------------------------------------- active set
__device__ __forceinline__ bool frustum_meets(const float* mu, const float* sc, const CamArgs& k, float nl, float nr,
                                              float nt, float nb) {
  float mc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float R0 = k.R[3 * i], R1 = k.R[3 * i + 1], R2 = k.R[3 * i + 2];
    mc[i] = ((R0 * mu[0] + R1 * mu[1]) + R2 * mu[2]) + k.t[i];
  }
  const float rr = kR99 * fmaxf(sc[0], sc[1]);
  const float W = (float)k.W, H = (float)k.H;
  bool a = (mc[2] - k.near_plane) >= -rr;
  a = a && (k.fx * mc[0] + k.cx * mc[2]) >= -(rr * nl);
  a = a && ((W - k.cx) * mc[2] - k.fx * mc[0]) >= -(rr * nr);
  a = a && (k.fy * mc[1] + k.cy * mc[2]) >= -(rr * nt);
  a = a && ((H - k.cy) * mc[2] - k.fy * mc[1]) >= -(rr * nb);
  return a;
}

// Thread per surfel: active flag and the block's active count.
__global__ __launch_bounds__(kAttCullBlock) void k_att_cull(int64_t n, const float* __restrict__ means,
                                                            const float* __restrict__ scales, CamArgs k,
                                                            uint8_t* __restrict__ active, uint32_t* __restrict__ blkcnt) {
  __shared__ uint32_t s_cnt[kAttCullBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kAttCullBlock + threadIdx.x;
  const float W = (float)k.W, H = (float)k.H;
  // plane normal lengths, the same FP32 operations for every thread
  const float nl = sqrtf(k.fx * k.fx + k.cx * k.cx);
  const float nr = sqrtf(k.fx * k.fx + (W - k.cx) * (W - k.cx));
  const float nt = sqrtf(k.fy * k.fy + k.cy * k.cy);
  const float nb = sqrtf(k.fy * k.fy + (H - k.cy) * (H - k.cy));
  bool a = false;
  if (i < n) {
    a = frustum_meets(means + 3 * i, scales + 2 * i, k, nl, nr, nt, nb);
    active[i] = a ? 1 : 0;
  }
  const uint64_t m = __ballot(a);
  if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = (uint32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kAttCullBlock / 64; ++w) c += s_cnt[w];
    blkcnt[blockIdx.x] = c;
  }
}

// One block: exclusive scan of the block counts; off[nb] = number active.
__global__ __launch_bounds__(1024) void k_att_scan(int64_t nb, const uint32_t* __restrict__ cnt,
                                                   uint32_t* __restrict__ off) {
  __shared__ uint32_t s_w[16];
  __shared__ uint32_t s_carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    const int64_t j = b0 + tid;
    const uint32_t v = j < nb ? cnt[j] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    uint32_t pre = s_carry, tot = 0;
    for (int w = 0; w < 16; ++w) {
      pre += w < wave ? s_w[w] : 0u;
      tot += s_w[w];
    }
    if (j < nb) off[j] = pre + x - v;
    __syncthreads();
    if (tid == 0) s_carry += tot;
    __syncthreads();
  }
  if (tid == 0) off[nb] = s_carry;
}

// Thread per surfel: active surfels to the list, in surfel order.
__global__ __launch_bounds__(kAttCullBlock) void k_att_compact(int64_t n, const uint8_t* __restrict__ active,
                                                               const uint32_t* __restrict__ off,
                                                               uint32_t* __restrict__ list) {
  __shared__ uint32_t s_cnt[kAttCullBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kAttCullBlock + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool a = i < n && active[i] != 0;
  const uint64_t m = __ballot(a);
  if (lane == 0) s_cnt[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t base = off[blockIdx.x];
  for (int w = 0; w < wave; ++w) base += s_cnt[w];
  if (a) list[base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)i;
}

// Q W_Q, rows padded to a multiple of 16 with zeros.
__global__ void k_att_qproj(int nq, int nqp, int c, int d, const float* __restrict__ q,
                            const float* __restrict__ wq, float* __restrict__ qp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nqp * d) return;
  const int i = t / d, j = t % d;
  float a = 0.0f;
  if (i < nq)
    for (int k = 0; k < c; ++k) a = fmaf(q[(size_t)i * c + k], wq[(size_t)k * d + j], a);
  qp[t] = a;
}

// psi(mu) channel ch: sin or cos of 2^(ch / 6) pi mu_(ch mod 3) / L.
__device__ __forceinline__ float posenc(const float (&mu)[3], int ch, float inv_len) {
  const int axis = ch % 3, band = ch / 6;
  const float arg = ldexpf(3.14159265358979f, band) * (mu[axis] * inv_len);
  return ((ch / 3) & 1) == 0 ? sinf(arg) : cosf(arg);
}

// ---------------------------------------------------------------- attention
// Block = 4 waves over the key range [k0, k1) of the active list.  CB = C/4
// k-steps of the projections, DB = d/16 column blocks, QW = 16-query blocks
// per wave (nqp / 64, rounded up).
template <typename FT, int C, int D, int QW>
__global__ __launch_bounds__(256) void k_att_main(const uint32_t* __restrict__ list, const uint32_t* __restrict__ nact,
                                                  const float* __restrict__ means, const FT* __restrict__ feat,
                                                  const float* __restrict__ wk, const float* __restrict__ wv,
                                                  const float* __restrict__ qp, int nqp, float inv_len, float scale,
                                                  int nblk, float* __restrict__ part) {
  constexpr int CS = C + 2, DS = D + 2;  // LDS row strides (= 2 mod 4)
  constexpr int DB = D / 16;
  __shared__ float s_wk[C * DS], s_wv[C * DS];
  __shared__ float s_k[kAttKeys * CS], s_v[kAttKeys * CS];
  __shared__ float s_kp[kAttKeys * DS], s_vp[kAttKeys * DS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = tid; t < C * D; t += 256) {
    s_wk[(t / D) * DS + t % D] = wk[t];
    s_wv[(t / D) * DS + t % D] = wv[t];
  }
  const uint32_t M = *nact;
  const uint32_t per = (uint32_t)((cdiv(cdiv(M, nblk), kAttKeys)) * kAttKeys);
  const uint32_t k0 = min((uint32_t)blockIdx.x * per, M), k1 = min(k0 + per, M);

  // score B operands: Qp[16 qb + li][4 ks + lk]; accumulators O^T per query block
  float qf[QW][D / 4];
  f4v o[QW][DB];
  float mrun[QW], srun[QW];
#pragma unroll
  for (int w = 0; w < QW; ++w) {
    const int qb = wave + 4 * w;
#pragma unroll
    for (int ks = 0; ks < D / 4; ++ks) qf[w][ks] = 16 * qb < nqp ? qp[(size_t)(16 * qb + li) * D + 4 * ks + lk] : 0.0f;
#pragma unroll
    for (int db = 0; db < DB; ++db) o[w][db] = f4v{0.f, 0.f, 0.f, 0.f};
    mrun[w] = -INFINITY;
    srun[w] = 0.0f;
  }

  for (uint32_t kc = k0; kc < k1; kc += kAttKeys) {
    const int nk = (int)min((uint32_t)kAttKeys, k1 - kc);
    __syncthreads();  // the previous step's LDS reads are done
    {
      // stage K = f + psi(mu) and V = f: 4 threads per key
      const int kk = tid >> 2;
      float mu[3] = {0.f, 0.f, 0.f};
      size_t row = 0;
      const bool ok = kk < nk;
      if (ok) {
        const uint32_t id = list[kc + kk];
        mu[0] = means[3 * (size_t)id];
        mu[1] = means[3 * (size_t)id + 1];
        mu[2] = means[3 * (size_t)id + 2];
        row = (size_t)id * C;
      }
      for (int ch = tid & 3; ch < C; ch += 4) {
        const float f = ok ? load_one<FT>(feat + row + ch) : 0.0f;
        s_v[kk * CS + ch] = f;
        s_k[kk * CS + ch] = ok ? f + posenc(mu, ch, inv_len) : 0.0f;
      }
    }
    __syncthreads();
    // projections of this wave's 16 keys: rows 16 wave .. +16 of K W_K, V W_V
#pragma unroll
    for (int db = 0; db < DB; ++db) {
      f4v ak = f4v{0.f, 0.f, 0.f, 0.f}, av = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < C / 4; ++ks) {
        const int r = (16 * wave + li) * CS + 4 * ks + lk;
        const int wrow = (4 * ks + lk) * DS + 16 * db + li;
        ak = mfma_16x16x4(s_k[r], s_wk[wrow], ak);
        av = mfma_16x16x4(s_v[r], s_wv[wrow], av);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        s_kp[(16 * wave + 4 * lk + r) * DS + 16 * db + li] = ak[r];
        s_vp[(16 * wave + 4 * lk + r) * DS + 16 * db + li] = av[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < QW; ++w) {
      const int qb = wave + 4 * w;
      if (16 * qb >= nqp) break;  // wave-uniform
      // S^T tiles: keys 16 kb + 4 lk + r, query li
      f4v s[4];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        s[kb] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < D / 4; ++ks)
          s[kb] = mfma_16x16x4(s_kp[(16 * kb + li) * DS + 4 * ks + lk], qf[w][ks], s[kb]);
      }
      float mx = -INFINITY;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const bool valid = 16 * kb + 4 * lk + r < nk;
          s[kb][r] = valid ? s[kb][r] * scale : -INFINITY;
          mx = fmaxf(mx, s[kb][r]);
        }
      mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
      mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
      const float mnew = fmaxf(mrun[w], mx);  // finite: the step has at least one key
      const float rescale = expf(mrun[w] - mnew);
      float ps = 0.0f;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          s[kb][r] = expf(s[kb][r] - mnew);  // exp(-inf) = 0 for the padding keys
          ps += s[kb][r];
        }
      ps += __shfl_xor(ps, 16, 64);
      ps += __shfl_xor(ps, 32, 64);
      srun[w] = srun[w] * rescale + ps;
      mrun[w] = mnew;
#pragma unroll
      for (int db = 0; db < DB; ++db) {
        o[w][db] *= rescale;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            o[w][db] = mfma_16x16x4(s_vp[(16 * kb + 4 * lk + r) * DS + 16 * db + li], s[kb][r], o[w][db]);
      }
    }
  }
  // partials of this block: [query][2 + D] = (max, sum, O)
#pragma unroll
  for (int w = 0; w < QW; ++w) {
    const int qb = wave + 4 * w;
    if (16 * qb >= nqp) break;
    float* pq = part + ((size_t)blockIdx.x * nqp + 16 * qb + li) * (2 + D);
    if (lk == 0) {
      pq[0] = mrun[w];
      pq[1] = srun[w];
    }
#pragma unroll
    for (int db = 0; db < DB; ++db)
#pragma unroll
      for (int r = 0; r < 4; ++r) pq[2 + 16 * db + 4 * lk + r] = o[w][db][r];
  }
}

// Block per query: merge the blocks' partials.  Thread t takes the blocks
// t, t + 256, ... in order, then the 256 threads are combined by a fixed tree
// (within each wave by xor shuffles, then the 4 waves in order), so the
// result does not depend on timing.
__device__ __forceinline__ float wave_allsum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int D>
__global__ __launch_bounds__(256) void k_att_combine(int nqp, int nblk, const float* __restrict__ part,
                                                     float* __restrict__ out) {
  __shared__ float s_red[4][D + 1];
  __shared__ float s_m[4];
  const int i = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const size_t stride = (size_t)nqp * (2 + D);
  const float* p = part + (size_t)i * (2 + D);
  float m = -INFINITY;
  for (int b = tid; b < nblk; b += 256) m = fmaxf(m, p[b * stride]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if (lane == 0) s_m[wave] = m;
  __syncthreads();
  m = fmaxf(fmaxf(s_m[0], s_m[1]), fmaxf(s_m[2], s_m[3]));
  float s = 0.0f, o[D];
#pragma unroll
  for (int j = 0; j < D; ++j) o[j] = 0.0f;
  if (m > -INFINITY) {
    for (int b = tid; b < nblk; b += 256) {
      const float* pb = p + b * stride;
      const float mb = pb[0];
      if (mb == -INFINITY) continue;  // an empty range
      const float e = expf(mb - m);
      s = fmaf(pb[1], e, s);
#pragma unroll
      for (int j = 0; j < D; ++j) o[j] = fmaf(pb[2 + j], e, o[j]);
    }
  }
  s = wave_allsum(s);
  if (lane == 0) s_red[wave][D] = s;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const float v = wave_allsum(o[j]);
    if (lane == 0) s_red[wave][j] = v;
  }
  __syncthreads();
  if (tid < D) {
    const float st = ((s_red[0][D] + s_red[1][D]) + s_red[2][D]) + s_red[3][D];
    const float ot = ((s_red[0][tid] + s_red[1][tid]) + s_red[2][tid]) + s_red[3][tid];
    out[(size_t)i * D + tid] = st > 0.0f ? ot / st : 0.0f;
  }
}

// ------------------------------------------------------------------ host
size_t attention_workspace_bytes(int64_t n, int nq, int d, int nblk) {
  const int64_t nb = cdiv(std::max<int64_t>(n, 1), kAttCullBlock);
  const int nqp = (int)cdiv(nq, 16) * 16;
  size_t b = 0;
  auto take = [&](size_t bytes) { b += (bytes + 255) & ~(size_t)255; };
  take((size_t)std::max<int64_t>(n, 1));          // active flags
  take((size_t)nb * 4);                           // block counts
  take((size_t)(nb + 1) * 4);                     // block offsets
  take((size_t)std::max<int64_t>(n, 1) * 4);      // active list
  take((size_t)nqp * d * 4);                      // Q W_Q
  take((size_t)nblk * nqp * (2 + d) * 4);         // partials
  return b;
}

template <typename FT, int C, int D>
static void att_main(const AttentionArgs& a, int nqp, int nblk, char* const* p, hipStream_t st) {
  const float scale = 1.0f / sqrtf((float)D);
  const float inv_len = 1.0f / a.pos_length;
  const int qw = (int)cdiv(nqp / 16, 4);
#define PSM_ATT(QWV)                                                                                                   \
  hipLaunchKernelGGL((k_att_main<FT, C, D, QWV>), dim3(nblk), dim3(256), 0, st, (const uint32_t*)p[3],                \
                     (const uint32_t*)p[2] + a.nb, a.means, (const FT*)a.feat, a.wk, a.wv, (const float*)p[4], nqp,   \
                     inv_len, scale, nblk, (float*)p[5])
  if (qw <= 1) PSM_ATT(1);
  else if (qw <= 2) PSM_ATT(2);
  else PSM_ATT(4);
#undef PSM_ATT
}

template <typename FT>
static bool att_dispatch(const AttentionArgs& a, int nqp, int nblk, char* const* p, hipStream_t st) {
  if (a.c == 16 && a.d == 16) att_main<FT, 16, 16>(a, nqp, nblk, p, st);
  else if (a.c == 32 && a.d == 32) att_main<FT, 32, 32>(a, nqp, nblk, p, st);
  else if (a.c == 64 && a.d == 32) att_main<FT, 64, 32>(a, nqp, nblk, p, st);
  else if (a.c == 64 && a.d == 64) att_main<FT, 64, 64>(a, nqp, nblk, p, st);
  else return false;
  return true;
}

bool attention_supported(int c, int d) {
  return (c == 16 && d == 16) || (c == 32 && d == 32) || (c == 64 && d == 32) || (c == 64 && d == 64);
}

void launch_attention(const AttentionArgs& a, char* ws, float* out, uint8_t* active_out, hipStream_t st) {
  const int64_t nb = cdiv(std::max<int64_t>(a.n, 1), kAttCullBlock);
  const int nqp = (int)cdiv(a.nq, 16) * 16;
  char* p[6];
  size_t o = 0;
  auto take = [&](size_t bytes) { char* r = ws + o; o += (bytes + 255) & ~(size_t)255; return r; };
  p[0] = take((size_t)std::max<int64_t>(a.n, 1));
  p[1] = take((size_t)nb * 4);
  p[2] = take((size_t)(nb + 1) * 4);
  p[3] = take((size_t)std::max<int64_t>(a.n, 1) * 4);
  p[4] = take((size_t)nqp * a.d * 4);
  p[5] = take((size_t)a.nblk * nqp * (2 + a.d) * 4);
  uint8_t* act = active_out ? active_out : (uint8_t*)p[0];
  AttentionArgs b = a;
  b.nb = nb;
  if (a.n > 0) {
    hipLaunchKernelGGL(k_att_cull, dim3((unsigned)nb), dim3(kAttCullBlock), 0, st, a.n, a.means, a.scales, a.cam, act,
                       (uint32_t*)p[1]);
  } else {
    launch_fill_u32(p[1], 0u, 1, st);
  }
  hipLaunchKernelGGL(k_att_scan, dim3(1), dim3(1024), 0, st, nb, (const uint32_t*)p[1], (uint32_t*)p[2]);
  if (a.n > 0)
    hipLaunchKernelGGL(k_att_compact, dim3((unsigned)nb), dim3(kAttCullBlock), 0, st, a.n, (const uint8_t*)act,
                       (const uint32_t*)p[2], (uint32_t*)p[3]);
  hipLaunchKernelGGL(k_att_qproj, dim3((unsigned)cdiv((int64_t)nqp * a.d, 256)), dim3(256), 0, st, a.nq, nqp, a.c,
                     a.d, a.q, a.wq, (float*)p[4]);
  if (a.feat_dtype == kF16) att_dispatch<__half>(b, nqp, a.nblk, p, st);
  else if (a.feat_dtype == kBF16) att_dispatch<uint16_t>(b, nqp, a.nblk, p, st);
  else att_dispatch<float>(b, nqp, a.nblk, p, st);
  if (a.d == 16)
    hipLaunchKernelGGL(k_att_combine<16>, dim3(a.nq), dim3(256), 0, st, nqp, a.nblk, (const float*)p[5], out);
  else if (a.d == 32)
    hipLaunchKernelGGL(k_att_combine<32>, dim3(a.nq), dim3(256), 0, st, nqp, a.nblk, (const float*)p[5], out);
  else
    hipLaunchKernelGGL(k_att_combine<64>, dim3(a.nq), dim3(256), 0, st, nqp, a.nblk, (const float*)p[5], out);
}

}  // namespace psm
