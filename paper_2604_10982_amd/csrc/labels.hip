// Instance labels of surfels from localized queries (Sec. 4.1, eqs. (4)-(7)):
//   z = f_q . f_g,  S = sigmoid(z),  D = exp(-(p_g - mu_q)^T P_q (p_g - mu_q) / 2),
//   A = S D,  l(g) = softmax over queries of A(., g),
// and their gradients.  The labels are rendered by the feature blend (eq. (8)).
//
// The affinity logits are a dense contraction over the feature dimension
// (surfels x queries), so they run on the matrix cores: FP32 MFMA
// (v_mfma_f32_16x16x4f32, exact products, FP32 accumulation).  A wave owns 16
// surfels; lane l holds A-operand row l & 15 / k-slice l >> 4, and the
// 16 x 16 result tile lands as rows 4 (l >> 4) + r, column l & 15, so each
// 16-lane DPP row holds 4 surfels x 16 queries and the softmax over queries
// is a reduction inside DPP rows.
//
// Backward: k_lab_bwd_surf recomputes the forward and writes dz = dL/dz and
// wD = dL/dD * D per (surfel, query) plus dL/dp_g; the feature gradients are
// two MFMA products (dF_g = dZ F_q, dF_q = dZ^T F_g over surfel segments) and
// the query means/precisions are reduced over surfel segments (FP64), then
// the segments are summed in a fixed order: deterministic.
#include "common.h"
#include "internal.h"

namespace psm {

// Reductions over the 16 lanes of a DPP row (rotations inside the row).
__device__ __forceinline__ float row_sum16(float v) {
  v += dpp_mov<0x128>(v);  // row_ror:8
  v += dpp_mov<0x124>(v);  // row_ror:4
  v += dpp_mov<0x122>(v);  // row_ror:2
  v += dpp_mov<0x121>(v);  // row_ror:1
  return v;
}
__device__ __forceinline__ float row_max16(float v) {
  v = fmaxf(v, dpp_mov<0x128>(v));
  v = fmaxf(v, dpp_mov<0x124>(v));
  v = fmaxf(v, dpp_mov<0x122>(v));
  v = fmaxf(v, dpp_mov<0x121>(v));
  return v;
}

// Query j's mean and precision (xx, xy, xz, yy, yz, zz).
struct QGeo {
  float mx, my, mz, pxx, pxy, pxz, pyy, pyz, pzz;
};
__device__ __forceinline__ QGeo load_qgeo(const LabelQueries& q, int j) {
  QGeo g;
  const float* m = q.mean + 3 * j;
  const float* p = q.prec + 6 * j;
  g.mx = m[0]; g.my = m[1]; g.mz = m[2];
  g.pxx = p[0]; g.pxy = p[1]; g.pxz = p[2]; g.pyy = p[3]; g.pyz = p[4]; g.pzz = p[5];
  return g;
}

// Forward terms of one (surfel, query) element.
struct LabTerm {
  float S, D, dx, dy, dz, Px, Py, Pz;  // S, D, d = p - mu, P d
};
__device__ __forceinline__ LabTerm lab_term(float z, float px, float py, float pz, const QGeo& g) {
  LabTerm t;
  t.S = 1.0f / (1.0f + expf(-z));
  t.dx = px - g.mx;
  t.dy = py - g.my;
  t.dz = pz - g.mz;
  t.Px = g.pxx * t.dx + g.pxy * t.dy + g.pxz * t.dz;
  t.Py = g.pxy * t.dx + g.pyy * t.dy + g.pyz * t.dz;
  t.Pz = g.pxz * t.dx + g.pyz * t.dy + g.pzz * t.dz;
  const float m = t.dx * t.Px + t.dy * t.Py + t.dz * t.Pz;
  t.D = expf(-0.5f * m);
  return t;
}

// z tiles of a wave's 16 surfels against all query blocks (MFMA over C).
template <typename FT, int NQB>
__device__ __forceinline__ void logits(int64_t n, const FT* __restrict__ fg, const LabelQueries& q, int64_t g0,
                                       f4v (&acc)[NQB]) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
  const int64_t ga = g0 + i;
#pragma unroll
  for (int qb = 0; qb < NQB; ++qb) acc[qb] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int c0 = 0; c0 < q.c; c0 += 4) {
    const float a = ga < n ? load_one<FT>(fg + ga * q.c + c0 + kq) : 0.0f;
#pragma unroll
    for (int qb = 0; qb < NQB; ++qb) {
      const int j = qb * 16 + i;
      const float b = j < q.nq ? q.feat[(size_t)j * q.c + c0 + kq] : 0.0f;
      acc[qb] = mfma_16x16x4(a, b, acc[qb]);
    }
  }
}

template <typename FT, int NQB>
__global__ __launch_bounds__(256) void k_lab_fwd(int64_t n, const float* __restrict__ means, const FT* __restrict__ fg,
                                                 LabelQueries q, float* __restrict__ out, int ld) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, i = lane & 15, kq = lane >> 4;
  const int64_t g0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (g0 >= n) return;
  f4v acc[NQB];
  logits<FT, NQB>(n, fg, q, g0, acc);
  float px[4], py[4], pz[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t g = g0 + 4 * kq + r;
    px[r] = g < n ? means[3 * g] : 0.0f;
    py[r] = g < n ? means[3 * g + 1] : 0.0f;
    pz[r] = g < n ? means[3 * g + 2] : 0.0f;
  }
  float A[NQB][4], mx[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) mx[r] = -INFINITY;
#pragma unroll
  for (int qb = 0; qb < NQB; ++qb) {
    const int j = qb * 16 + i;
    const bool vq = j < q.nq;
    const QGeo gq = load_qgeo(q, vq ? j : 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const LabTerm t = lab_term(acc[qb][r], px[r], py[r], pz[r], gq);
      A[qb][r] = vq ? t.S * t.D : -INFINITY;
      mx[r] = fmaxf(mx[r], A[qb][r]);
    }
  }
  float sum[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    mx[r] = row_max16(mx[r]);
    sum[r] = 0.0f;
  }
#pragma unroll
  for (int qb = 0; qb < NQB; ++qb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float e = qb * 16 + i < q.nq ? expf(A[qb][r] - mx[r]) : 0.0f;
      A[qb][r] = e;
      sum[r] += e;
    }
  const int npad = (q.nq + 7) & ~7;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float inv = 1.0f / row_sum16(sum[r]);
    const int64_t g = g0 + 4 * kq + r;
    if (g >= n) continue;
#pragma unroll
    for (int qb = 0; qb < NQB; ++qb) {
      const int j = qb * 16 + i;
      if (j < npad) out[g * ld + j] = j < q.nq ? A[qb][r] * inv : 0.0f;
    }
  }
}

// Backward per (surfel, query): dz = dL/dz, wD = dL/dD * D (into padded
// [n][16 NQB] arrays) and dL/dp_g.
template <typename FT, int NQB>
__global__ __launch_bounds__(256) void k_lab_bwd_surf(int64_t n, const float* __restrict__ means,
                                                      const FT* __restrict__ fg, LabelQueries q,
                                                      const float* __restrict__ dl, int ld, float* __restrict__ dZ,
                                                      float* __restrict__ wDo, float* __restrict__ d_means) {
  constexpr int NQP = NQB * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, i = lane & 15, kq = lane >> 4;
  const int64_t g0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (g0 >= n) return;
  f4v acc[NQB];
  logits<FT, NQB>(n, fg, q, g0, acc);
  float px[4], py[4], pz[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t g = g0 + 4 * kq + r;
    px[r] = g < n ? means[3 * g] : 0.0f;
    py[r] = g < n ? means[3 * g + 1] : 0.0f;
    pz[r] = g < n ? means[3 * g + 2] : 0.0f;
  }
  // forward again: A, softmax
  float A[NQB][4], mx[4], sum[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) mx[r] = -INFINITY;
#pragma unroll
  for (int qb = 0; qb < NQB; ++qb) {
    const int j = qb * 16 + i;
    const bool vq = j < q.nq;
    const QGeo gq = load_qgeo(q, vq ? j : 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const LabTerm t = lab_term(acc[qb][r], px[r], py[r], pz[r], gq);
      A[qb][r] = vq ? t.S * t.D : -INFINITY;
      mx[r] = fmaxf(mx[r], A[qb][r]);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    mx[r] = row_max16(mx[r]);
    sum[r] = 0.0f;
  }
#pragma unroll
  for (int qb = 0; qb < NQB; ++qb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float e = qb * 16 + i < q.nq ? expf(A[qb][r] - mx[r]) : 0.0f;
      A[qb][r] = e;
      sum[r] += e;
    }
  // labels and sum_q l dl per surfel
  float dot[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float inv = 1.0f / row_sum16(sum[r]);
    const int64_t g = g0 + 4 * kq + r;
    dot[r] = 0.0f;
#pragma unroll
    for (int qb = 0; qb < NQB; ++qb) {
      const int j = qb * 16 + i;
      A[qb][r] *= inv;  // label
      const float u = (g < n && j < q.nq) ? dl[g * ld + j] : 0.0f;
      dot[r] = fmaf(A[qb][r], u, dot[r]);
    }
    dot[r] = row_sum16(dot[r]);
  }
  float gx[4] = {0.f, 0.f, 0.f, 0.f}, gy[4] = {0.f, 0.f, 0.f, 0.f}, gz[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int qb = 0; qb < NQB; ++qb) {
    const int j = qb * 16 + i;
    const bool vq = j < q.nq;
    const QGeo gq = load_qgeo(q, vq ? j : 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t g = g0 + 4 * kq + r;
      const LabTerm t = lab_term(acc[qb][r], px[r], py[r], pz[r], gq);
      const float u = (g < n && vq) ? dl[g * ld + j] : 0.0f;
      const float dA = A[qb][r] * (u - dot[r]);
      const float dz = vq ? dA * t.D * t.S * (1.0f - t.S) : 0.0f;
      const float wD = vq ? dA * t.S * t.D : 0.0f;
      gx[r] = fmaf(-wD, t.Px, gx[r]);
      gy[r] = fmaf(-wD, t.Py, gy[r]);
      gz[r] = fmaf(-wD, t.Pz, gz[r]);
      if (g < n) {
        dZ[g * NQP + j] = dz;
        wDo[g * NQP + j] = wD;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float sx = row_sum16(gx[r]), sy = row_sum16(gy[r]), sz = row_sum16(gz[r]);
    const int64_t g = g0 + 4 * kq + r;
    if (i == 0 && g < n) {
      d_means[3 * g] = sx;
      d_means[3 * g + 1] = sy;
      d_means[3 * g + 2] = sz;
    }
  }
}

// dF_g = dZ F_q: a wave computes 16 surfels x 16 channels (MFMA over queries).
template <int NQB>
__global__ __launch_bounds__(256) void k_lab_dfg(int64_t n, LabelQueries q, const float* __restrict__ dZ,
                                                 float* __restrict__ dfg) {
  constexpr int NQP = NQB * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, i = lane & 15, k = lane >> 4;
  const int64_t g0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  const int c0 = blockIdx.y * 16;
  if (g0 >= n) return;
  f4v acc = {0.f, 0.f, 0.f, 0.f};
  const int64_t ga = g0 + i;
  for (int j0 = 0; j0 < NQP; j0 += 4) {
    const float a = ga < n ? dZ[ga * NQP + j0 + k] : 0.0f;
    const bool vb = j0 + k < q.nq && c0 + i < q.c;
    const float b = vb ? q.feat[(size_t)(j0 + k) * q.c + c0 + i] : 0.0f;
    acc = mfma_16x16x4(a, b, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t g = g0 + 4 * k + r;
    if (g < n && c0 + i < q.c) dfg[g * q.c + c0 + i] = acc[r];
  }
}

// Partial dF_q = dZ^T F_g over one surfel segment: a wave computes 16 queries x
// 16 channels (MFMA over the segment's surfels).
template <typename FT, int NQB>
__global__ __launch_bounds__(64) void k_lab_dfq(int64_t n, int64_t seg_len, LabelQueries q,
                                                const float* __restrict__ dZ, const FT* __restrict__ fg,
                                                float* __restrict__ part) {
  constexpr int NQP = NQB * 16;
  const int lane = threadIdx.x & 63, i = lane & 15, k = lane >> 4;
  const int j0 = blockIdx.x * 16, c0 = blockIdx.y * 16, s = blockIdx.z;
  const int64_t gs = (int64_t)s * seg_len, ge = min(n, gs + seg_len);
  f4v acc = {0.f, 0.f, 0.f, 0.f};
  for (int64_t g = gs; g < ge; g += 4) {
    const int64_t gk = g + k;
    const float a = gk < ge ? dZ[gk * NQP + j0 + i] : 0.0f;
    const float b = (gk < ge && c0 + i < q.c) ? load_one<FT>(fg + gk * q.c + c0 + i) : 0.0f;
    acc = mfma_16x16x4(a, b, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int j = j0 + 4 * k + r;
    if (c0 + i < q.c) part[((size_t)s * NQP + j) * q.c + c0 + i] = acc[r];
  }
}

// Partial query-mean / precision gradients over one surfel segment (FP64
// accumulation, fixed-order block reduction).
template <int NQB>
__global__ __launch_bounds__(256) void k_lab_qgeo(int64_t n, int64_t seg_len, const float* __restrict__ means,
                                                  LabelQueries q, const float* __restrict__ wD,
                                                  double* __restrict__ part) {
  constexpr int NQP = NQB * 16;
  __shared__ double s_red[256];
  const int j = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int64_t gs = (int64_t)s * seg_len, ge = min(n, gs + seg_len);
  const QGeo gq = load_qgeo(q, j);
  double v[9];
#pragma unroll
  for (int x = 0; x < 9; ++x) v[x] = 0.0;
  for (int64_t g = gs + tid; g < ge; g += 256) {
    const double w = wD[g * NQP + j];
    const double dx = (double)means[3 * g] - gq.mx, dy = (double)means[3 * g + 1] - gq.my,
                 dz = (double)means[3 * g + 2] - gq.mz;
    const double Px = gq.pxx * dx + gq.pxy * dy + gq.pxz * dz;
    const double Py = gq.pxy * dx + gq.pyy * dy + gq.pyz * dz;
    const double Pz = gq.pxz * dx + gq.pyz * dy + gq.pzz * dz;
    v[0] += w * Px;
    v[1] += w * Py;
    v[2] += w * Pz;
    // dL/dP = -wD/2 d d^T; an off-diagonal number appears twice in P
    v[3] += -0.5 * w * dx * dx;
    v[4] += -w * dx * dy;
    v[5] += -w * dx * dz;
    v[6] += -0.5 * w * dy * dy;
    v[7] += -w * dy * dz;
    v[8] += -0.5 * w * dz * dz;
  }
  for (int x = 0; x < 9; ++x) {
    s_red[tid] = v[x];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) s_red[tid] += s_red[tid + o];
      __syncthreads();
    }
    if (tid == 0) part[((size_t)s * NQP + j) * 9 + x] = s_red[0];
    __syncthreads();
  }
}

// Sum of the segment partials in segment order.
__global__ __launch_bounds__(256) void k_lab_sum(int nseg, int nq, int nqp, int c, const float* __restrict__ pfq,
                                                 const double* __restrict__ pgeo, float* __restrict__ d_qfeat,
                                                 float* __restrict__ d_qmean, float* __restrict__ d_qprec) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nf = (int64_t)nq * c;
  if (t < nf) {
    const int j = (int)(t / c), cc = (int)(t % c);
    double a = 0.0;
    for (int s = 0; s < nseg; ++s) a += pfq[((size_t)s * nqp + j) * c + cc];
    d_qfeat[t] = (float)a;
  } else if (t < nf + (int64_t)nq * 9) {
    const int64_t u = t - nf;
    const int j = (int)(u / 9), x = (int)(u % 9);
    double a = 0.0;
    for (int s = 0; s < nseg; ++s) a += pgeo[((size_t)s * nqp + j) * 9 + x];
    if (x < 3) d_qmean[3 * j + x] = (float)a;
    else d_qprec[6 * j + (x - 3)] = (float)a;
  }
}

// ------------------------------------------------------------- host wrappers
int label_blocks16(int nq) { return pow2_ge_host((nq + 15) / 16); }

size_t label_workspace_bytes(int64_t n, int nq, int c) {
  const int64_t nqp = (int64_t)label_blocks16(nq) * 16;
  const int64_t nseg = label_segments(n);
  size_t o = 0;
  o = align256(o + (size_t)std::max<int64_t>(n, 1) * nqp * 4);  // dZ
  o = align256(o + (size_t)std::max<int64_t>(n, 1) * nqp * 4);  // wD
  o = align256(o + (size_t)nseg * nqp * c * 4);                  // dF_q partials
  o = align256(o + (size_t)nseg * nqp * 9 * 8);                  // mean / precision partials
  return o;
}

int64_t label_segments(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>(256, cdiv(n, 1024))); }

template <typename FT, int NQB>
static void lab_fwd_t(int64_t n, const float* means, const void* fg, const LabelQueries& q, float* out, int ld,
                      hipStream_t st) {
  hipLaunchKernelGGL((k_lab_fwd<FT, NQB>), dim3((unsigned)cdiv(n, 64)), dim3(256), 0, st, n, means, (const FT*)fg, q,
                     out, ld);
}

template <typename FT, int NQB>
static void lab_bwd_t(int64_t n, const float* means, const void* fg, const LabelQueries& q, const float* dl, int ld,
                      char* ws, float* d_means, float* d_fg, float* d_qfeat, float* d_qmean, float* d_qprec,
                      hipStream_t st) {
  constexpr int NQP = NQB * 16;
  const int64_t nseg = label_segments(n);
  const int64_t seg_len = cdiv(std::max<int64_t>(n, 1), nseg);
  size_t o = 0;
  float* dZ = (float*)(ws + o);
  o = align256(o + (size_t)std::max<int64_t>(n, 1) * NQP * 4);
  float* wD = (float*)(ws + o);
  o = align256(o + (size_t)std::max<int64_t>(n, 1) * NQP * 4);
  float* pfq = (float*)(ws + o);
  o = align256(o + (size_t)nseg * NQP * q.c * 4);
  double* pgeo = (double*)(ws + o);
  if (n > 0) {
    const unsigned nb = (unsigned)cdiv(n, 64);
    hipLaunchKernelGGL((k_lab_bwd_surf<FT, NQB>), dim3(nb), dim3(256), 0, st, n, means, (const FT*)fg, q, dl, ld, dZ,
                       wD, d_means);
    hipLaunchKernelGGL((k_lab_dfg<NQB>), dim3(nb, (unsigned)cdiv(q.c, 16)), dim3(256), 0, st, n, q, (const float*)dZ,
                       d_fg);
  }
  hipLaunchKernelGGL((k_lab_dfq<FT, NQB>), dim3(NQB, (unsigned)cdiv(q.c, 16), (unsigned)nseg), dim3(64), 0, st, n,
                     seg_len, q, (const float*)dZ, (const FT*)fg, pfq);
  hipLaunchKernelGGL((k_lab_qgeo<NQB>), dim3((unsigned)q.nq, (unsigned)nseg), dim3(256), 0, st, n, seg_len, means, q,
                     (const float*)wD, pgeo);
  const int64_t tot = (int64_t)q.nq * (q.c + 9);
  hipLaunchKernelGGL(k_lab_sum, dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, st, (int)nseg, q.nq, NQP, q.c,
                     (const float*)pfq, (const double*)pgeo, d_qfeat, d_qmean, d_qprec);
}

template <typename FT>
static void lab_fwd_dt(int64_t n, const float* means, const void* fg, const LabelQueries& q, float* out, int ld,
                       hipStream_t st) {
  switch (label_blocks16(q.nq)) {
    case 1: lab_fwd_t<FT, 1>(n, means, fg, q, out, ld, st); break;
    case 2: lab_fwd_t<FT, 2>(n, means, fg, q, out, ld, st); break;
    case 4: lab_fwd_t<FT, 4>(n, means, fg, q, out, ld, st); break;
    case 8: lab_fwd_t<FT, 8>(n, means, fg, q, out, ld, st); break;
    default: lab_fwd_t<FT, 16>(n, means, fg, q, out, ld, st); break;
  }
}

template <typename FT>
static void lab_bwd_dt(int64_t n, const float* means, const void* fg, const LabelQueries& q, const float* dl, int ld,
                       char* ws, float* d_means, float* d_fg, float* d_qfeat, float* d_qmean, float* d_qprec,
                       hipStream_t st) {
  switch (label_blocks16(q.nq)) {
    case 1: lab_bwd_t<FT, 1>(n, means, fg, q, dl, ld, ws, d_means, d_fg, d_qfeat, d_qmean, d_qprec, st); break;
    case 2: lab_bwd_t<FT, 2>(n, means, fg, q, dl, ld, ws, d_means, d_fg, d_qfeat, d_qmean, d_qprec, st); break;
    case 4: lab_bwd_t<FT, 4>(n, means, fg, q, dl, ld, ws, d_means, d_fg, d_qfeat, d_qmean, d_qprec, st); break;
    case 8: lab_bwd_t<FT, 8>(n, means, fg, q, dl, ld, ws, d_means, d_fg, d_qfeat, d_qmean, d_qprec, st); break;
    default: lab_bwd_t<FT, 16>(n, means, fg, q, dl, ld, ws, d_means, d_fg, d_qfeat, d_qmean, d_qprec, st); break;
  }
}

void launch_labels(int64_t n, const float* means, const void* fg, int dtype, const LabelQueries& q, float* out,
                   int ld, hipStream_t st) {
  if (n == 0) return;
  if (dtype == kF32) lab_fwd_dt<float>(n, means, fg, q, out, ld, st);
  else if (dtype == kF16) lab_fwd_dt<__half>(n, means, fg, q, out, ld, st);
  else lab_fwd_dt<uint16_t>(n, means, fg, q, out, ld, st);
}

void launch_labels_backward(int64_t n, const float* means, const void* fg, int dtype, const LabelQueries& q,
                            const float* dl, int ld, char* ws, float* d_means, float* d_fg, float* d_qfeat,
                            float* d_qmean, float* d_qprec, hipStream_t st) {
  if (dtype == kF32) lab_bwd_dt<float>(n, means, fg, q, dl, ld, ws, d_means, d_fg, d_qfeat, d_qmean, d_qprec, st);
  else if (dtype == kF16) lab_bwd_dt<__half>(n, means, fg, q, dl, ld, ws, d_means, d_fg, d_qfeat, d_qmean, d_qprec, st);
  else lab_bwd_dt<uint16_t>(n, means, fg, q, dl, ld, ws, d_means, d_fg, d_qfeat, d_qmean, d_qprec, st);
}

}  // namespace psm
