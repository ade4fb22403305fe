// Key stage of the rasterizer (Sec. 5, Precise Tile Intersection):
//   preprocess  -- per surfel: rotation, camera space, culling, the projected
//                  cutoff ellipse, its footprint count, the walk record;
//   count scan  -- exclusive prefix of the counts in depth order;
//   emission    -- (tile id, surfel id) pairs, written in depth order;
//   tile ranges -- [start, end) of every tile in the tile-sorted pair list.
//
// Every floating-point decision here (cull, depth key, footprint) follows one
// prescribed sequence of IEEE FP32 operations: this translation unit is built
// with -ffp-contract=off and correctly rounded division and square root.
#include "common.h"
#include "internal.h"

#pragma clang fp contract(off)

namespace psm {

using Cam = CamArgs;

// Projected cutoff ellipse of a visible surfel; with the low-pass filter also
// the projected centre and the filter disk's radius^2 (rf2 = 0: no filter).
struct Foot {
  float ecx, ecy, S00, S01, S11, ex, ey, gam, kk;
  float xc, yc, rf2;
};

// Quantities of the prescribed FP32 key stage for one surfel.
struct Key {
  int cull;
  int flip;
  float mc2, p, q, xc, yc, A00, A01, A10, A11, dA;
  float nc[3];
  Foot f;
};

// Opacity-aware footprint radius^2 (an exact work reduction): a pixel is
// skipped when alpha = o exp(-rho/2) < 1/255 (Sec. 3.1), i.e. when
// rho > 2 ln(255 o), so a surfel's footprint only needs rho <= min(9,
// 2 ln(255 o)).  The bound gets a 2^-10 absolute and relative margin (the
// per-pixel FP32 alpha is within a few ulp of exact) and is rounded up to a
// multiple of 2^-12 in FP64, which is exact in FP32, so correctly rounded
// and faithful FP64 logarithms give the same value.
__device__ __forceinline__ float opacity_foot2(float o) {
  const double L = 2.0 * log(255.0 * (double)o);
  const double r = ceil((L + 0x1p-10) * (1.0 + 0x1p-10) * 4096.0) * (1.0 / 4096.0);
  return (float)fmin((double)kFoot2, fmax(r, 1.0 / 4096.0));
}

// foot2: footprint radius^2 (kFoot2, or the opacity-aware bound).  The cull
// decisions always use kFoot2, so both footprints keep the same visible set.
// lowpass: the footprint also takes the low-pass filter's disk.
__device__ __forceinline__ Key key_stage(const float* mu, const float* sc, const float* qq, const Cam& k, float foot2,
                                      int lowpass) {
  Key r;
  r.cull = 0;
  r.flip = 0;
  const float nq = ((qq[0] * qq[0] + qq[1] * qq[1]) + qq[2] * qq[2]) + qq[3] * qq[3];
  if (!(nq > 0.0f)) { r.cull = 1; return r; }
  const float rn = 1.0f / sqrtf(nq);
  const float w = qq[0] * rn, x = qq[1] * rn, y = qq[2] * rn, z = qq[3] * rn;
  const float xx = x * x, yy = y * y, zz = z * z;
  const float xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  const float tu0 = 1.0f - 2.0f * (yy + zz), tu1 = 2.0f * (xy + wz), tu2 = 2.0f * (xz - wy);
  const float tv0 = 2.0f * (xy - wz), tv1 = 1.0f - 2.0f * (xx + zz), tv2 = 2.0f * (yz + wx);
  const float nn0 = 2.0f * (xz + wy), nn1 = 2.0f * (yz - wx), nn2 = 1.0f - 2.0f * (xx + yy);
  float mc[3], a[3], b[3], rnv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float R0 = k.R[3 * i], R1 = k.R[3 * i + 1], R2 = k.R[3 * i + 2];
    mc[i] = ((R0 * mu[0] + R1 * mu[1]) + R2 * mu[2]) + k.t[i];
    const float ra = (R0 * tu0 + R1 * tu1) + R2 * tu2;
    const float rb = (R0 * tv0 + R1 * tv1) + R2 * tv2;
    rnv[i] = (R0 * nn0 + R1 * nn1) + R2 * nn2;
    a[i] = sc[0] * ra;
    b[i] = sc[1] * rb;
  }
  const float dn = (rnv[0] * mc[0] + rnv[1] * mc[1]) + rnv[2] * mc[2];
  r.flip = dn > 0.0f ? 1 : 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) r.nc[i] = r.flip ? -rnv[i] : rnv[i];
  if (!(mc[2] > k.near_plane)) { r.cull = 2; return r; }
  const float zmin = mc[2] - kCut * sqrtf(a[2] * a[2] + b[2] * b[2]);
  if (!(zmin > k.near_plane)) { r.cull = 3; return r; }
  const float iz = 1.0f / mc[2];
  const float p = a[2] * iz, q = b[2] * iz;
  const float g2 = p * p + q * q;
  const float gam = 1.0f - kFoot2 * g2;
  if (!(gam > 0.0f)) { r.cull = 3; return r; }
  const float mx = mc[0] * iz, my = mc[1] * iz;
  const float xc = k.fx * mx + k.cx, yc = k.fy * my + k.cy;
  const float A00 = k.fx * ((a[0] - mx * a[2]) * iz);
  const float A01 = k.fx * ((b[0] - mx * b[2]) * iz);
  const float A10 = k.fy * ((a[1] - my * a[2]) * iz);
  const float A11 = k.fy * ((b[1] - my * b[2]) * iz);
  const float dA = A00 * A11 - A01 * A10;
  if (!(fabsf(dA) > 0.0f)) { r.cull = 4; return r; }
  float cc = kFoot2 / gam;
  const float w0 = A00 * p + A01 * q, w1 = A10 * p + A11 * q;
  float S00 = cc * ((A00 * A00 + A01 * A01) + cc * (w0 * w0));
  float S01 = cc * ((A00 * A10 + A01 * A11) + cc * (w0 * w1));
  float S11 = cc * ((A10 * A10 + A11 * A11) + cc * (w1 * w1));
  if (!(S00 > 0.0f && S11 > 0.0f && S00 < 1e24f && S11 < 1e24f)) { r.cull = 4; return r; }
  float gf = gam;
  if (foot2 != kFoot2) {  // the same ellipse formulas at the smaller radius
    gf = 1.0f - foot2 * g2;
    cc = foot2 / gf;
    S00 = cc * ((A00 * A00 + A01 * A01) + cc * (w0 * w0));
    S01 = cc * ((A00 * A10 + A01 * A11) + cc * (w0 * w1));
    S11 = cc * ((A10 * A10 + A11 * A11) + cc * (w1 * w1));
  }
  r.mc2 = mc[2]; r.p = p; r.q = q; r.xc = xc; r.yc = yc;
  r.A00 = A00; r.A01 = A01; r.A10 = A10; r.A11 = A11; r.dA = dA;
  r.f.ecx = xc - cc * w0;
  r.f.ecy = yc - cc * w1;
  r.f.S00 = S00; r.f.S01 = S01; r.f.S11 = S11;
  r.f.ex = sqrtf(S00);
  r.f.ey = sqrtf(S11);
  r.f.gam = gf;
  r.f.kk = fabsf(cc * dA);
  r.f.xc = xc;
  r.f.yc = yc;
  r.f.rf2 = lowpass ? 0.5f * foot2 + kLpPad : 0.0f;
  return r;
}

// Walk record of a visible surfel (not part of any decision): the centred,
// depth-normalised homography's A^-1, e = (p, q) A^-1 and the projected centre,
// evaluated and kept in FP64 (the per-pixel solve is FP64 as well).
__device__ __forceinline__ void walk_record(const float* mu_f, const float* sc, const float* qf, float o,
                                         const float* rgb, const float* nc, const Cam& k, WalkRec* out) {
  const double q0 = qf[0], q1 = qf[1], q2 = qf[2], q3 = qf[3];
  const double rn = 1.0 / sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const double w = q0 * rn, x = q1 * rn, y = q2 * rn, z = q3 * rn;
  const double tu[3] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y)};
  const double tv[3] = {2.0 * (x * y - w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z + w * x)};
  double mc[3], a[3], b[3];
  for (int i = 0; i < 3; ++i) {
    const double R0 = k.R[3 * i], R1 = k.R[3 * i + 1], R2 = k.R[3 * i + 2];
    mc[i] = R0 * mu_f[0] + R1 * mu_f[1] + R2 * mu_f[2] + (double)k.t[i];
    a[i] = sc[0] * (R0 * tu[0] + R1 * tu[1] + R2 * tu[2]);
    b[i] = sc[1] * (R0 * tv[0] + R1 * tv[1] + R2 * tv[2]);
  }
  const double iz = 1.0 / mc[2];
  const double p = a[2] * iz, q = b[2] * iz, mx = mc[0] * iz, my = mc[1] * iz;
  const double xc = (double)k.fx * mx + (double)k.cx, yc = (double)k.fy * my + (double)k.cy;
  const double A00 = k.fx * (a[0] - mx * a[2]) * iz, A01 = k.fx * (b[0] - mx * b[2]) * iz;
  const double A10 = k.fy * (a[1] - my * a[2]) * iz, A11 = k.fy * (b[1] - my * b[2]) * iz;
  const double idA = 1.0 / (A00 * A11 - A01 * A10);
  const double i00 = A11 * idA, i01 = -A01 * idA, i10 = -A10 * idA, i11 = A00 * idA;
  const double e0 = p * i00 + q * i10, e1 = p * i01 + q * i11;
  WalkRec r;
  r.d0 = make_double2(i00, i01);
  r.d1 = make_double2(i10, i11);
  r.d2 = make_double2(e0, e1);
  r.d3 = make_double2(xc, yc);
  r.f0 = make_float4((float)mc[2], o, rgb[0], rgb[1]);
  r.f1 = make_float4(rgb[2], nc[0], nc[1], nc[2]);
  *out = r;
}

// Tiles whose pixel-centre hull [t*T + 0.5, min(t*T + T - 0.5, npix - 0.5)]
// meets [lo, hi] along one axis (T = the tile's size along it).
__device__ __forceinline__ bool tile_span(float lo, float hi, int npix, int T, int nt, int& t0, int& t1) {
  if (!(hi >= 0.5f) || !(lo <= (float)npix - 0.5f)) return false;
  float f0 = ceilf((lo - ((float)T - 0.5f)) / (float)T);
  float f1 = floorf((hi - 0.5f) / (float)T);
  f0 = fmaxf(f0, 0.0f);
  f1 = fminf(f1, (float)(nt - 1));
  if (!(f0 <= f1)) return false;
  t0 = (int)f0;
  t1 = (int)f1;
  return true;
}

// Calls fn(ty, tx0, tx1) for each tile row of the footprint of mode `mode`.
// With the low-pass filter the footprint is the union with the filter's disk:
// the disk's box joins every mode's box, and the exact mode takes, per row,
// the hull of the ellipse's and the disk's x-extents within the row's band.
template <class F>
__device__ __forceinline__ void for_each_row(const Foot& f, int mode, int W, int H, int tw, int th, int ntx, int nty,
                                             F&& fn) {
  const bool lp = f.rf2 > 0.0f;
  const float rf = lp ? sqrtf(f.rf2) : 0.0f;
  int ax0, ax1, ay0, ay1;
  float bx0, bx1, by0, by1;
  if (mode == kSphere) {
    const float hs = 0.5f * (f.S00 + f.S11);
    const float hd = 0.5f * (f.S00 - f.S11);
    const float lmax = hs + sqrtf(hd * hd + f.S01 * f.S01);
    const float rr = fmaxf(sqrtf(lmax), fmaxf(f.ex, f.ey));
    bx0 = f.ecx - rr;
    bx1 = f.ecx + rr;
    by0 = f.ecy - rr;
    by1 = f.ecy + rr;
  } else {
    bx0 = f.ecx - f.ex;
    bx1 = f.ecx + f.ex;
    by0 = f.ecy - f.ey;
    by1 = f.ecy + f.ey;
  }
  if (lp) {
    bx0 = fminf(bx0, f.xc - rf);
    bx1 = fmaxf(bx1, f.xc + rf);
    by0 = fminf(by0, f.yc - rf);
    by1 = fmaxf(by1, f.yc + rf);
  }
  if (!tile_span(bx0, bx1, W, tw, ntx, ax0, ax1)) return;
  if (!tile_span(by0, by1, H, th, nty, ay0, ay1)) return;
  if (mode != kEllipse) {
    for (int ty = ay0; ty <= ay1; ++ty) fn(ty, ax0, ax1);
    return;
  }
  // exact ellipse: x-extent of the ellipse inside each tile row's band
  const float yr = f.S01 / f.ex;
  for (int ty = ay0; ty <= ay1; ++ty) {
    const float rlo = (float)(ty * th) + 0.5f;
    const float rhi = fminf((float)(ty * th) + ((float)th - 0.5f), (float)H - 0.5f);
    const float ylo = rlo - f.ecy;
    const float yhi = rhi - f.ecy;
    const float lo = fmaxf(ylo, -f.ey), hi = fminf(yhi, f.ey);
    bool have = false;
    float xl = 0.0f, xr = 0.0f;
    if (lo <= hi) {
      const float dR = fminf(fmaxf(yr, lo), hi);
      const float dL = fminf(fmaxf(-yr, lo), hi);
      const float hR = sqrtf(fmaxf(0.0f, (f.S11 - dR * dR) / f.gam)) * f.kk;
      const float hL = sqrtf(fmaxf(0.0f, (f.S11 - dL * dL) / f.gam)) * f.kk;
      const float xR = (f.S01 * dR + hR) / f.S11;
      const float xL = (f.S01 * dL - hL) / f.S11;
      xl = f.ecx + xL;
      xr = f.ecx + xR;
      have = true;
    }
    if (lp) {  // the disk's widest chord within the band
      const float dlo = rlo - f.yc, dhi = rhi - f.yc;
      const float dy = fminf(fmaxf(0.0f, dlo), dhi);
      const float h2 = f.rf2 - dy * dy;
      if (h2 >= 0.0f) {
        const float h = sqrtf(h2);
        const float dl = f.xc - h, dr = f.xc + h;
        xl = have ? fminf(xl, dl) : dl;
        xr = have ? fmaxf(xr, dr) : dr;
        have = true;
      }
    }
    if (!have) continue;
    int x0, x1;
    if (!tile_span(xl, xr, W, tw, ntx, x0, x1)) continue;
    x0 = max(x0, ax0);
    x1 = min(x1, ax1);
    if (x0 <= x1) fn(ty, x0, x1);
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = i; j < count; j += stride) p[j] = v;
}

__global__ void k_init_status(uint32_t* __restrict__ st, uint32_t n, uint32_t tiles, uint64_t total, uint32_t cap) {
  const int i = threadIdx.x;
  uint32_t v = 0u;
  v = i == kStN ? n : v;
  v = i == kStTiles ? tiles : v;
  v = i == kStSigLo ? (uint32_t)total : v;
  v = i == kStSigHi ? (uint32_t)(total >> 32) : v;
  v = i == kStSigCap ? cap : v;
  v = i == kStSigTiles ? tiles : v;
  if (i < kStWords) st[i] = v;
}

// Thread per virtual surfel v = b * N + i (surfel i seen by camera b).
__global__ __launch_bounds__(256) void k_preprocess(
    int64_t nv, const float* __restrict__ means, const float* __restrict__ scales,
    const float* __restrict__ quats, const float* __restrict__ opacity, const float* __restrict__ rgb,
    CamTable ct, int mode, int opacity_foot, int lowpass, WalkRec* __restrict__ rec, float4* __restrict__ fp,
    float4* __restrict__ ext,
    uint32_t* __restrict__ key, uint32_t* __restrict__ ids, uint32_t* __restrict__ count,
    int32_t* __restrict__ cull, uint32_t* __restrict__ status) {
  __shared__ uint32_t s_cnt[5];
  __shared__ Cam s_cam[kMaxCams];  // cameras by constant index (no private copy of the table)
  if (threadIdx.x < 5) s_cnt[threadIdx.x] = 0;
#pragma unroll
  for (int b = 0; b < kMaxCams; ++b)
    if (threadIdx.x == b && b < ct.n) s_cam[b] = ct.cam[b];
  __syncthreads();
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nv) {
    const int b = camera_of(ct, v);
    const int64_t i = v - (int64_t)b * ct.nsurf;
    const Cam& cam = s_cam[b];
    const float foot2 = opacity_foot ? opacity_foot2(opacity[i]) : kFoot2;
    const Key kk = key_stage(means + 3 * i, scales + 2 * i, quats + 4 * i, cam, foot2, lowpass);
    ids[v] = (uint32_t)v;
    cull[v] = kk.cull | (kk.flip << 8);  // bit 8: normal flipped toward the camera
    atomicAdd(&s_cnt[kk.cull], 1u);
    if (kk.cull != 0) {
      key[v] = 0xFFFFFFFFu;
      count[v] = 0;
    } else {
      key[v] = __float_as_uint(kk.mc2);
      uint32_t c = 0;
      for_each_row(kk.f, mode, cam.W, cam.H, ct.tw, ct.th, ct.ntx[b], ct.nty[b],
                   [&](int, int x0, int x1) { c += (uint32_t)(x1 - x0 + 1); });
      count[v] = c;
      fp[3 * v + 0] = make_float4(kk.f.ecx, kk.f.ecy, kk.f.S00, kk.f.S01);
      fp[3 * v + 1] = make_float4(kk.f.S11, kk.f.ex, kk.f.ey, kk.f.gam);
      fp[3 * v + 2] = make_float4(kk.f.kk, kk.f.xc, kk.f.yc, kk.f.rf2);
      if (lowpass) {  // the walks' band culling sees the union's extent
        const float rf = sqrtf(kk.f.rf2);
        const float x0 = fminf(kk.f.ecx - kk.f.ex, kk.f.xc - rf), x1 = fmaxf(kk.f.ecx + kk.f.ex, kk.f.xc + rf);
        const float y0 = fminf(kk.f.ecy - kk.f.ey, kk.f.yc - rf), y1 = fmaxf(kk.f.ecy + kk.f.ey, kk.f.yc + rf);
        ext[v] = make_float4(0.5f * (x0 + x1), 0.5f * (y0 + y1), 0.5f * (x1 - x0), 0.5f * (y1 - y0));
      } else {
        ext[v] = make_float4(kk.f.ecx, kk.f.ecy, kk.f.ex, kk.f.ey);
      }
      walk_record(means + 3 * i, scales + 2 * i, quats + 4 * i, opacity[i], rgb + 3 * i, kk.nc, cam,
                  rec + v);
    }
  }
  __syncthreads();
  if (threadIdx.x < 5 && s_cnt[threadIdx.x]) atomicAdd(&status[kStCull + threadIdx.x], s_cnt[threadIdx.x]);
  if (threadIdx.x == 0 && s_cnt[0]) atomicAdd(&status[kStVisible], s_cnt[0]);
}

// ---- exclusive scan of the pair counts, gathered in depth order ------------
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(int64_t n, const uint32_t* __restrict__ order,
                                                             const uint32_t* __restrict__ count,
                                                             uint64_t* __restrict__ bsum) {
  __shared__ uint64_t s[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint64_t acc = 0;
#pragma unroll 4
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t r = base + (int64_t)j * kScanThreads + threadIdx.x;
    if (r < n) acc += count[order[r]];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kScanThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

// One block: exclusive scan of the block sums, total -> status.
__global__ __launch_bounds__(1024) void k_scan_top(int64_t nb, uint64_t* __restrict__ bsum, int64_t cap,
                                                   uint32_t* __restrict__ status) {
  __shared__ uint64_t s[1024];
  const int t = threadIdx.x;
  const int64_t per = cdiv(nb, 1024);
  const int64_t b0 = t * per, b1 = min<int64_t>(nb, b0 + per);
  uint64_t acc = 0;
  for (int64_t b = b0; b < b1; ++b) acc += bsum[b];
  s[t] = acc;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    uint64_t v = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  uint64_t run = s[t] - acc;
  for (int64_t b = b0; b < b1; ++b) {
    const uint64_t v = bsum[b];
    bsum[b] = run;
    run += v;
  }
  if (t == 1023) {
    const uint64_t total = s[1023];
    status[kStReqLo] = (uint32_t)total;
    status[kStReqHi] = (uint32_t)(total >> 32);
    status[kStP] = (uint32_t)(total < (uint64_t)cap ? total : (uint64_t)cap);
    status[kStOverflow] = total > (uint64_t)cap ? 1u : 0u;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(int64_t n, const uint32_t* __restrict__ order,
                                                           const uint32_t* __restrict__ count,
                                                           const uint64_t* __restrict__ bsum,
                                                           uint32_t* __restrict__ offs) {
  __shared__ uint64_t s[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint64_t acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t r = base + j;
    v[j] = r < n ? count[order[r]] : 0u;
    acc += v[j];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    uint64_t x = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += x;
    __syncthreads();
  }
  uint64_t run = bsum[blockIdx.x] + s[threadIdx.x] - acc;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t r = base + j;
    if (r < n) offs[r] = (uint32_t)run;
    run += v[j];
  }
}

// ---- pair emission in depth order --------------------------------------------
// Thread per depth rank r: the pairs of virtual surfel v = order[r] go to
// [offs[r], offs[r] + count[v]), tile rows in order; vbase[v] = offs[r].
__global__ __launch_bounds__(256) void k_emit(int64_t nv, const uint32_t* __restrict__ order,
                                              const uint32_t* __restrict__ count,
                                              const uint32_t* __restrict__ offs, const float4* __restrict__ fp,
                                              CamTable ct, int mode, int64_t cap, uint32_t* __restrict__ vbase,
                                              uint32_t* __restrict__ ptile, uint32_t* __restrict__ eid,
                                              uint32_t* __restrict__ sid_emit) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nv) return;
  const uint32_t v = order[r];
  vbase[v] = offs[r];
  if (count[v] == 0) return;
  const int b = camera_of(ct, v);
  const int ntx = ct.ntx[b], t0 = ct.tile0[b];
  const float4 f0 = fp[3 * (size_t)v], f1 = fp[3 * (size_t)v + 1], f2 = fp[3 * (size_t)v + 2];
  const Foot f{f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w, f2.x, f2.y, f2.z, f2.w};
  int64_t o = offs[r];
  for_each_row(f, mode, ct.cam[b].W, ct.cam[b].H, ct.tw, ct.th, ntx, ct.nty[b], [&](int ty, int x0, int x1) {
    for (int tx = x0; tx <= x1; ++tx, ++o) {
      if (o < cap) {
        ptile[o] = (uint32_t)(t0 + ty * ntx + tx);
        eid[o] = (uint32_t)o;
        sid_emit[o] = v;
      }
    }
  });
}

// Per-surfel key-stage results in surfel order (inspection / tests).
__global__ __launch_bounds__(256) void k_export_keys(int64_t n, const int32_t* __restrict__ cull,
                                                     const uint32_t* __restrict__ skey,
                                                     const uint32_t* __restrict__ sid,
                                                     const uint32_t* __restrict__ count, int32_t* __restrict__ o_cull,
                                                     uint32_t* __restrict__ o_depth, int32_t* __restrict__ o_count) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  if (o_cull) o_cull[r] = cull[r] & 0xFF;
  if (o_count) o_count[r] = (int32_t)count[r];
  if (o_depth) {
    const uint32_t i = sid[r];  // depth-sorted rank r holds surfel i
    o_depth[i] = cull[i] & 0xFF ? 0u : skey[r];
  }
}

// After the tile sort: surfel id of each sorted pair and the tile ranges.  The
// sorted values keep each pair's emission index, where the backward writes the
// pair's partial sums.
__global__ __launch_bounds__(256) void k_finalize_pairs(const uint32_t* __restrict__ ptile,
                                                        const uint32_t* __restrict__ eid,
                                                        const uint32_t* __restrict__ sid_emit,
                                                        const uint32_t* __restrict__ status, uint32_t* __restrict__ pid,
                                                        uint2* __restrict__ ranges) {
  const uint32_t P = status[kStP];
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P) return;
  pid[j] = sid_emit[eid[j]];
  const uint32_t t = ptile[j];
  if (j == 0 || ptile[j - 1] != t) ranges[t].x = j;
  if (j == P - 1 || ptile[j + 1] != t) ranges[t].y = j + 1;
}

// Tile work order for the persistent scheduler, longest lists first: tiles
// binned by the bit length of their list length (one block), the bins taken
// in descending order.  The order within a bin does not matter: it only
// decides which block starts a tile, never a result.
__global__ __launch_bounds__(1024) void k_tile_order(int64_t tiles, const uint2* __restrict__ ranges,
                                                     uint32_t* __restrict__ order) {
  __shared__ uint32_t s_cnt[33], s_off[33];
  const int tid = threadIdx.x;
  if (tid < 33) s_cnt[tid] = 0u;
  __syncthreads();
  for (int64_t t = tid; t < tiles; t += 1024) {
    const uint2 r = ranges[t];
    const uint32_t len = r.y - r.x;
    atomicAdd(&s_cnt[len ? 32 - __clz(len) : 0], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int bin = 32; bin >= 0; --bin) {
      s_off[bin] = run;
      run += s_cnt[bin];
    }
  }
  __syncthreads();
  for (int64_t t = tid; t < tiles; t += 1024) {
    const uint2 r = ranges[t];
    const uint32_t len = r.y - r.x;
    order[atomicAdd(&s_off[len ? 32 - __clz(len) : 0], 1u)] = (uint32_t)t;
  }
}

// ------------------------------------------------------------- host wrappers
void launch_fill_u32(void* p, uint32_t v, int64_t count, hipStream_t st) {
  if (count <= 0) return;
  const int64_t blocks = std::min<int64_t>(cdiv(count, 256), 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t*)p, v, count);
}

void launch_init_status(uint32_t* status, const Layout& L, hipStream_t st) {
  static_assert(kStWords <= 64, "status words are written by one wave");
  hipLaunchKernelGGL(k_init_status, dim3(1), dim3(64), 0, st, status, (uint32_t)L.n, (uint32_t)L.tiles,
                     (uint64_t)L.total, (uint32_t)L.cap);
}

void launch_preprocess(const SurfelArgs& s, const CamTable& ct, int mode, bool opacity_foot, bool lowpass,
                       const Layout& L, char* ws, hipStream_t st) {
  if (L.n == 0) return;
  hipLaunchKernelGGL(k_preprocess, dim3((unsigned)cdiv(L.n, 256)), dim3(256), 0, st, L.n, s.means, s.scales,
                     s.quats, s.opacity, s.rgb, ct, mode, opacity_foot ? 1 : 0, lowpass ? 1 : 0, (WalkRec*)(ws + L.rec),
                     (float4*)(ws + L.fp),
                     (float4*)(ws + L.ext),
                     (uint32_t*)(ws + L.key0), (uint32_t*)(ws + L.id0), (uint32_t*)(ws + L.count),
                     (int32_t*)(ws + L.cull), (uint32_t*)(ws + L.status));
}

void launch_scan_counts(const Layout& L, char* ws, hipStream_t st) {
  const int64_t nb = std::max<int64_t>(cdiv(L.n, kScanTile), 1);
  const uint32_t* order = (const uint32_t*)(ws + L.id0);
  const uint32_t* count = (const uint32_t*)(ws + L.count);
  uint64_t* bsum = (uint64_t*)(ws + L.bsum);
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, L.n, order, count, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, nb, bsum, L.cap, (uint32_t*)(ws + L.status));
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, st, L.n, order, count,
                     (const uint64_t*)bsum, (uint32_t*)(ws + L.offs));
}

void launch_emit(const CamTable& ct, int mode, const Layout& L, char* ws, hipStream_t st) {
  if (L.n == 0) return;
  hipLaunchKernelGGL(k_emit, dim3((unsigned)cdiv(L.n, 256)), dim3(256), 0, st, L.n,
                     (const uint32_t*)(ws + L.id0), (const uint32_t*)(ws + L.count),
                     (const uint32_t*)(ws + L.offs), (const float4*)(ws + L.fp), ct, mode, L.cap,
                     (uint32_t*)(ws + L.vbase), (uint32_t*)(ws + L.ptile0), (uint32_t*)(ws + L.eid0),
                     (uint32_t*)(ws + L.sid_emit));
}

void launch_export_keys(const Layout& L, char* ws, int32_t* cull, uint32_t* depth, int32_t* count, hipStream_t st) {
  if (L.n == 0 || (!cull && !depth && !count)) return;
  hipLaunchKernelGGL(k_export_keys, dim3((unsigned)cdiv(L.n, 256)), dim3(256), 0, st, L.n,
                     (const int32_t*)(ws + L.cull), (const uint32_t*)(ws + L.key0), (const uint32_t*)(ws + L.id0),
                     (const uint32_t*)(ws + L.count), cull, depth, count);
}

void launch_ranges(const Layout& L, char* ws, hipStream_t st) {
  if (L.cap == 0) return;
  hipLaunchKernelGGL(k_finalize_pairs, dim3((unsigned)cdiv(L.cap, 256)), dim3(256), 0, st,
                     (const uint32_t*)(ws + L.ptile0), (const uint32_t*)(ws + L.eid0),
                     (const uint32_t*)(ws + L.sid_emit), (const uint32_t*)(ws + L.status), (uint32_t*)(ws + L.pid),
                     (uint2*)(ws + L.ranges));
}

void launch_tile_order(const Layout& L, char* ws, hipStream_t st) {
  if (L.tiles == 0) return;
  hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, st, L.tiles, (const uint2*)(ws + L.ranges),
                     (uint32_t*)(ws + L.torder0));
}

}  // namespace psm
