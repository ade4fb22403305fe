// Shared definitions of the gfx950 rasterizer: constants, workspace layout,
// the per-surfel walk record and the per-pixel ray/surfel evaluation used by
// both the forward and the backward walk (so both take identical decisions).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psm {

// ----------------------------------------------------------------- constants
// Cutoff r = 3 in tangent units ("3 sigma", Sec. 5), applied per pixel.
constexpr float kCut2 = 9.0f;
constexpr float kCut = 3.0f;
// Footprint radius^2 = 9 (1 + 2^-10): a superset of the FP32 per-pixel test.
constexpr float kFoot2 = 9.0087890625f;
// Low-pass filter disk in the footprint: radius^2 = foot2 / 2 + 1/16 about the
// FP32 projected centre (the pad covers that centre's rounding).
constexpr float kLpPad = 0.0625f;
// Thresholds the paper leaves to the 3DGS conventions.
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

// A tile has kTilePix = 256 pixels, one per thread of a 4-wave block: tw x th
// pixels with tw in {8, 16, 32, 64} (a launch choice, 16 x 16 by default),
// row-major inside the tile, so wave w owns the tile rows
// [w * 64 / tw, (w + 1) * 64 / tw).
constexpr int kTilePix = 256;
constexpr int kTileDefault = 16;
constexpr int kMaxK = 32;
constexpr int kRecWords = 6;             // 16-byte words per surfel walk record

enum : int { kSphere = 0, kAabb = 1, kEllipse = 2 };
enum : int { kFull = 0, kTopK = 1 };
enum : int { kF32 = 0, kF16 = 1, kBF16 = 2 };

// Status words kept in the workspace (uint32 each).
enum : int {
  kStP = 0,        // pairs emitted (min(required, capacity))
  kStOverflow = 1, // 1 if required > capacity
  kStN = 2,        // number of virtual surfels
  kStVisible = 3,
  kStCull = 4,     // 4 .. 8: cull codes 0..4
  kStTiles = 9,    // number of tiles (length of the tile work order)
  kStReqLo = 10,   // required pairs, 64-bit
  kStReqHi = 11,
  kStWalked = 12,  // 64-bit: pixel x list-entry evaluations of the forward walk
  kStBlended = 14, // 64-bit: blended (pixel, surfel) pairs
  kStQueue = 16,   // 16 .. 19: work-queue heads of the persistent tile kernels
  kStWide = 20,    // tiles the Top-K blend left to its windowed pass
  kStSigCap = 21,  // layout the forward ran with: pair capacity, tiles, total bytes (64-bit)
  kStSigTiles = 22,
  kStBwdEntries = 24,  // 64-bit: sum over pixels of n_last (list entries the backward walk must evaluate)
  kStSigLo = 26,
  kStSigHi = 27,
  kStUnique = 28,  // 64-bit, written by the stats read-back: distinct selected virtual surfels
  kStSelected = 30,  // 64-bit, written by the stats read-back: (pixel, slot) selections
  kStSelPairs = 32,  // 64-bit, written by the stats read-back: (tile, surfel) pairs with a selection
  kStHeavy = 34,     // backward: surfels with more than kHeavyRows flagged rows (length of their list)
  kStWords = 36
};
// Words updated by 64-bit atomics must be 8-byte aligned (a misaligned atomic
// is a memory violation); the status block itself starts the workspace.
static_assert(kStReqLo % 2 == 0 && kStWalked % 2 == 0 && kStBlended % 2 == 0 && kStBwdEntries % 2 == 0 &&
                  kStUnique % 2 == 0 && kStSelected % 2 == 0 && kStSelPairs % 2 == 0 && kStSigLo % 2 == 0,
              "64-bit status words sit at even word indices");
enum : int { kQWalk = 0, kQBlend = 1, kQFeatBwd = 2, kQWalkBwd = 3 };
// Radix sort tiling.
// Surfels with more flagged feature-gradient rows than this (over all
// cameras) have them summed by a block of their own rather than a lane group.
constexpr int kHeavyRows = 64;

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
// Count-scan tiling.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ----------------------------------------------------------------- cameras
constexpr int kMaxCams = 8;

struct CamArgs {
  float R[9], t[3], fx, fy, cx, cy, near_plane;
  int W, H;
};

// The cameras of one call, passed to kernels by value.  Surfel i seen by
// camera b is the virtual surfel v = b * N + i; camera b's tiles are the
// global tiles [tile0[b], tile0[b + 1]) and its images start at pixel
// pix0[b] of the concatenated output maps.
struct CamTable {
  int n;
  int64_t nsurf;
  int tw, th, tsh;  // tile width and height in pixels (tw * th = 256), log2(tw)
  CamArgs cam[kMaxCams];
  int ntx[kMaxCams], nty[kMaxCams];
  int tile0[kMaxCams + 1];
  int64_t pix0[kMaxCams + 1];
};

// Tile-local column and row of pixel p (0..255) of a tile.
__host__ __device__ inline int tile_lx(const CamTable& ct, int p) { return p & (ct.tw - 1); }
__host__ __device__ inline int tile_ly(const CamTable& ct, int p) { return p >> ct.tsh; }

// Where global tile g lies: its camera, tile coordinates and image.
struct TileLoc {
  int b, tx, ty, W, H;
  int64_t pix0;  // first pixel of the camera's images
  int64_t v0;    // first virtual surfel of the camera
};

// Camera of virtual surfel v (no 64-bit division).
__host__ __device__ inline int camera_of(const CamTable& ct, int64_t v) {
  int b = 0;
#pragma unroll
  for (int k = 1; k < kMaxCams; ++k) b += (k < ct.n && v >= (int64_t)k * ct.nsurf) ? 1 : 0;
  return b;
}

__host__ __device__ inline TileLoc locate(const CamTable& ct, int g) {
  int b = 0;
#pragma unroll
  for (int k = 1; k < kMaxCams; ++k) b += (k < ct.n && g >= ct.tile0[k]) ? 1 : 0;
  const int lt = g - ct.tile0[b];
  TileLoc t;
  t.b = b;
  t.tx = lt % ct.ntx[b];
  t.ty = lt / ct.ntx[b];
  t.W = ct.cam[b].W;
  t.H = ct.cam[b].H;
  t.pix0 = ct.pix0[b];
  t.v0 = (int64_t)b * ct.nsurf;
  return t;
}

// ---------------------------------------------------------- workspace layout
struct Layout {
  int64_t n, nreal, cap, tiles, spix;  // n = virtual surfels; spix = tiles * 256 (tile-major pixels)
  int k, c, ncam;
  size_t rec, fp, ext, key0, key1, id0, id1, vbase, count, offs, cull, ptile0, ptile1, eid0, eid1, sid_emit, pid, ranges,
      torder0, wide, nlast, tfinal, selpos, selw, seldot, gflag, fflag, gpart, fpart, hist, bsum, ubits, heavy,
      status, total;
};

inline Layout make_layout(const CamTable& ct, int k, int c, int64_t cap) {
  Layout L{};
  L.nreal = ct.nsurf;
  L.ncam = ct.n;
  L.n = ct.nsurf * ct.n;
  L.cap = cap;
  L.k = k;
  L.c = c;
  L.tiles = ct.tile0[ct.n];
  L.spix = L.tiles * kTilePix;
  const int64_t n1 = L.n > 0 ? L.n : 1, cap1 = cap > 0 ? cap : 1, t1 = L.tiles > 0 ? L.tiles : 1;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  L.status = take(kStWords * 4);  // first, so a read-back can check the layout before any other access
  L.rec = take(n1 * 16 * kRecWords);  // walk record
  L.fp = take(n1 * 48);           // footprint floats, 12
  L.ext = take(n1 * 16);          // ellipse centre and half-extents (x, y), for band culling
  L.key0 = take(n1 * 4);          // depth keys (sort ping-pong)
  L.key1 = take(n1 * 4);
  L.id0 = take(n1 * 4);           // virtual surfel ids (sort ping-pong)
  L.id1 = take(n1 * 4);
  L.vbase = take(n1 * 4);         // first emitted pair of each virtual surfel
  L.count = take(n1 * 4);         // pairs per virtual surfel
  L.offs = take((n1 + 1) * 4);    // exclusive scan of counts in depth order
  L.cull = take(n1 * 4);
  L.ptile0 = take(cap1 * 4);      // pair tile ids (sort keys, ping-pong)
  L.ptile1 = take(cap1 * 4);
  L.eid0 = take(cap1 * 4);        // pair emission index (sort values, ping-pong)
  L.eid1 = take(cap1 * 4);
  L.sid_emit = take(cap1 * 4);    // virtual surfel id of each emitted pair
  L.pid = take(cap1 * 4);         // virtual surfel id of each sorted pair
  L.ranges = take(t1 * 8);        // [start, end) per tile
  L.torder0 = take(t1 * 4);       // tile work order, longest lists first
  L.wide = take(t1 * 4);          // tiles of the Top-K blend's windowed pass
  L.nlast = take(L.spix * 4);
  L.tfinal = take(L.spix * 4);
  L.selpos = take(L.spix * (size_t)k * 4);
  L.selw = take(L.spix * (size_t)k * 4);
  L.seldot = take(L.spix * (size_t)k * 4);
  // backward partial sums per (tile, surfel) pair, at the pair's emission index
  L.gflag = take(cap1);
  L.fflag = take(cap1);
  L.gpart = take(cap1 * 64);      // 16 floats: geometric and colour terms
  L.fpart = take(cap1 * (size_t)(c > 0 ? c : 1) * 4);  // feature gradient rows
  int64_t big = n1 > cap1 ? n1 : cap1;
  big = big > t1 ? big : t1;
  const int64_t nb = cdiv(big, kSortTile);
  L.hist = take((256 * nb + 256) * 4);
  L.bsum = take((cdiv(n1, kScanTile) + 1) * 8);
  L.ubits = take(cdiv(n1, 32) * 4);  // one bit per virtual surfel: selected somewhere (stats read-back)
  // surfels with more than kHeavyRows flagged rows: the rows are pairs, whose
  // ranges are disjoint inside the capacity, so at most cap / (kHeavyRows + 1)
  L.heavy = take((cap1 / (kHeavyRows + 1) + 1) * 4);
  L.total = o;
  return L;
}

// ------------------------------------------------------------ walk record
// Per surfel (global, 6 x 16 bytes), computed in FP64 from the FP32 inputs:
//   d0 = (Ai00, Ai01), d1 = (Ai10, Ai11)   FP64: inverse of A, the centred,
//                                          depth-normalised homography [[A,0],[p q 1]]
//   d2 = (e0, e1)                          FP64: e = (p, q) A^-1
//   d3 = (xc, yc)                          FP64: projected surfel centre
//   f0 = (mz, o, r, g), f1 = (b, n0, n1, n2)  FP32
// For a pixel offset d = (x - xc, y - yc):  u' = A^-1 d, w' = 1 - e.d,
// (u, v) = u'/w', intersection depth z = mz / w'.
//
// The solve is FP64: for a surfel seen at a grazing angle A is ill-conditioned
// and an FP32 evaluation of u' loses eps * cond(A) relative accuracy (1e-4 in
// rho at cond(A) ~ 100), far beyond the 1e-5 image tolerance; FP32 pixel
// coordinates near 10^3 would also carry 6e-5 px of rounding.

struct __align__(16) WalkRec {
  double2 d0, d1, d2, d3;
  float4 f0, f1;
};
static_assert(sizeof(WalkRec) == 16 * kRecWords, "walk record layout");

// Tile-local copy staged in LDS: the tile origin's offset (ox, oy) from the
// centre, so a pixel's offset is d = (lx + ox, ly + oy) for its tile-local
// centre (lx, ly).
struct LRec {
  double a00, a01, a10, a11, e0, e1, ox, oy;
  float mz, o, r, g, b, n0, n1, n2;
};

// LDS staging of a batch of tile-local records (structure of arrays, so a
// batch is written with consecutive addresses and read by broadcast).
template <int B>
struct Staged {
  double2 a0[B], a1[B], e[B], o[B];
  float4 f0[B], f1[B];

  __device__ __forceinline__ void put(int slot, const WalkRec& r, float tx0, float ty0) {
    a0[slot] = r.d0;
    a1[slot] = r.d1;
    e[slot] = r.d2;
    o[slot] = make_double2((double)tx0 - r.d3.x, (double)ty0 - r.d3.y);
    f0[slot] = r.f0;
    f1[slot] = r.f1;
  }
  __device__ __forceinline__ LRec get(int k) const {
    LRec s;
    const double2 x0 = a0[k], x1 = a1[k], x2 = e[k], x3 = o[k];
    const float4 y0 = f0[k], y1 = f1[k];
    s.a00 = x0.x; s.a01 = x0.y; s.a10 = x1.x; s.a11 = x1.y;
    s.e0 = x2.x; s.e1 = x2.y; s.ox = x3.x; s.oy = x3.y;
    s.mz = y0.x; s.o = y0.y; s.r = y0.z; s.g = y0.w;
    s.b = y1.x; s.n0 = y1.y; s.n1 = y1.z; s.n2 = y1.w;
    return s;
  }
};

// Per-pixel evaluation of one surfel (Sec. 3.1): the intersection (u, v) of
// the pixel ray with the surfel plane, rho = u^2 + v^2, hit iff rho <= 9,
// alpha = min(0.99, o exp(-rho/2)).  Returns true for a contributor
// (hit and alpha >= 1/255).  The hit decision is taken in FP64; rho, alpha
// and the values handed on are FP32.
//
// LP: the optional screen-space low-pass filter (the 2DGS variant),
// rho = min(u^2 + v^2, 2 |d|^2) with d the pixel's offset from the projected
// centre; the term is chosen in FP64, ties to the ray-splat term.  Where the
// filter term is taken (filt), u = v = 0 and iw = 1, so the depth mz * iw is
// the centre's depth.
struct PixEval {
  float dx, dy, u, v, iw, G, alpha;
  bool clamped, filt;
};

template <bool LP = false>
__device__ __forceinline__ bool eval_pixel(const LRec& s, float lx, float ly, PixEval& e) {
  const double dx = (double)lx + s.ox, dy = (double)ly + s.oy;
  const double u1 = fma(s.a00, dx, s.a01 * dy);
  const double v1 = fma(s.a10, dx, s.a11 * dy);
  const double w1 = 1.0 - fma(s.e0, dx, s.e1 * dy);
  const double num = fma(u1, u1, v1 * v1);
  float rho;
  if constexpr (LP) {
    const double rf = 2.0 * fma(dx, dx, dy * dy);
    const bool splat = w1 > 0.0 && num <= rf * (w1 * w1);
    if (splat ? !(num <= 9.0 * (w1 * w1)) : !(rf <= 9.0)) return false;
    e.filt = !splat;
    e.dx = (float)dx;
    e.dy = (float)dy;
    if (splat) {
      const float wf = (float)w1;
      e.iw = __builtin_amdgcn_rcpf(wf);
      e.u = (float)u1 * e.iw;
      e.v = (float)v1 * e.iw;
      rho = fmaf(e.u, e.u, e.v * e.v);
    } else {
      e.iw = 1.0f;
      e.u = 0.0f;
      e.v = 0.0f;
      rho = 2.0f * fmaf(e.dx, e.dx, e.dy * e.dy);
    }
  } else {
    if (!(w1 > 0.0) || !(num <= 9.0 * (w1 * w1))) return false;
    e.filt = false;
    e.dx = (float)dx;
    e.dy = (float)dy;
    const float wf = (float)w1;
    e.iw = __builtin_amdgcn_rcpf(wf);
    e.u = (float)u1 * e.iw;
    e.v = (float)v1 * e.iw;
    rho = fmaf(e.u, e.u, e.v * e.v);
  }
  e.G = __builtin_amdgcn_exp2f(rho * -0.72134752044448170f);  // exp(-rho/2)
  const float oG = s.o * e.G;
  e.clamped = oG > kAlphaMax;
  e.alpha = e.clamped ? kAlphaMax : oG;
  return e.alpha >= kAlphaMin;
}

// Band culling of the walks: a wave owns 64 / tw rows of its tile and skips
// a surfel whose footprint ellipse's y-extent (centre ecy, half-extent ey,
// the key stage's FP32 values) misses the rows' pixel centres.  The footprint
// contains every pixel the per-pixel test can hit; the slack covers the FP32
// rounding of the band edges (ulp(16384) = 2^-9 px).
constexpr float kBandSlack = 0.015625f;

__device__ __forceinline__ bool band_meets(float ecy, float ey, float yb0, float yb1) {
  return (ecy + ey) + kBandSlack >= yb0 && (ecy - ey) - kBandSlack <= yb1;
}

// Tile index of a block: consecutive block ids are dispatched round-robin
// over the 8 XCDs, so give each XCD a contiguous run of tiles (neighbouring
// tiles share surfels, and each XCD has its own L2).
__device__ inline int xcd_tile(int bid, int tiles) {
  const int per = (tiles + 7) >> 3;
  return (bid & 7) * per + (bid >> 3);
}
inline int xcd_grid(int64_t tiles) { return (int)(((tiles + 7) >> 3) << 3); }

// Tile scheduling of the per-tile kernels.  Grid mode (order == null): one
// block per tile, XCD-aware.  Persistent mode: a grid that fills the device
// once takes tiles from a work queue ordered longest list first, so long
// tiles start early and blocks that finish keep taking work.  Every block
// leaves the loop once the queue is drained.
struct TileQueue {
  const uint32_t* order;  // tile ids, longest list first; null: grid mode
  uint32_t* head;         // queue head, zero before the launch
  int tiles;
};

template <bool PERSIST, class F>
__device__ __forceinline__ void for_tiles(const TileQueue& q, int* s_item, F&& body) {
  if constexpr (!PERSIST) {
    const int tile = xcd_tile(blockIdx.x, q.tiles);
    if (tile < q.tiles) body(tile);
  } else {
    for (;;) {
      __syncthreads();  // the previous tile is finished by every thread
      if (threadIdx.x == 0) *s_item = (int)atomicAdd(q.head, 1u);
      __syncthreads();
      const int it = *s_item;
      if (it >= q.tiles) break;
      body((int)q.order[it]);
    }
  }
}

// ------------------------------------------------------------ wave helpers
// Cross-lane exchanges without LDS: v_permlane32_swap / v_permlane16_swap
// (gfx950) exchange halves of the wave / of 32-lane halves between two
// registers, DPP row operations pair lanes inside a 16-lane row.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
constexpr int kDppRowRor8 = 0x128;      // lane l <- lane l ^ 8 within a row
constexpr int kDppRowHalfMirror = 0x141;  // lane l <- lane 7 - l within 8 lanes
constexpr int kDppXor2 = 0x4E;          // quad_perm [2,3,0,1]
constexpr int kDppXor1 = 0xB1;          // quad_perm [1,0,3,2]

// x + x(lane ^ 32) (first) and y + y(lane ^ 32) (second), for the lanes whose
// bit 5 selects x (lanes 0-31) or y (lanes 32-63).
__device__ __forceinline__ float swap32_add(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_add(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float wave_sum(float v) {
  v = swap32_add(v, v);
  v = swap16_add(v, v);
  v += dpp_mov<kDppRowRor8>(v);
  v += dpp_mov<kDppRowHalfMirror>(v);
  v += dpp_mov<kDppXor2>(v);
  v += dpp_mov<kDppXor1>(v);
  return v;
}

// Sums 16 per-lane values over the wave: each step halves the number of
// values a lane carries (16 -> 8 -> 4 -> 2 -> 1), pairing lanes that differ in
// lane bit 5, 4, 3, 2; then two in-quad steps.  Lane l returns the wave total
// of value index (l >> 2) & 15.
__device__ __forceinline__ float wave_reduce16(const float (&v)[16]) {
  const int lane = threadIdx.x & 63;
  float a[8], b[4], c[2];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = swap32_add(v[i], v[8 + i]);
#pragma unroll
  for (int i = 0; i < 4; ++i) b[i] = swap16_add(a[i], a[4 + i]);
  const bool b3 = lane & 8, b2 = lane & 4;
#pragma unroll
  for (int i = 0; i < 2; ++i) c[i] = (b3 ? b[2 + i] : b[i]) + dpp_mov<kDppRowRor8>(b3 ? b[i] : b[2 + i]);
  float d = (b2 ? c[1] : c[0]) + dpp_mov<kDppRowHalfMirror>(b2 ? c[0] : c[1]);
  d += dpp_mov<kDppXor2>(d);
  d += dpp_mov<kDppXor1>(d);
  return d;
}

// ------------------------------------------------ feature loads (to float)
// Storage types: float, __half, and uint16_t holding bf16 bits.
template <typename FT>
struct VecN {
  static constexpr int N = 16 / sizeof(FT);  // elements per 16-byte load
};

template <typename FT>
__device__ __forceinline__ void load_vec(const FT* p, float* v);
template <>
__device__ __forceinline__ void load_vec<float>(const float* p, float* v) {
  const float4 x = *reinterpret_cast<const float4*>(p);
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
template <>
__device__ __forceinline__ void load_vec<__half>(const __half* p, float* v) {
  const uint4 x = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[2 * i] = __half2float(__ushort_as_half((unsigned short)(w[i] & 0xFFFF)));
    v[2 * i + 1] = __half2float(__ushort_as_half((unsigned short)(w[i] >> 16)));
  }
}
template <>
__device__ __forceinline__ void load_vec<uint16_t>(const uint16_t* p, float* v) {
  const uint4 x = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[2 * i] = __uint_as_float(w[i] << 16);
    v[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
  }
}
// LDS ordering between the lanes of one wave (no block barrier involved).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FP32 matrix-core product on a 16 x 16 tile, k = 4 (v_mfma_f32_16x16x4f32):
// lane l supplies A[l & 15][l >> 4] and B[l >> 4][l & 15] and holds
// D[4 (l >> 4) + r][l & 15] in component r.  Products are exact and summed in
// FP32 in a fixed order, so a sequence of these is deterministic.
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4v mfma_16x16x4(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename FT>
__device__ __forceinline__ float load_one(const FT* p);
template <>
__device__ __forceinline__ float load_one<float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float load_one<__half>(const __half* p) { return __half2float(*p); }
template <>
__device__ __forceinline__ float load_one<uint16_t>(const uint16_t* p) {
  return __uint_as_float(((uint32_t)*p) << 16);
}

// Four consecutive feature channels as float.
template <typename FT>
__device__ __forceinline__ float4 load4(const FT* p);
template <>
__device__ __forceinline__ float4 load4<float>(const float* p) {
  return *reinterpret_cast<const float4*>(p);
}
template <>
__device__ __forceinline__ float4 load4<__half>(const __half* p) {
  const uint2 x = *reinterpret_cast<const uint2*>(p);
  return make_float4(__half2float(__ushort_as_half((unsigned short)(x.x & 0xFFFF))),
                     __half2float(__ushort_as_half((unsigned short)(x.x >> 16))),
                     __half2float(__ushort_as_half((unsigned short)(x.y & 0xFFFF))),
                     __half2float(__ushort_as_half((unsigned short)(x.y >> 16))));
}
template <>
__device__ __forceinline__ float4 load4<uint16_t>(const uint16_t* p) {
  const uint2 x = *reinterpret_cast<const uint2*>(p);
  return make_float4(__uint_as_float(x.x << 16), __uint_as_float(x.x & 0xFFFF0000u), __uint_as_float(x.y << 16),
                     __uint_as_float(x.y & 0xFFFF0000u));
}

// The feature rows a render blends: channels [0, ca) from a (storage type FT,
// row stride ca) and channels [ca, ca + cb) from b (FP32, row stride cb; the
// second source is optional: cb = 0).  Both widths are multiples of 8, so a
// group of 4 channels starting at a multiple of 4 lies in one source.
template <typename FT>
struct FeatSrc {
  const FT* a;
  const float* b;
  int ca, cb;
  __device__ __forceinline__ float4 load4(size_t row, int c) const {
    return c < ca ? psm::load4<FT>(a + row * ca + c) : psm::load4<float>(b + row * cb + (c - ca));
  }
  __device__ __forceinline__ float load1(size_t row, int c) const {
    return c < ca ? load_one<FT>(a + row * ca + c) : b[row * cb + (c - ca)];
  }
};

__device__ __forceinline__ int pow2_ge(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace psm
