// CPU oracle for the 2D-surfel renderer of Psi-Map (arXiv 2604.10982).
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code with
// the GPU path (paper_2604_10982_amd/csrc): every formula here is written
// independently from the paper and the readings listed in the design notes.
//
// What it computes
//   * Key stage, FP32 in a prescribed operation order: per-surfel cull code,
//     depth key, normal orientation, and the (tile, surfel) lists of the three
//     footprint modes (isotropic square = the paper's "bounding sphere"
//     baseline, the AABB of eq. (17), and the exact projected ellipse of the
//     Precise Tile Intersection, Sec. 5).  FP32 is the precision that decides
//     these integers on the GPU as well, so lists and order are compared
//     bit-exactly.
//   * Forward render, FP64: the surfel kernel d_sigma and alpha of Sec. 3.1,
//     the front-to-back blend of eq. (1) for RGB, depth, normal and alpha,
//     and the feature channel either densely (eq. (1) with c_i = f_i) or with
//     Top-K hard selection (eq. (18), Sec. 5).
//   * Backward, FP64: gradients of L = <upstream, outputs> with respect to
//     every surfel parameter.  Per-pixel adjoints of the blend are written out
//     by the product rule; the per-surfel Jacobians of alpha, depth and normal
//     use forward-mode dual numbers over (mu, s, q, o).
//
// Parity pins for each function live in tests/test_oracle_*.py.
#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ------------------------------------------------------------------ constants
// Cutoff radius r = 3 in tangent units (the "3 sigma" confidence of Sec. 5,
// applied per pixel as well, so the footprint mode never changes an image).
constexpr double kCut2 = 9.0;
constexpr float kCutF = 3.0f;
// Footprint radius^2 inflated by 2^-10 (relative) so the FP32 footprint is a
// superset of the per-pixel FP32 hit test.
constexpr float kFoot2F = 9.0087890625f;  // 9 * (1 + 2^-10), exact in FP32
// 3DGS conventions for the thresholds the paper leaves unstated.
constexpr double kAlphaMin = 1.0 / 255.0;
constexpr double kAlphaMax = 0.99;
constexpr double kTMin = 1e-4;
// Optional screen-space low-pass filter (the 2DGS variant): the kernel value
// is the larger of the ray-splat Gaussian and an isotropic screen-space
// Gaussian of variance 1/2 px^2 about the projected centre c, i.e.
// rho = min(u^2 + v^2, 2 |x - c|^2).  Its listed disk has radius^2
// foot2 / 2 + 1/16 about the FP32 centre (1/16 px^2 covers the FP32 centre's
// rounding at any image size).
constexpr float kLpPadF = 0.0625f;

enum Cull { kVisible = 0, kCullQuat = 1, kCullNear = 2, kCullDisk = 3, kCullDegenerate = 4 };
enum Mode { kSphere = 0, kAabb = 1, kEllipse = 2 };

struct Cam {
  float R[9], t[3], fx, fy, cx, cy, near_plane;
  int W, H;
};

Cam load_cam(const float* c) {
  Cam k;
  std::memcpy(k.R, c, 9 * sizeof(float));
  std::memcpy(k.t, c + 9, 3 * sizeof(float));
  k.fx = c[12]; k.fy = c[13]; k.cx = c[14]; k.cy = c[15]; k.near_plane = c[16];
  k.W = (int)c[17]; k.H = (int)c[18];
  return k;
}

inline uint32_t fbits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }

// ============================================================== FP32 key stage
// Every line below is one FP32 operation in the prescribed order; no
// contraction (built with -ffp-contract=off), IEEE sqrt and division.
struct KeyF {
  int cull;
  uint32_t depth_bits;
  int flip;
  float ecx, ecy, S00, S01, S11, ex, ey, gam, kk;  // ellipse centre, shape; kk = |c * det A|
  float xc, yc, rf2;  // projected centre; low-pass disk radius^2 (0: no filter)
};

// Opacity-aware footprint bound (exact work reduction, reading of Sec. 3.1):
// alpha = o G < 1/255 skips a pixel, G = exp(-rho/2), so only rho <=
// 2 ln(255 o) can contribute.  The bound is widened by 2^-10 (absolute, then
// relative), rounded up to the 2^-12 grid in double precision, kept at least
// 2^-12 and at most the standard footprint radius^2.
float opacity_foot2_f32(float o) {
  double bound = 2.0 * std::log(255.0 * (double)o);
  double widened = (bound + 1.0 / 1024.0) * (1.0 + 1.0 / 1024.0);
  double grid = std::ceil(widened * 4096.0) / 4096.0;
  if (!(grid >= 1.0 / 4096.0)) grid = 1.0 / 4096.0;
  if (grid > (double)kFoot2F) grid = (double)kFoot2F;
  return (float)grid;
}

// foot2: radius^2 of the listed footprint; culling always uses kFoot2F.
// lowpass: also list the low-pass filter's disk.
KeyF key_f32(const float* mu, const float* sc, const float* q, const Cam& k, float foot2 = kFoot2F,
             int lowpass = 0) {
  KeyF r;
  std::memset(&r, 0, sizeof(r));
  // quaternion (w,x,y,z) -> unit
  float nq = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
  if (!(nq > 0.0f)) { r.cull = kCullQuat; return r; }
  float rn = 1.0f / std::sqrt(nq);
  float w = q[0] * rn, x = q[1] * rn, y = q[2] * rn, z = q[3] * rn;
  // rotation columns t_u, t_v, n (Hamilton convention)
  float xx = x * x, yy = y * y, zz = z * z;
  float xy = x * y, xz = x * z, yz = y * z;
  float wx = w * x, wy = w * y, wz = w * z;
  float tu[3] = {1.0f - 2.0f * (yy + zz), 2.0f * (xy + wz), 2.0f * (xz - wy)};
  float tv[3] = {2.0f * (xy - wz), 1.0f - 2.0f * (xx + zz), 2.0f * (yz + wx)};
  float nn[3] = {2.0f * (xz + wy), 2.0f * (yz - wx), 1.0f - 2.0f * (xx + yy)};
  // camera space
  float mc[3], a[3], b[3], rnv[3];
  for (int i = 0; i < 3; ++i) {
    const float* Ri = k.R + 3 * i;
    mc[i] = ((Ri[0] * mu[0] + Ri[1] * mu[1]) + Ri[2] * mu[2]) + k.t[i];
    float ra = (Ri[0] * tu[0] + Ri[1] * tu[1]) + Ri[2] * tu[2];
    float rb = (Ri[0] * tv[0] + Ri[1] * tv[1]) + Ri[2] * tv[2];
    rnv[i] = (Ri[0] * nn[0] + Ri[1] * nn[1]) + Ri[2] * nn[2];
    a[i] = sc[0] * ra;
    b[i] = sc[1] * rb;
  }
  float dn = (rnv[0] * mc[0] + rnv[1] * mc[1]) + rnv[2] * mc[2];
  r.flip = dn > 0.0f ? 1 : 0;
  // culling: centre and whole cutoff disk in front of the near plane
  if (!(mc[2] > k.near_plane)) { r.cull = kCullNear; return r; }
  float zmin = mc[2] - kCutF * std::sqrt(a[2] * a[2] + b[2] * b[2]);
  if (!(zmin > k.near_plane)) { r.cull = kCullDisk; return r; }
  float iz = 1.0f / mc[2];
  float p = a[2] * iz, qv = b[2] * iz;
  float g2 = p * p + qv * qv;
  float gam = 1.0f - kFoot2F * g2;
  if (!(gam > 0.0f)) { r.cull = kCullDisk; return r; }
  // centred, depth-normalised homography [[A, 0], [p q 1]]
  float mx = mc[0] * iz, my = mc[1] * iz;
  float xc = k.fx * mx + k.cx, yc = k.fy * my + k.cy;
  float A00 = k.fx * ((a[0] - mx * a[2]) * iz);
  float A01 = k.fx * ((b[0] - mx * b[2]) * iz);
  float A10 = k.fy * ((a[1] - my * a[2]) * iz);
  float A11 = k.fy * ((b[1] - my * b[2]) * iz);
  float dA = A00 * A11 - A01 * A10;
  if (!(std::fabs(dA) > 0.0f)) { r.cull = kCullDegenerate; return r; }
  // ellipse shape S = c A (I + c g g^T) A^T with c = r^2 / gamma
  float cc = kFoot2F / gam;
  float w0 = A00 * p + A01 * qv, w1 = A10 * p + A11 * qv;
  float S00 = cc * ((A00 * A00 + A01 * A01) + cc * (w0 * w0));
  float S01 = cc * ((A00 * A10 + A01 * A11) + cc * (w0 * w1));
  float S11 = cc * ((A10 * A10 + A11 * A11) + cc * (w1 * w1));
  if (!(S00 > 0.0f && S11 > 0.0f && S00 < 1e24f && S11 < 1e24f)) {
    r.cull = kCullDegenerate; return r;
  }
  if (foot2 != kFoot2F) {
    // smaller listed footprint: the same shape formulas at radius^2 foot2
    gam = 1.0f - foot2 * g2;
    cc = foot2 / gam;
    S00 = cc * ((A00 * A00 + A01 * A01) + cc * (w0 * w0));
    S01 = cc * ((A00 * A10 + A01 * A11) + cc * (w0 * w1));
    S11 = cc * ((A10 * A10 + A11 * A11) + cc * (w1 * w1));
  }
  r.cull = kVisible;
  r.depth_bits = fbits(mc[2]);
  // perspective moves the ellipse centre off the projected surfel centre
  r.ecx = xc - cc * w0;
  r.ecy = yc - cc * w1;
  r.S00 = S00; r.S01 = S01; r.S11 = S11;
  r.ex = std::sqrt(S00); r.ey = std::sqrt(S11);
  r.gam = gam; r.kk = std::fabs(cc * dA);
  r.xc = xc; r.yc = yc;
  r.rf2 = lowpass ? 0.5f * foot2 + kLpPadF : 0.0f;
  return r;
}

// Tiles whose pixel-centre hull meets [lo, hi] along one axis.
bool span_f32(float lo, float hi, int npix, int tsz, int nt, int& t0, int& t1) {
  if (!(hi >= 0.5f) || !(lo <= (float)npix - 0.5f)) return false;
  float f0 = std::ceil((lo - ((float)tsz - 0.5f)) / (float)tsz);
  float f1 = std::floor((hi - 0.5f) / (float)tsz);
  f0 = std::fmax(f0, 0.0f);
  f1 = std::fmin(f1, (float)(nt - 1));
  if (!(f0 <= f1)) return false;
  t0 = (int)f0; t1 = (int)f1;
  return true;
}

struct Row { int ty, tx0, tx1; };

// Footprint rows of a visible surfel for one mode.  With the low-pass filter
// the footprint is the union with the filter's disk: its bounding box joins
// the box of every mode, and in the exact mode each row takes the hull of the
// ellipse's and the disk's x-extents within the row's band.
void footprint(const KeyF& f, const Cam& k, int tw, int th, int mode, std::vector<Row>& rows) {
  rows.clear();
  const int ntx = (k.W + tw - 1) / tw, nty = (k.H + th - 1) / th;
  const bool lp = f.rf2 > 0.0f;
  const float rf = lp ? std::sqrt(f.rf2) : 0.0f;
  int ax0, ax1, ay0, ay1;
  float bx0, bx1, by0, by1;
  if (mode == kSphere) {
    float hs = 0.5f * (f.S00 + f.S11);
    float hd = 0.5f * (f.S00 - f.S11);
    float lmax = hs + std::sqrt(hd * hd + f.S01 * f.S01);
    float rr = std::fmax(std::sqrt(lmax), std::fmax(f.ex, f.ey));
    bx0 = f.ecx - rr; bx1 = f.ecx + rr; by0 = f.ecy - rr; by1 = f.ecy + rr;
  } else {
    bx0 = f.ecx - f.ex; bx1 = f.ecx + f.ex; by0 = f.ecy - f.ey; by1 = f.ecy + f.ey;
  }
  if (lp) {
    bx0 = std::fmin(bx0, f.xc - rf); bx1 = std::fmax(bx1, f.xc + rf);
    by0 = std::fmin(by0, f.yc - rf); by1 = std::fmax(by1, f.yc + rf);
  }
  if (!span_f32(bx0, bx1, k.W, tw, ntx, ax0, ax1)) return;
  if (!span_f32(by0, by1, k.H, th, nty, ay0, ay1)) return;
  if (mode != kEllipse) {
    for (int ty = ay0; ty <= ay1; ++ty) rows.push_back({ty, ax0, ax1});
    return;
  }
  // exact ellipse: per tile row, the x-extent of E within the row's band
  const float yr = f.S01 / f.ex;  // dy of the rightmost point of E
  for (int ty = ay0; ty <= ay1; ++ty) {
    float rlo = (float)(ty * th) + 0.5f;
    float rhi = std::fmin((float)(ty * th) + ((float)th - 0.5f), (float)k.H - 0.5f);
    float ylo = rlo - f.ecy;
    float yhi = rhi - f.ecy;
    float lo = std::fmax(ylo, -f.ey), hi = std::fmin(yhi, f.ey);
    bool have = false;
    float xl = 0.0f, xr = 0.0f;
    if (lo <= hi) {
      float dR = std::fmin(std::fmax(yr, lo), hi);
      float dL = std::fmin(std::fmax(-yr, lo), hi);
      float hR = std::sqrt(std::fmax(0.0f, (f.S11 - dR * dR) / f.gam)) * f.kk;
      float hL = std::sqrt(std::fmax(0.0f, (f.S11 - dL * dL) / f.gam)) * f.kk;
      float xR = (f.S01 * dR + hR) / f.S11;
      float xL = (f.S01 * dL - hL) / f.S11;
      xl = f.ecx + xL;
      xr = f.ecx + xR;
      have = true;
    }
    if (lp) {  // the disk's chord nearest its centre within the band
      float dlo = rlo - f.yc, dhi = rhi - f.yc;
      float dy = std::fmin(std::fmax(0.0f, dlo), dhi);
      float h2 = f.rf2 - dy * dy;
      if (h2 >= 0.0f) {
        float h = std::sqrt(h2);
        float dl = f.xc - h, dr = f.xc + h;
        xl = have ? std::fmin(xl, dl) : dl;
        xr = have ? std::fmax(xr, dr) : dr;
        have = true;
      }
    }
    if (!have) continue;
    int x0, x1;
    if (!span_f32(xl, xr, k.W, tw, ntx, x0, x1)) continue;
    x0 = std::max(x0, ax0); x1 = std::min(x1, ax1);
    if (x0 <= x1) rows.push_back({ty, x0, x1});
  }
}

// ================================================================ FP64 model
// Minimal forward-mode dual number over D seeds.
template <int D>
struct Dual {
  double v;
  double d[D];
  Dual() : v(0) { for (int i = 0; i < D; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < D; ++i) d[i] = 0; }
};
template <int D> Dual<D> operator+(const Dual<D>& a, const Dual<D>& b) { Dual<D> r(a.v + b.v); for (int i = 0; i < D; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int D> Dual<D> operator-(const Dual<D>& a, const Dual<D>& b) { Dual<D> r(a.v - b.v); for (int i = 0; i < D; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int D> Dual<D> operator-(const Dual<D>& a) { Dual<D> r(-a.v); for (int i = 0; i < D; ++i) r.d[i] = -a.d[i]; return r; }
template <int D> Dual<D> operator*(const Dual<D>& a, const Dual<D>& b) { Dual<D> r(a.v * b.v); for (int i = 0; i < D; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int D> Dual<D> operator/(const Dual<D>& a, const Dual<D>& b) { Dual<D> r(a.v / b.v); for (int i = 0; i < D; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v); return r; }
template <int D> Dual<D> operator*(double s, const Dual<D>& a) { Dual<D> r(s * a.v); for (int i = 0; i < D; ++i) r.d[i] = s * a.d[i]; return r; }
template <int D> Dual<D> dsqrt(const Dual<D>& a) { double s = std::sqrt(a.v); Dual<D> r(s); for (int i = 0; i < D; ++i) r.d[i] = a.d[i] / (2.0 * s); return r; }
template <int D> Dual<D> dexp(const Dual<D>& a) { double e = std::exp(a.v); Dual<D> r(e); for (int i = 0; i < D; ++i) r.d[i] = a.d[i] * e; return r; }
inline double dsqrt(double a) { return std::sqrt(a); }
inline double dexp(double a) { return std::exp(a); }
template <int D> double val(const Dual<D>& a) { return a.v; }
inline double val(double a) { return a; }

constexpr int kNP = 10;  // dual seeds: mu(3) s(2) q(4) o(1)
using D10 = Dual<kNP>;

// Surfel geometry in camera space (Sec. 3.1): the 3x3 homography
// M = K [a | b | mu_c] with a = s_u R t_u, b = s_v R t_v, and the normal
// n_c = +-R n turned toward the camera.
template <class S>
struct Geo {
  S M[9];
  S nc[3];
};

template <class S>
Geo<S> geometry(const S mu[3], const S sc[2], const S q[4], const Cam& k, int flip) {
  Geo<S> g;
  S nq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  S rn = S(1.0) / dsqrt(nq);
  S w = q[0] * rn, x = q[1] * rn, y = q[2] * rn, z = q[3] * rn;
  // Hamilton rotation matrix of the unit quaternion (w first)
  S Rq[9] = {
      S(1.0) - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
      2.0 * (x * y + w * z), S(1.0) - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
      2.0 * (x * z - w * y), 2.0 * (y * z + w * x), S(1.0) - 2.0 * (x * x + y * y)};
  S mc[3], a[3], b[3], n[3];
  for (int i = 0; i < 3; ++i) {
    double R0 = k.R[3 * i], R1 = k.R[3 * i + 1], R2 = k.R[3 * i + 2];
    mc[i] = R0 * mu[0] + R1 * mu[1] + R2 * mu[2] + S((double)k.t[i]);
    a[i] = sc[0] * (R0 * Rq[0] + R1 * Rq[3] + R2 * Rq[6]);
    b[i] = sc[1] * (R0 * Rq[1] + R1 * Rq[4] + R2 * Rq[7]);
    n[i] = R0 * Rq[2] + R1 * Rq[5] + R2 * Rq[8];
  }
  const double fx = k.fx, fy = k.fy, cx = k.cx, cy = k.cy;
  S cols[3][3] = {{a[0], a[1], a[2]}, {b[0], b[1], b[2]}, {mc[0], mc[1], mc[2]}};
  for (int j = 0; j < 3; ++j) {
    g.M[0 * 3 + j] = fx * cols[j][0] + cx * cols[j][2];
    g.M[1 * 3 + j] = fy * cols[j][1] + cy * cols[j][2];
    g.M[2 * 3 + j] = cols[j][2];
  }
  for (int i = 0; i < 3; ++i) g.nc[i] = flip ? -n[i] : n[i];
  return g;
}

// Ray-surfel intersection by the homogeneous solve: (u, v, 1) is orthogonal
// to the rows x*M2 - M0 and y*M2 - M1, so it is parallel to their cross
// product.  Returns false when the cross product has no finite (u, v).
template <class S>
bool solve_uv(const Geo<S>& g, double x, double y, S& u, S& v, S& z) {
  S h1[3], h2[3];
  for (int j = 0; j < 3; ++j) {
    h1[j] = x * g.M[6 + j] - g.M[0 + j];
    h2[j] = y * g.M[6 + j] - g.M[3 + j];
  }
  S p0 = h1[1] * h2[2] - h1[2] * h2[1];
  S p1 = h1[2] * h2[0] - h1[0] * h2[2];
  S p2 = h1[0] * h2[1] - h1[1] * h2[0];
  if (val(p2) == 0.0) return false;
  u = p0 / p2;
  v = p1 / p2;
  z = g.M[6] * u + g.M[7] * v + g.M[8];  // depth = third row of M (u, v, 1)
  return true;
}

struct SurfIn {  // float inputs of one surfel
  const float *mu, *s, *q;
  float o;
};

Geo<double> geo_d(const SurfIn& in, const Cam& k, int flip) {
  double mu[3] = {in.mu[0], in.mu[1], in.mu[2]};
  double s[2] = {in.s[0], in.s[1]};
  double q[4] = {in.q[0], in.q[1], in.q[2], in.q[3]};
  return geometry<double>(mu, s, q, k, flip);
}

Geo<D10> geo_dual(const SurfIn& in, const Cam& k, int flip, D10& o) {
  D10 mu[3], s[2], q[4];
  for (int i = 0; i < 3; ++i) { mu[i] = D10(in.mu[i]); mu[i].d[i] = 1.0; }
  for (int i = 0; i < 2; ++i) { s[i] = D10(in.s[i]); s[i].d[3 + i] = 1.0; }
  for (int i = 0; i < 4; ++i) { q[i] = D10(in.q[i]); q[i].d[5 + i] = 1.0; }
  o = D10(in.o); o.d[9] = 1.0;
  return geometry<D10>(mu, s, q, k, flip);
}

// Per-(pixel, surfel) evaluation (Sec. 3.1): rho = u^2 + v^2, hit iff
// rho <= r^2, alpha = min(0.99, o exp(-rho/2)).  With the low-pass filter
// rho = min(u^2 + v^2, 2 |x - c|^2); where the filter term is the smaller
// (ties go to the ray-splat term) the depth is the centre's camera depth.
struct Eval {
  bool hit;
  double rho, G, alpha, z;
  bool clamped;
  bool filt;        // the filter term was taken
  double bmargin;   // relative gap between the two terms (INFINITY: no filter)
};

Eval eval_pixel(const Geo<double>& g, double o, double x, double y, bool lowpass = false) {
  Eval e{};
  e.bmargin = INFINITY;
  double u, v, z;
  const bool ok = solve_uv(g, x, y, u, v, z);
  e.rho = ok ? u * u + v * v : INFINITY;
  e.z = ok ? z : 0.0;
  if (lowpass) {
    const double cx = g.M[2] / g.M[8], cy = g.M[5] / g.M[8];  // projected centre
    const double rf = 2.0 * ((x - cx) * (x - cx) + (y - cy) * (y - cy));
    e.bmargin = std::fabs(e.rho - rf) / std::max(e.rho, rf);
    if (!(e.rho <= rf)) {
      e.filt = true;
      e.rho = rf;
      e.z = g.M[8];
    }
  }
  if (!std::isfinite(e.rho)) { e.hit = false; e.rho = INFINITY; return e; }
  e.hit = e.rho <= kCut2;
  e.G = std::exp(-0.5 * e.rho);
  double a = o * e.G;
  e.clamped = a > kAlphaMax;
  e.alpha = e.clamped ? kAlphaMax : a;
  return e;
}

// ------------------------------------------------------------ scene binding
struct Scene {
  int64_t n;
  const float *means, *scales, *quats, *opacity, *rgb;
  const double* feat;  // N x C, already rounded to the storage dtype
  int C;
  int lowpass;  // screen-space low-pass filter on
  SurfIn in(int64_t i) const { return {means + 3 * i, scales + 2 * i, quats + 4 * i, opacity[i]}; }
};

struct Prepared {
  std::vector<KeyF> key;
  std::vector<Geo<double>> geo;
  std::vector<std::vector<int64_t>> bins;  // per tile, candidates in (depth, id) order
  int ntx, nty, tw, th;
};

// Conservative FP64 candidate bins for the walk: the bounding box of the
// projected disk of radius 1.01 r, from its dual conic M diag(r^2,r^2,-1) M^T.
// Only an acceleration: the walk re-tests every candidate per pixel.
void prepare(const Scene& sc, const Cam& k, int tw, int th, Prepared& P) {
  P.tw = tw; P.th = th;
  P.ntx = (k.W + tw - 1) / tw;
  P.nty = (k.H + th - 1) / th;
  P.key.resize(sc.n);
  P.geo.resize(sc.n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < sc.n; ++i) {
    SurfIn in = sc.in(i);
    P.key[i] = key_f32(in.mu, in.s, in.q, k);
    if (P.key[i].cull == kVisible) P.geo[i] = geo_d(in, k, P.key[i].flip);
  }
  std::vector<int64_t> order;
  order.reserve(sc.n);
  for (int64_t i = 0; i < sc.n; ++i) if (P.key[i].cull == kVisible) order.push_back(i);
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    if (P.key[a].depth_bits != P.key[b].depth_bits) return P.key[a].depth_bits < P.key[b].depth_bits;
    return a < b;
  });
  P.bins.assign((size_t)P.ntx * P.nty, {});
  const double rb2 = kCut2 * 1.01 * 1.01;
  for (int64_t i : order) {
    const double* M = P.geo[i].M;
    double Cs[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        Cs[r][c] = rb2 * (M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1]) - M[3 * r + 2] * M[3 * c + 2];
    double x0, x1, y0, y1;
    if (Cs[2][2] >= 0.0) {  // inflated disk reaches the camera plane: whole image
      x0 = -1e30; x1 = 1e30; y0 = -1e30; y1 = 1e30;
    } else {
      double xc = Cs[0][2] / Cs[2][2], yc = Cs[1][2] / Cs[2][2];
      double dx = std::sqrt(std::max(0.0, Cs[0][2] * Cs[0][2] - Cs[0][0] * Cs[2][2])) / std::fabs(Cs[2][2]);
      double dy = std::sqrt(std::max(0.0, Cs[1][2] * Cs[1][2] - Cs[1][1] * Cs[2][2])) / std::fabs(Cs[2][2]);
      x0 = xc - dx; x1 = xc + dx; y0 = yc - dy; y1 = yc + dy;
    }
    if (sc.lowpass) {  // the filter's disk 2 |x - c|^2 <= r^2, inflated by 1%
      const double cx = M[2] / M[8], cy = M[5] / M[8], rl = std::sqrt(0.5 * kCut2) * 1.01;
      x0 = std::min(x0, cx - rl); x1 = std::max(x1, cx + rl);
      y0 = std::min(y0, cy - rl); y1 = std::max(y1, cy + rl);
    }
    int tx0 = (int)std::max(0.0, std::floor((x0 - 0.5) / tw));
    int tx1 = (int)std::min((double)P.ntx - 1, std::floor((x1 - 0.5) / tw));
    int ty0 = (int)std::max(0.0, std::floor((y0 - 0.5) / th));
    int ty1 = (int)std::min((double)P.nty - 1, std::floor((y1 - 0.5) / th));
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) P.bins[(size_t)ty * P.ntx + tx].push_back(i);
  }
}

// One contributor of a pixel's walk.
struct Contrib {
  int64_t id;
  double alpha, T, w, z;
  bool clamped;
  bool filt;  // low-pass filter term taken
};

// Relative distance of the pixel's decisions from their thresholds, by kind:
// [0] rho vs r^2 (hit), [1] alpha vs 1/255 and vs the 0.99 clamp,
// [2] T' vs 1e-4 (stop), [3] Top-K gap between the K-th and (K+1)-th weight.
struct Margins {
  double m[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
};

// Front-to-back walk of one pixel (eq. (1)): skip non-hits and alpha < 1/255,
// stop before a surfel that would take T below 1e-4.  With topk_stop = K > 0
// (feature-only rendering) the walk also ends once K weights are held and
// 0.99 T is at most the smallest of them: every later weight is alpha T' with
// alpha <= 0.99 and T' <= T, so none can enter the K largest (a tie goes to
// the earlier surfel), and the Top-K selection is that of the full walk.
void walk_pixel(const Scene& sc, const Prepared& P, const Cam& k, int px, int py,
                std::vector<Contrib>& out, double& T_final, Margins& margin, int topk_stop = 0) {
  out.clear();
  margin = Margins();
  const double x = px + 0.5, y = py + 0.5;
  const auto& bin = P.bins[(size_t)(py / P.th) * P.ntx + (px / P.tw)];
  double T = 1.0;
  std::vector<double> held;  // the K largest weights so far, a min-heap
  for (int64_t id : bin) {
    Eval e = eval_pixel(P.geo[id], sc.opacity[id], x, y, sc.lowpass != 0);
    if (std::isfinite(e.rho)) margin.m[0] = std::min(margin.m[0], std::fabs(e.rho - kCut2) / kCut2);
    if (!e.hit) continue;
    margin.m[0] = std::min(margin.m[0], e.bmargin);  // which term a hit takes
    double a_raw = sc.opacity[id] * e.G;
    margin.m[1] = std::min(margin.m[1], std::fabs(a_raw / kAlphaMax - 1.0));
    margin.m[1] = std::min(margin.m[1], std::fabs(e.alpha / kAlphaMin - 1.0));
    if (e.alpha < kAlphaMin) continue;
    double Tn = T * (1.0 - e.alpha);
    margin.m[2] = std::min(margin.m[2], std::fabs(Tn / kTMin - 1.0));
    if (Tn < kTMin) break;
    out.push_back({id, e.alpha, T, e.alpha * T, e.z, e.clamped, e.filt});
    T = Tn;
    if (topk_stop > 0) {
      const double w = out.back().w;
      const auto gt = std::greater<double>();
      if ((int)held.size() < topk_stop) {
        held.push_back(w);
        std::push_heap(held.begin(), held.end(), gt);
      } else if (w > held.front()) {
        std::pop_heap(held.begin(), held.end(), gt);
        held.back() = w;
        std::push_heap(held.begin(), held.end(), gt);
      }
      if ((int)held.size() == topk_stop && kAlphaMax * T <= held.front()) break;
    }
  }
  T_final = T;
}

// Top-K hard selection (eq. (18)): the K contributors of largest weight,
// ties broken by earlier list position; returned as a flag per contributor.
void select_topk(const std::vector<Contrib>& c, int K, std::vector<char>& sel, double& gap) {
  const int n = (int)c.size();
  sel.assign(n, 0);
  gap = INFINITY;
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return c[a].w > c[b].w; });
  for (int i = 0; i < std::min(K, n); ++i) sel[idx[i]] = 1;
  if (n > K) gap = (c[idx[K - 1]].w - c[idx[K]].w) / c[idx[K - 1]].w;
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

// FP32 key stage.  cam: R(9) t(3) fx fy cx cy near W H.
// Writes per surfel: cull code, depth key bits, normal flip, pair count for
// `mode`, and 8 footprint floats (ellipse centre x y, S00 S01 S11, ex ey, gamma) when fp_out
// is non-null.  If cap >= P, also writes the P pairs sorted by
// (tile, depth bits, surfel id).  Returns P.
// opacity: non-null selects the opacity-aware footprint (per-surfel opacities).
// lowpass: list the union with the low-pass filter's disk.
int64_t orc_keystage(int64_t n, const float* means, const float* scales, const float* quats,
                     const float* opacity, const float* cam, int tw, int th, int mode, int lowpass,
                     int32_t* cull_out, uint32_t* depth_out, int32_t* flip_out, int32_t* count_out,
                     float* fp_out, int64_t cap, int32_t* tile_out, int32_t* id_out) {
  Cam k = load_cam(cam);
  std::vector<KeyF> key(n);
  std::vector<int64_t> cnt(n, 0);
  const int ntx = (k.W + tw - 1) / tw;
#pragma omp parallel
  {
    std::vector<Row> rows;
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      const float foot2 = opacity ? opacity_foot2_f32(opacity[i]) : kFoot2F;
      key[i] = key_f32(means + 3 * i, scales + 2 * i, quats + 4 * i, k, foot2, lowpass);
      if (key[i].cull == kVisible) {
        footprint(key[i], k, tw, th, mode, rows);
        int64_t c = 0;
        for (const Row& r : rows) c += r.tx1 - r.tx0 + 1;
        cnt[i] = c;
      }
    }
  }
  int64_t P = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (cull_out) cull_out[i] = key[i].cull;
    if (depth_out) depth_out[i] = key[i].depth_bits;
    if (flip_out) flip_out[i] = key[i].flip;
    if (count_out) count_out[i] = (int32_t)cnt[i];
    if (fp_out) {
      float* f = fp_out + 8 * i;
      f[0] = key[i].ecx; f[1] = key[i].ecy; f[2] = key[i].S00; f[3] = key[i].S01;
      f[4] = key[i].S11; f[5] = key[i].ex; f[6] = key[i].ey; f[7] = key[i].gam;
    }
    P += cnt[i];
  }
  if (cap < P || !tile_out || !id_out) return P;
  struct Pair { int32_t tile; uint32_t depth; int32_t id; };
  std::vector<Pair> pairs;
  pairs.reserve(P);
  std::vector<Row> rows;
  for (int64_t i = 0; i < n; ++i) {
    if (key[i].cull != kVisible) continue;
    footprint(key[i], k, tw, th, mode, rows);
    for (const Row& r : rows)
      for (int tx = r.tx0; tx <= r.tx1; ++tx)
        pairs.push_back({r.ty * ntx + tx, key[i].depth_bits, (int32_t)i});
  }
  std::sort(pairs.begin(), pairs.end(), [](const Pair& a, const Pair& b) {
    if (a.tile != b.tile) return a.tile < b.tile;
    if (a.depth != b.depth) return a.depth < b.depth;
    return a.id < b.id;
  });
  for (int64_t j = 0; j < P; ++j) { tile_out[j] = pairs[j].tile; id_out[j] = pairs[j].id; }
  return P;
}

// FP64 rho = u^2 + v^2 and intersection depth of every surfel at image
// points (xs[j], ys[j]) (pixel units, pixel centres at i + 0.5).  Culled
// surfels or rays with no solution give rho = +inf.  Output [n][npts].
void orc_eval_points(int64_t n, const float* means, const float* scales, const float* quats,
                     const float* cam, int64_t npts, const double* xs, const double* ys,
                     double* rho_out, double* z_out) {
  Cam k = load_cam(cam);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    KeyF kf = key_f32(means + 3 * i, scales + 2 * i, quats + 4 * i, k);
    for (int64_t j = 0; j < npts; ++j) { rho_out[i * npts + j] = INFINITY; if (z_out) z_out[i * npts + j] = 0; }
    if (kf.cull != kVisible) continue;
    SurfIn in{means + 3 * i, scales + 2 * i, quats + 4 * i, 1.0f};
    Geo<double> g = geo_d(in, k, kf.flip);
    for (int64_t j = 0; j < npts; ++j) {
      double u, v, z;
      if (solve_uv(g, xs[j], ys[j], u, v, z)) {
        rho_out[i * npts + j] = u * u + v * v;
        if (z_out) z_out[i * npts + j] = z;
      }
    }
  }
}

// FP64 forward render (Sec. 3.1 eq. (1); Sec. 5 eq. (18)).
// blend: 0 = dense feature blend, 1 = Top-K.  pix: optional list of pixel
// indices (y*W + x); outputs are indexed by list entry (or by pixel if
// pix == null).  Per entry: rgb[3] depth normal[3] alpha feat[C], the number
// of blended surfels, T_final, the id of the last blended surfel, the
// selected ids in front-to-back order with their weights (K slots, -1 pad)
// and the four decision margins (see Margins).
void orc_render(int64_t n, const float* means, const float* scales, const float* quats,
                const float* opacity, const float* rgb, const double* feat, int C,
                const float* cam, int tw, int th, int K, int blend, int lowpass,
                int64_t npix, const int64_t* pix,
                double* rgb_out, double* depth_out, double* normal_out, double* alpha_out,
                double* feat_out, int32_t* ncontrib_out, double* tfinal_out, int64_t* last_out,
                int64_t* sel_id_out, double* sel_w_out, double* margin_out) {
  Cam k = load_cam(cam);
  Scene sc{n, means, scales, quats, opacity, rgb, feat, C, lowpass};
  Prepared P;
  prepare(sc, k, tw, th, P);
  const int64_t S = (int64_t)k.W * k.H;
  const int64_t cnt = pix ? npix : S;
#pragma omp parallel
  {
    std::vector<Contrib> cs;
    std::vector<char> sel;
#pragma omp for schedule(dynamic, 64)
    for (int64_t e = 0; e < cnt; ++e) {
      const int64_t p = pix ? pix[e] : e;
      const int px = (int)(p % k.W), py = (int)(p / k.W);
      double T_final, gap;
      Margins margin;
      walk_pixel(sc, P, k, px, py, cs, T_final, margin, blend == 2 ? K : 0);
      double col[3] = {0, 0, 0}, nor[3] = {0, 0, 0}, dep = 0;
      for (const Contrib& c : cs) {
        const Geo<double>& g = P.geo[c.id];
        for (int j = 0; j < 3; ++j) {
          col[j] += c.w * rgb[3 * c.id + j];
          nor[j] += c.w * g.nc[j];
        }
        dep += c.w * c.z;
      }
      if (blend >= 1) select_topk(cs, K, sel, gap);
      else { sel.assign(cs.size(), 1); gap = INFINITY; }
      if (blend >= 1) margin.m[3] = gap;
      if (feat_out) {
        double* F = feat_out + e * C;
        for (int j = 0; j < C; ++j) F[j] = 0;
        double Wsel = 0;
        for (size_t i = 0; i < cs.size(); ++i)
          if (sel[i]) {
            Wsel += cs[i].w;
            for (int j = 0; j < C; ++j) F[j] += cs[i].w * feat[cs[i].id * (int64_t)C + j];
          }
        // blend mode 3: Top-K with the selected weights renormalised to sum 1
        if (blend == 3 && Wsel > 0)
          for (int j = 0; j < C; ++j) F[j] /= Wsel;
      }
      for (int j = 0; j < 3; ++j) {
        if (rgb_out) rgb_out[3 * e + j] = col[j];
        if (normal_out) normal_out[3 * e + j] = nor[j];
      }
      if (depth_out) depth_out[e] = dep;
      if (alpha_out) alpha_out[e] = 1.0 - T_final;
      if (ncontrib_out) ncontrib_out[e] = (int32_t)cs.size();
      if (tfinal_out) tfinal_out[e] = T_final;
      if (last_out) last_out[e] = cs.empty() ? -1 : cs.back().id;
      if (margin_out)
        for (int j = 0; j < 4; ++j) margin_out[4 * e + j] = margin.m[j];
      if (sel_id_out || sel_w_out) {
        int s = 0;
        for (size_t i = 0; i < cs.size() && s < K; ++i) {
          if (!sel[i]) continue;
          if (sel_id_out) sel_id_out[e * K + s] = cs[i].id;
          if (sel_w_out) sel_w_out[e * K + s] = cs[i].w;
          ++s;
        }
        for (; s < K; ++s) {
          if (sel_id_out) sel_id_out[e * K + s] = -1;
          if (sel_w_out) sel_w_out[e * K + s] = 0.0;
        }
      }
    }
  }
}

// FP64 backward of L = sum over listed pixels of <upstream, outputs>.
// Upstream arrays are indexed like orc_render's outputs.  Gradients are
// accumulated (+=) into the d_* arrays, which the caller zeroes.  When mask
// is non-null only surfels with mask[i] != 0 receive gradients (the others
// still take part in every pixel's walk).
void orc_backward(int64_t n, const float* means, const float* scales, const float* quats,
                  const float* opacity, const float* rgb, const double* feat, int C,
                  const float* cam, int tw, int th, int K, int blend, int lowpass,
                  int64_t npix, const int64_t* pix,
                  const double* g_rgb, const double* g_depth, const double* g_normal,
                  const double* g_alpha, const double* g_feat, const uint8_t* mask,
                  double* d_means, double* d_scales, double* d_quats, double* d_opacity,
                  double* d_rgb, double* d_feat) {
  Cam k = load_cam(cam);
  Scene sc{n, means, scales, quats, opacity, rgb, feat, C, lowpass};
  Prepared P;
  prepare(sc, k, tw, th, P);
  const int64_t S = (int64_t)k.W * k.H;
  const int64_t cnt = pix ? npix : S;
#pragma omp parallel
  {
    std::vector<Contrib> cs;
    std::vector<char> sel;
    std::vector<double> e_i, dfdot;
#pragma omp for schedule(dynamic, 16)
    for (int64_t e = 0; e < cnt; ++e) {
      const int64_t p = pix ? pix[e] : e;
      const int px = (int)(p % k.W), py = (int)(p / k.W);
      double T_final, gap;
      Margins margin;
      walk_pixel(sc, P, k, px, py, cs, T_final, margin, blend == 2 ? K : 0);
      const int m = (int)cs.size();
      if (m == 0) continue;
      if (blend >= 1) select_topk(cs, K, sel, gap);
      else sel.assign(m, 1);
      const double* gC = g_rgb + 3 * e;
      const double* gN = g_normal + 3 * e;
      const double gD = g_depth[e], gA = g_alpha[e];
      const double* gF = g_feat + e * C;
      // renormalised Top-K (blend mode 3): F = sum_sel w_i f_i / W, so the
      // feature part of d/dw_i is gF . (f_i - F) / W and d/df_i = w_i gF / W
      double Wsel = 0.0, gFF = 0.0;
      if (blend == 3) {
        for (int i = 0; i < m; ++i)
          if (sel[i]) Wsel += cs[i].w;
        if (Wsel > 0)
          for (int i = 0; i < m; ++i)
            if (sel[i]) {
              double d = 0;
              for (int j = 0; j < C; ++j) d += gF[j] * feat[cs[i].id * (int64_t)C + j];
              gFF += cs[i].w * d / Wsel;
            }
      }
      // e_i = d<upstream, outputs>/d(weight of contributor i)
      e_i.assign(m, 0.0);
      for (int i = 0; i < m; ++i) {
        const int64_t id = cs[i].id;
        double v = gD * cs[i].z;
        for (int j = 0; j < 3; ++j) v += gC[j] * rgb[3 * id + j] + gN[j] * P.geo[id].nc[j];
        if (sel[i]) {
          double d = 0;
          for (int j = 0; j < C; ++j) d += gF[j] * feat[id * (int64_t)C + j];
          v += blend == 3 ? (Wsel > 0 ? (d - gFF) / Wsel : 0.0) : d;
        }
        e_i[i] = v;
      }
      // out = sum_i w_i x_i with w_i = alpha_i prod_{j<i}(1 - alpha_j), and
      // alpha-map = 1 - prod_i (1 - alpha_i).  Product rule:
      //   dL/dalpha_i = T_i e_i - (sum_{j>i} w_j e_j - gA T_final) / (1 - alpha_i)
      double suffix = 0.0;
      for (int i = m - 1; i >= 0; --i) {
        const Contrib& c = cs[i];
        const int64_t id = c.id;
        const double dalpha = c.T * e_i[i] - (suffix - gA * T_final) / (1.0 - c.alpha);
        suffix += c.w * e_i[i];
        if (mask && !mask[id]) continue;
        // direct terms
        for (int j = 0; j < 3; ++j) {
#pragma omp atomic
          d_rgb[3 * id + j] += c.w * gC[j];
        }
        if (sel[i]) {
          const double wf = blend == 3 ? (Wsel > 0 ? c.w / Wsel : 0.0) : c.w;
          for (int j = 0; j < C; ++j) {
#pragma omp atomic
            d_feat[id * (int64_t)C + j] += wf * gF[j];
          }
        }
        // chain through alpha, depth and normal with dual numbers
        D10 o;
        Geo<D10> g = geo_dual(sc.in(id), k, P.key[id].flip, o);
        D10 u, v, z, rho;
        if (c.filt) {  // low-pass term: 2 |x - c|^2 about the projected centre, centre depth
          const D10 dx = D10(px + 0.5) - g.M[2] / g.M[8], dy = D10(py + 0.5) - g.M[5] / g.M[8];
          rho = 2.0 * (dx * dx + dy * dy);
          z = g.M[8];
        } else {
          solve_uv(g, px + 0.5, py + 0.5, u, v, z);
          rho = u * u + v * v;
        }
        D10 alpha = o * dexp(-0.5 * rho);
        double grad[kNP];
        for (int t = 0; t < kNP; ++t) {
          double s = (c.clamped ? 0.0 : dalpha * alpha.d[t]) + c.w * gD * z.d[t];
          for (int j = 0; j < 3; ++j) s += c.w * gN[j] * g.nc[j].d[t];
          grad[t] = s;
        }
        for (int j = 0; j < 3; ++j) {
#pragma omp atomic
          d_means[3 * id + j] += grad[j];
        }
        for (int j = 0; j < 2; ++j) {
#pragma omp atomic
          d_scales[2 * id + j] += grad[3 + j];
        }
        for (int j = 0; j < 4; ++j) {
#pragma omp atomic
          d_quats[4 * id + j] += grad[5 + j];
        }
#pragma omp atomic
        d_opacity[id] += grad[9];
      }
    }
  }
}

// Per-pixel signature of the decisions a finite difference must not cross:
// the ordered contributor ids, the clamp flags and the Top-K set, hashed.
void orc_decisions(int64_t n, const float* means, const float* scales, const float* quats,
                   const float* opacity, const float* rgb, const double* feat, int C,
                   const float* cam, int tw, int th, int K, int blend, int lowpass,
                   int64_t npix, const int64_t* pix, uint64_t* sig_out) {
  Cam k = load_cam(cam);
  Scene sc{n, means, scales, quats, opacity, rgb, feat, C, lowpass};
  Prepared P;
  prepare(sc, k, tw, th, P);
#pragma omp parallel
  {
    std::vector<Contrib> cs;
    std::vector<char> sel;
#pragma omp for schedule(dynamic, 64)
    for (int64_t e = 0; e < npix; ++e) {
      const int64_t p = pix[e];
      double T_final, gap;
      Margins margin;
      walk_pixel(sc, P, k, (int)(p % k.W), (int)(p / k.W), cs, T_final, margin, blend == 2 ? K : 0);
      if (blend >= 1) select_topk(cs, K, sel, gap);
      else sel.assign(cs.size(), 1);
      uint64_t h = 1469598103934665603ull;
      for (size_t i = 0; i < cs.size(); ++i) {
        uint64_t v = (uint64_t)cs[i].id * 8 + (cs[i].filt ? 4 : 0) + (cs[i].clamped ? 2 : 0) + (sel[i] ? 1 : 0);
        h = (h ^ v) * 1099511628211ull;
      }
      sig_out[e] = h;
    }
  }
}

// Threads of the OpenMP loops from now on (timing on a given number of host
// cores); no effect on any result.
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
