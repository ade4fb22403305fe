// SOGMM geometric loss of surfels (Sec. 3.2 eq. (3), Sec. 4.2 eq. (13) and
// the anisotropy term):
//   component k of the plane prior: weight pi_k, mean mu_k, covariance
//     Sigma_k, reference normal n_k = eigenvector of Sigma_k's smallest
//     eigenvalue;
//   surfel i takes the component of largest posterior pi_k N(mu_i; mu_k,
//     Sigma_k): the smallest score (x - mu_k)^T Sigma_k^-1 (x - mu_k) +
//     ln det Sigma_k - 2 ln pi_k, evaluated in FP32 in a prescribed order
//     (ties to the lower index);
//   L_geo = sum_i |(mu_i - mu_k) . n_k| + lambda_n (1 - |n_i . n_k|),
//   L_iso = sum_i (s_i1 - s_i2)^2,
// and the gradients with the assignment held fixed.
//
// k_gmm_prep: thread per component (FP64): precision by the adjugate, the
//   score constant, the reference normal by cyclic Jacobi sweeps; an FP32
//   record of 16 floats.
// k_geo_loss: thread per surfel; the component records stream through LDS
//   in chunks, every thread scans them (plain vector work: the scan is a
//   minimum, not a contraction), then forms its loss terms and gradients;
//   per-block FP64 sums in a fixed order, summed over the blocks in order.
#include "common.h"
#include "internal.h"

namespace psm {

constexpr int kGmmRec = 16;     // floats per component record
constexpr int kGmmChunk = 1024; // components staged per chunk (64 KB)

// record: mean (3), precision xx xy xz yy yz zz (6), constant (1), normal (3)
__global__ void k_gmm_prep(int k, const float* __restrict__ mean, const float* __restrict__ cov,
                           const float* __restrict__ weight, float* __restrict__ rec) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double a[3][3];
  const float* c = cov + 6 * (size_t)j;
  a[0][0] = c[0]; a[0][1] = a[1][0] = c[1]; a[0][2] = a[2][0] = c[2];
  a[1][1] = c[3]; a[1][2] = a[2][1] = c[4]; a[2][2] = c[5];
  // precision = adjugate / det
  const double A00 = a[1][1] * a[2][2] - a[1][2] * a[2][1];
  const double A01 = a[0][2] * a[2][1] - a[0][1] * a[2][2];
  const double A02 = a[0][1] * a[1][2] - a[0][2] * a[1][1];
  const double A11 = a[0][0] * a[2][2] - a[0][2] * a[2][0];
  const double A12 = a[0][2] * a[1][0] - a[0][0] * a[1][2];
  const double A22 = a[0][0] * a[1][1] - a[0][1] * a[1][0];
  const double det = a[0][0] * A00 + a[0][1] * (a[1][2] * a[2][0] - a[1][0] * a[2][2]) + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  const double id = 1.0 / det;
  float* r = rec + (size_t)kGmmRec * j;
  r[0] = mean[3 * (size_t)j];
  r[1] = mean[3 * (size_t)j + 1];
  r[2] = mean[3 * (size_t)j + 2];
  r[3] = (float)(A00 * id);
  r[4] = (float)(A01 * id);
  r[5] = (float)(A02 * id);
  r[6] = (float)(A11 * id);
  r[7] = (float)(A12 * id);
  r[8] = (float)(A22 * id);
  r[9] = (float)(log(det) - 2.0 * log((double)weight[j]));
  // cyclic Jacobi: a -> V^T a V diagonal; the column of V at the smallest
  // diagonal entry is the reference normal
  double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 12; ++sweep) {
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        const double apq = a[p][q];
        if (apq == 0.0) continue;
        const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int m = 0; m < 3; ++m) {  // columns p, q of a
          const double amp = a[m][p], amq = a[m][q];
          a[m][p] = cs * amp - sn * amq;
          a[m][q] = sn * amp + cs * amq;
        }
        for (int m = 0; m < 3; ++m) {  // rows p, q of a
          const double apm = a[p][m], aqm = a[q][m];
          a[p][m] = cs * apm - sn * aqm;
          a[q][m] = sn * apm + cs * aqm;
        }
        for (int m = 0; m < 3; ++m) {
          const double vmp = V[m][p], vmq = V[m][q];
          V[m][p] = cs * vmp - sn * vmq;
          V[m][q] = sn * vmp + cs * vmq;
        }
      }
  }
  int im = 0;
  if (a[1][1] < a[im][im]) im = 1;
  if (a[2][2] < a[im][im]) im = 2;
  r[10] = (float)V[0][im];
  r[11] = (float)V[1][im];
  r[12] = (float)V[2][im];
  r[13] = r[14] = r[15] = 0.0f;
}

__device__ __forceinline__ double block_sum_f64(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  const double t = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void k_geo_loss(int64_t n, const float* __restrict__ means,
                                                  const float* __restrict__ scales, const float* __restrict__ quats,
                                                  int k, const float* __restrict__ rec, float lambda_n,
                                                  int32_t* __restrict__ assign, float* __restrict__ d_means,
                                                  float* __restrict__ d_scales, float* __restrict__ d_quats,
                                                  double* __restrict__ part) {
  __shared__ float s_rec[kGmmChunk * 10];  // mean, precision, constant of the chunk
  __shared__ double s_red[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = i < n;
  float x0 = 0.f, x1 = 0.f, x2 = 0.f;
  if (ok) {
    x0 = means[3 * i];
    x1 = means[3 * i + 1];
    x2 = means[3 * i + 2];
  }
  float best = INFINITY;
  int bk = 0;
  for (int k0 = 0; k0 < k; k0 += kGmmChunk) {
    const int nk = min(kGmmChunk, k - k0);
    __syncthreads();
    for (int t = threadIdx.x; t < nk * 10; t += blockDim.x) s_rec[t] = rec[(size_t)(k0 + t / 10) * kGmmRec + t % 10];
    __syncthreads();
    for (int j = 0; j < nk; ++j) {
      const float* r = s_rec + 10 * j;
      const float d0 = x0 - r[0], d1 = x1 - r[1], d2 = x2 - r[2];
      const float t0 = (r[3] * d0 + r[4] * d1) + r[5] * d2;
      const float t1 = (r[4] * d0 + r[6] * d1) + r[7] * d2;
      const float t2 = (r[5] * d0 + r[7] * d1) + r[8] * d2;
      const float s = ((d0 * t0 + d1 * t1) + d2 * t2) + r[9];
      if (s < best) {  // strict: the first minimum (lowest index) stays
        best = s;
        bk = k0 + j;
      }
    }
  }
  double geo = 0.0, iso = 0.0;
  if (ok) {
    // loss terms and gradients in FP64 (the projection onto the unit
    // quaternion's tangent space cancels most of its input)
    const float* r = rec + (size_t)kGmmRec * bk;
    const double nk0 = r[10], nk1 = r[11], nk2 = r[12];
    const double delta = ((x0 - (double)r[0]) * nk0 + (x1 - (double)r[1]) * nk1) + (x2 - (double)r[2]) * nk2;
    // surfel normal: third column of the rotation of the normalised quaternion
    const double q0 = quats[4 * i], q1 = quats[4 * i + 1], q2 = quats[4 * i + 2], q3 = quats[4 * i + 3];
    const double qq = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
    const double rq = qq > 0.0 ? 1.0 / sqrt(qq) : 0.0;
    const double w = q0 * rq, x = q1 * rq, y = q2 * rq, z = q3 * rq;
    const double n0 = 2.0 * (x * z + w * y), n1 = 2.0 * (y * z - w * x), n2 = 1.0 - 2.0 * (x * x + y * y);
    const double dot = (n0 * nk0 + n1 * nk1) + n2 * nk2;
    const double s0 = scales[2 * i], s1 = scales[2 * i + 1];
    geo = fabs(delta) + (double)lambda_n * (1.0 - fabs(dot));
    iso = (s0 - s1) * (s0 - s1);
    const double sd = delta > 0.0 ? 1.0 : (delta < 0.0 ? -1.0 : 0.0);
    d_means[3 * i] = (float)(sd * nk0);
    d_means[3 * i + 1] = (float)(sd * nk1);
    d_means[3 * i + 2] = (float)(sd * nk2);
    d_scales[2 * i] = (float)(2.0 * (s0 - s1));
    d_scales[2 * i + 1] = (float)(-2.0 * (s0 - s1));
    // dL/dn = -lambda_n sign(dot) n_k, through n(w, x, y, z) and q / |q|
    const double sg = dot > 0.0 ? 1.0 : (dot < 0.0 ? -1.0 : 0.0);
    const double g0 = -lambda_n * sg * nk0, g1 = -lambda_n * sg * nk1, g2 = -lambda_n * sg * nk2;
    const double gw = 2.0 * y * g0 - 2.0 * x * g1;
    const double gx = 2.0 * z * g0 - 2.0 * w * g1 - 4.0 * x * g2;
    const double gy = 2.0 * w * g0 + 2.0 * z * g1 - 4.0 * y * g2;
    const double gz = 2.0 * x * g0 + 2.0 * y * g1;
    const double pr = ((gw * w + gx * x) + gy * y) + gz * z;
    d_quats[4 * i] = (float)((gw - w * pr) * rq);
    d_quats[4 * i + 1] = (float)((gx - x * pr) * rq);
    d_quats[4 * i + 2] = (float)((gy - y * pr) * rq);
    d_quats[4 * i + 3] = (float)((gz - z * pr) * rq);
    if (assign) assign[i] = bk;
  }
  const double bg = block_sum_f64(geo, s_red);
  const double bi = block_sum_f64(iso, s_red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = bg;
    part[2 * blockIdx.x + 1] = bi;
  }
}

// One wave: the block sums in block order (lane-strided, then a fixed tree).
__global__ void k_geo_sum(int64_t nb, const double* __restrict__ part, double* __restrict__ out) {
  const int lane = threadIdx.x;
  double g = 0.0, s = 0.0;
  for (int64_t b = lane; b < nb; b += 64) {
    g += part[2 * b];
    s += part[2 * b + 1];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    g += __shfl_xor(g, o, 64);
    s += __shfl_xor(s, o, 64);
  }
  if (lane == 0) {
    out[0] = g;
    out[1] = s;
  }
}

size_t geometry_workspace_bytes(int64_t n, int k) {
  const int64_t nb = cdiv(std::max<int64_t>(n, 1), 256);
  return (((size_t)k * kGmmRec * 4 + 255) & ~(size_t)255) + (size_t)nb * 16;
}

void launch_geometry_loss(const GeometryArgs& a, char* ws, hipStream_t st) {
  const int64_t nb = cdiv(std::max<int64_t>(a.n, 1), 256);
  float* rec = (float*)ws;
  double* part = (double*)(ws + (((size_t)a.k * kGmmRec * 4 + 255) & ~(size_t)255));
  hipLaunchKernelGGL(k_gmm_prep, dim3((unsigned)cdiv(a.k, 64)), dim3(64), 0, st, a.k, a.gmean, a.gcov, a.gweight,
                     rec);
  hipLaunchKernelGGL(k_geo_loss, dim3((unsigned)nb), dim3(256), 0, st, a.n, a.means, a.scales, a.quats, a.k,
                     (const float*)rec, a.lambda_n, a.assign, a.d_means, a.d_scales, a.d_quats, part);
  hipLaunchKernelGGL(k_geo_sum, dim3(1), dim3(64), 0, st, nb, (const double*)part, a.losses);
}

}  // namespace psm
