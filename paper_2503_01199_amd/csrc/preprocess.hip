// Projection of 3-D Gaussians into screen-space records and its backward.
//
// Sec. 3: each primitive {p, Sigma, c, o} becomes {x, y, Sigma_screen, c, o} per
// view. Sigma = R diag(exp(2 s)) R^T from a normalised quaternion; the screen
// covariance is the EWA local-affine projection J W Sigma W^T J^T plus a 0.3 px^2
// low-pass, with the Jacobian evaluated within 1.3x the half field of view; the
// colour is a degree <= 3 real SH expansion at the camera-to-mean direction, plus
// 1/2, clamped at 0; o = sigmoid(logit). The support is where alpha = o G >= 1/255,
// i.e. the ellipse d^T Q d <= 2 ln(255 o); its bounding box gives the tile rect.
//
// This stage is memory-bound (236 B of parameters per Gaussian at SH degree 3), so
// it runs in FP64: on gfx950 FP64 vector math costs half the FP32 rate, which is
// free here, and it lets the records carry the screen mean as a float-float pair
// and the conic in a cancellation-free factored form, which is what keeps the
// FP32 raster within 1e-5 of an FP64 reference at 1600-pixel image widths.
//
// One thread per compact slot; a slot is projected into every view of the frame
// (records r = slot * V + view), so its parameters are read once per frame.
#include <math.h>

#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr int kThreads = 128;
static_assert(kThreads == GSR_CLUSTER, "the SH kernels take one cluster (a run of consecutive Gaussians) per block");

typedef float f32x4 __attribute__((ext_vector_type(4)));

// SH rows (R floats per Gaussian) of a block's consecutive Gaussians move between
// global memory and LDS with coalesced float4 accesses (a wave moves 1 KB per
// instruction), instead of one strided 4- or 16-byte access per thread and row. In
// LDS a row has stride R + 1 floats (odd for R = 12, 48), so the threads' walks
// along their own rows hit distinct banks. Gradient rows leave with streaming
// (non-temporal) stores: nothing in the step reads them again, and written through
// the caches they would evict the scene data that the next frame reads first.
template <int R>
__device__ __forceinline__ void rows_to_lds(float* lds, const float* __restrict__ src, int nrows) {
  constexpr int S = R + 1;
  const int t = threadIdx.x;
  if constexpr (R % 4 == 0) {
    if (nrows == kThreads) {
      const float4* s4 = reinterpret_cast<const float4*>(src);
      float4 v[R / 4];
#pragma unroll
      for (int m = 0; m < R / 4; ++m) v[m] = s4[m * kThreads + t];
#pragma unroll
      for (int m = 0; m < R / 4; ++m) {
        const int e = 4 * (m * kThreads + t);  // 4 floats of one row (R % 4 == 0)
        float* d = lds + (e / R) * S + e % R;
        d[0] = v[m].x;
        d[1] = v[m].y;
        d[2] = v[m].z;
        d[3] = v[m].w;
      }
      return;
    }
  }
  for (int e = t; e < nrows * R; e += kThreads) lds[(e / R) * S + e % R] = src[e];
}

template <int R>
__device__ __forceinline__ void rows_from_lds(float* __restrict__ dst, const float* lds, int nrows) {
  constexpr int S = R + 1;
  const int t = threadIdx.x;
  if constexpr (R % 4 == 0) {
    if (nrows == kThreads) {
      f32x4* d4 = reinterpret_cast<f32x4*>(dst);
#pragma unroll
      for (int m = 0; m < R / 4; ++m) {
        const int e = 4 * (m * kThreads + t);
        const float* s = lds + (e / R) * S + e % R;
        const f32x4 x = {s[0], s[1], s[2], s[3]};
        __builtin_nontemporal_store(x, d4 + m * kThreads + t);
      }
      return;
    }
  }
  for (int e = t; e < nrows * R; e += kThreads) dst[e] = lds[(e / R) * S + e % R];
}

template <int R>
__device__ __forceinline__ void zero_rows(float* __restrict__ dst, int nrows) {
  const int t = threadIdx.x;
  if constexpr (R % 4 == 0) {
    if (nrows == kThreads) {
      f32x4* d4 = reinterpret_cast<f32x4*>(dst);
      const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int m = 0; m < R / 4; ++m) __builtin_nontemporal_store(z, d4 + m * kThreads + t);
      return;
    }
  }
  for (int e = t; e < nrows * R; e += kThreads) dst[e] = 0.0f;
}

struct GaussParams {
  double m[3];
  double s[3];     // scales
  double q[4];     // normalised quaternion
  double qn;       // norm of the input quaternion
  double R[9];     // rotation of q, row-major
  double Sig[6];   // 3-D covariance: xx, xy, xz, yy, yz, zz
  double o;        // activated opacity
};

__device__ inline void load_gaussian(const gsr_scene& sc, int64_t i, GaussParams& g) {
  for (int a = 0; a < 3; ++a) {
    g.m[a] = (double)sc.means[3 * i + a];
    g.s[a] = exp((double)sc.log_scales[3 * i + a]);
  }
  double q[4];
  double nn = 0.0;
  for (int a = 0; a < 4; ++a) {
    q[a] = (double)sc.quats[4 * i + a];
    nn += q[a] * q[a];
  }
  g.qn = sqrt(nn);
  for (int a = 0; a < 4; ++a) g.q[a] = q[a] / g.qn;
  const double w = g.q[0], x = g.q[1], y = g.q[2], z = g.q[3];
  g.R[0] = 1 - 2 * (y * y + z * z); g.R[1] = 2 * (x * y - w * z);     g.R[2] = 2 * (x * z + w * y);
  g.R[3] = 2 * (x * y + w * z);     g.R[4] = 1 - 2 * (x * x + z * z); g.R[5] = 2 * (y * z - w * x);
  g.R[6] = 2 * (x * z - w * y);     g.R[7] = 2 * (y * z + w * x);     g.R[8] = 1 - 2 * (x * x + y * y);
  double L[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) L[3 * r + k] = g.R[3 * r + k] * g.s[k];
  int idx = 0;
  for (int r = 0; r < 3; ++r)
    for (int c = r; c < 3; ++c) {
      g.Sig[idx++] = L[3 * r + 0] * L[3 * c + 0] + L[3 * r + 1] * L[3 * c + 1] + L[3 * r + 2] * L[3 * c + 2];
    }
  g.o = 1.0 / (1.0 + exp(-(double)sc.opacity_logits[i]));
}

__device__ inline double sig(const GaussParams& g, int r, int c) {
  // symmetric access into the packed upper triangle
  if (r > c) {
    const int t = r;
    r = c;
    c = t;
  }
  const int base[3] = {0, 3, 5};
  return g.Sig[base[r] + (c - r)];
}

// Real SH basis of degree <= 3 (orthonormal, no Condon-Shortley phase) at the unit
// direction (x, y, z), index l*l + l + m, and optionally its gradient in R^3.
template <int deg, typename R = double>
__device__ inline void sh_basis(R x, R y, R z, R* Y, R (*dY)[3]) {
  Y[0] = (R)(0.5 * sqrt(1.0 / 3.14159265358979323846));
  if (dY) dY[0][0] = dY[0][1] = dY[0][2] = 0.0;
  if constexpr (deg < 1) return;
  const R c1 = (R)sqrt(3.0 / (4.0 * 3.14159265358979323846));
  Y[1] = c1 * y;
  Y[2] = c1 * z;
  Y[3] = c1 * x;
  if (dY) {
    dY[1][0] = 0; dY[1][1] = c1; dY[1][2] = 0;
    dY[2][0] = 0; dY[2][1] = 0;  dY[2][2] = c1;
    dY[3][0] = c1; dY[3][1] = 0; dY[3][2] = 0;
  }
  if constexpr (deg < 2) return;
  const R xx = x * x, yy = y * y, zz = z * z;
  const R c2a = (R)(0.5 * sqrt(15.0 / 3.14159265358979323846));   // xy, yz, xz
  const R c2b = (R)(0.25 * sqrt(5.0 / 3.14159265358979323846));   // 2z^2 - x^2 - y^2
  const R c2c = (R)(0.25 * sqrt(15.0 / 3.14159265358979323846));  // x^2 - y^2
  Y[4] = c2a * x * y;
  Y[5] = c2a * y * z;
  Y[6] = c2b * (2 * zz - xx - yy);
  Y[7] = c2a * x * z;
  Y[8] = c2c * (xx - yy);
  if (dY) {
    dY[4][0] = c2a * y;      dY[4][1] = c2a * x;       dY[4][2] = 0;
    dY[5][0] = 0;            dY[5][1] = c2a * z;       dY[5][2] = c2a * y;
    dY[6][0] = -2 * c2b * x; dY[6][1] = -2 * c2b * y;  dY[6][2] = 4 * c2b * z;
    dY[7][0] = c2a * z;      dY[7][1] = 0;             dY[7][2] = c2a * x;
    dY[8][0] = 2 * c2c * x;  dY[8][1] = -2 * c2c * y;  dY[8][2] = 0;
  }
  if constexpr (deg < 3) return;
  const R c3a = (R)(0.25 * sqrt(35.0 / (2.0 * 3.14159265358979323846)));  // m = +-3
  const R c3b = (R)(0.5 * sqrt(105.0 / 3.14159265358979323846));          // m = -2
  const R c3c = (R)(0.25 * sqrt(21.0 / (2.0 * 3.14159265358979323846)));  // m = +-1
  const R c3d = (R)(0.25 * sqrt(7.0 / 3.14159265358979323846));           // m = 0
  const R c3e = (R)(0.25 * sqrt(105.0 / 3.14159265358979323846));         // m = 2
  const R f1 = 4 * zz - xx - yy;
  Y[9] = c3a * y * (3 * xx - yy);
  Y[10] = c3b * x * y * z;
  Y[11] = c3c * y * f1;
  Y[12] = c3d * z * (2 * zz - 3 * xx - 3 * yy);
  Y[13] = c3c * x * f1;
  Y[14] = c3e * z * (xx - yy);
  Y[15] = c3a * x * (xx - 3 * yy);
  if (dY) {
    dY[9][0] = c3a * 6 * x * y;           dY[9][1] = c3a * (3 * xx - 3 * yy);   dY[9][2] = 0;
    dY[10][0] = c3b * y * z;              dY[10][1] = c3b * x * z;              dY[10][2] = c3b * x * y;
    dY[11][0] = -2 * c3c * x * y;         dY[11][1] = c3c * (4 * zz - xx - 3 * yy); dY[11][2] = 8 * c3c * y * z;
    dY[12][0] = -6 * c3d * x * z;         dY[12][1] = -6 * c3d * y * z;         dY[12][2] = c3d * (6 * zz - 3 * xx - 3 * yy);
    dY[13][0] = c3c * (4 * zz - 3 * xx - yy); dY[13][1] = -2 * c3c * x * y;    dY[13][2] = 8 * c3c * x * z;
    dY[14][0] = 2 * c3e * x * z;          dY[14][1] = -2 * c3e * y * z;         dY[14][2] = c3e * (xx - yy);
    dY[15][0] = c3a * (3 * xx - 3 * yy);  dY[15][1] = -6 * c3a * x * y;        dY[15][2] = 0;
  }
}

// Gradient on R^3 of P(x, y, z) = sum_k w_k Y_k(x, y, z) for the basis above,
// accumulated term by term (no table of basis gradients is kept).
template <int deg>
__device__ __forceinline__ void sh_weighted_grad(float x, float y, float z, const float* w, float g[3]) {
  g[0] = g[1] = g[2] = 0.0f;
  if constexpr (deg < 1) return;
  const float c1 = (float)sqrt(3.0 / (4.0 * 3.14159265358979323846));
  g[0] += c1 * w[3];
  g[1] += c1 * w[1];
  g[2] += c1 * w[2];
  if constexpr (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  const float c2a = (float)(0.5 * sqrt(15.0 / 3.14159265358979323846));
  const float c2b = (float)(0.25 * sqrt(5.0 / 3.14159265358979323846));
  const float c2c = (float)(0.25 * sqrt(15.0 / 3.14159265358979323846));
  float t;
  t = c2a * w[4]; g[0] += t * y; g[1] += t * x;
  t = c2a * w[5]; g[1] += t * z; g[2] += t * y;
  t = c2b * w[6]; g[0] -= 2 * t * x; g[1] -= 2 * t * y; g[2] += 4 * t * z;
  t = c2a * w[7]; g[0] += t * z; g[2] += t * x;
  t = c2c * w[8]; g[0] += 2 * t * x; g[1] -= 2 * t * y;
  if constexpr (deg < 3) return;
  const float c3a = (float)(0.25 * sqrt(35.0 / (2.0 * 3.14159265358979323846)));
  const float c3b = (float)(0.5 * sqrt(105.0 / 3.14159265358979323846));
  const float c3c = (float)(0.25 * sqrt(21.0 / (2.0 * 3.14159265358979323846)));
  const float c3d = (float)(0.25 * sqrt(7.0 / 3.14159265358979323846));
  const float c3e = (float)(0.25 * sqrt(105.0 / 3.14159265358979323846));
  t = c3a * w[9];  g[0] += t * 6 * x * y; g[1] += t * (3 * xx - 3 * yy);
  t = c3b * w[10]; g[0] += t * y * z; g[1] += t * x * z; g[2] += t * x * y;
  t = c3c * w[11]; g[0] -= t * 2 * x * y; g[1] += t * (4 * zz - xx - 3 * yy); g[2] += t * 8 * y * z;
  t = c3d * w[12]; g[0] -= t * 6 * x * z; g[1] -= t * 6 * y * z; g[2] += t * (6 * zz - 3 * xx - 3 * yy);
  t = c3c * w[13]; g[0] += t * (4 * zz - 3 * xx - yy); g[1] -= t * 2 * x * y; g[2] += t * 8 * x * z;
  t = c3e * w[14]; g[0] += t * 2 * x * z; g[1] -= t * 2 * y * z; g[2] += t * (xx - yy);
  t = c3a * w[15]; g[0] += t * (3 * xx - 3 * yy); g[1] -= t * 6 * x * y;
}

// Camera-side projection of one Gaussian into one view.
struct ViewProj {
  double tx, ty, tz;
  double xt, yt;       // clamped tx/tz, ty/tz
  bool clx, cly;
  double J00, J02, J11, J12;
  double M[6];         // J W
  double cov[3];       // a', b', c' (dilated)
  double det;
  double u, v;
  double dir[3], dist;
};

// Returns false when the Gaussian is dropped by the near plane or a degenerate
// covariance. Camera-space coordinates are formed as ((r0 x + r1 y) + r2 z) + t
// with no fused operations, so the FP32 depth key is a reproducible function of
// the inputs.
__device__ inline bool project_view(const GaussParams& g, const ViewDev& w, ViewProj& p) {
  const double* m = g.m;
  const double R0 = w.R[0], R1 = w.R[1], R2 = w.R[2], R3 = w.R[3], R4 = w.R[4], R5 = w.R[5];
  const double R6 = w.R[6], R7 = w.R[7], R8 = w.R[8];
  p.tx = ((R0 * m[0] + R1 * m[1]) + R2 * m[2]) + (double)w.t[0];
  p.ty = ((R3 * m[0] + R4 * m[1]) + R5 * m[2]) + (double)w.t[1];
  p.tz = ((R6 * m[0] + R7 * m[1]) + R8 * m[2]) + (double)w.t[2];
  if (!(p.tz > (double)w.near_plane)) return false;
  const double fx = w.fx, fy = w.fy;
  const double xr = p.tx / p.tz, yr = p.ty / p.tz;
  p.clx = (xr < -w.limx) || (xr > w.limx);
  p.cly = (yr < -w.limy) || (yr > w.limy);
  p.xt = fmin(fmax(xr, -w.limx), w.limx);
  p.yt = fmin(fmax(yr, -w.limy), w.limy);
  p.J00 = fx / p.tz;
  p.J02 = -fx * p.xt / p.tz;
  p.J11 = fy / p.tz;
  p.J12 = -fy * p.yt / p.tz;
  // M = J W (2x3)
  p.M[0] = p.J00 * R0 + p.J02 * R6;
  p.M[1] = p.J00 * R1 + p.J02 * R7;
  p.M[2] = p.J00 * R2 + p.J02 * R8;
  p.M[3] = p.J11 * R3 + p.J12 * R6;
  p.M[4] = p.J11 * R4 + p.J12 * R7;
  p.M[5] = p.J11 * R5 + p.J12 * R8;
  double SM[2][3];  // Sigma M^T columns
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k)
      SM[r][k] = sig(g, k, 0) * p.M[3 * r + 0] + sig(g, k, 1) * p.M[3 * r + 1] + sig(g, k, 2) * p.M[3 * r + 2];
  const double c00 = p.M[0] * SM[0][0] + p.M[1] * SM[0][1] + p.M[2] * SM[0][2];
  const double c01 = p.M[0] * SM[1][0] + p.M[1] * SM[1][1] + p.M[2] * SM[1][2];
  const double c11 = p.M[3] * SM[1][0] + p.M[4] * SM[1][1] + p.M[5] * SM[1][2];
  p.cov[0] = c00 + kDilation;
  p.cov[1] = c01;
  p.cov[2] = c11 + kDilation;
  p.det = p.cov[0] * p.cov[2] - p.cov[1] * p.cov[1];
  if (!(p.det > 0.0)) return false;
  p.u = fx * p.tx / p.tz + (double)w.cx;
  p.v = fy * p.ty / p.tz + (double)w.cy;
  const double d0 = m[0] - w.campos[0], d1 = m[1] - w.campos[1], d2 = m[2] - w.campos[2];
  p.dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  p.dir[0] = d0 / p.dist;
  p.dir[1] = d1 / p.dist;
  p.dir[2] = d2 / p.dist;
  return true;
}

template <int DEG>
__global__ __launch_bounds__(kThreads) void k_preprocess_fwd(gsr_scene sc, const ViewDev* __restrict__ views,
                                                             int32_t V, int64_t ncap,
                                                             uint32_t* __restrict__ header,
                                                             const uint32_t* __restrict__ cluster_list,
                                                             uint32_t* __restrict__ compact2full,
                                                             Record* __restrict__ rec, uint32_t* __restrict__ dkey,
                                                             uint32_t* __restrict__ tiles,
                                                             ushort4* __restrict__ rect,
                                                             float* __restrict__ grad2d,
                                                             unsigned long long* __restrict__ grad_fx,
                                                             int radius_mode) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  __shared__ float lsh[kThreads * (3 * K + 1)];  // the cluster's SH rows
  if (frame_aborted(header)) return;  // the cluster scan gave up: its list may be garbage
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;  // block = compact slot p (grid covers ncap)
  const uint32_t nvis = header[kHdrVisibleClusters];
  if (j == 0) header[kHdrRecords] = nvis * GSR_CLUSTER * (uint32_t)V;
  const int64_t p = blockIdx.x;
  (void)ncap;
  int64_t i = -1;
  if (p < (int64_t)nvis) {  // uniform over the block
    const int64_t i0 = (int64_t)cluster_list[p] * GSR_CLUSTER;
    rows_to_lds<3 * K>(lsh, sc.sh + i0 * (3 * K), (int)min<int64_t>(kThreads, sc.n - i0));
    __syncthreads();
    i = i0 + threadIdx.x;
    if (i >= sc.n) i = -1;
  }
  compact2full[j] = i < 0 ? 0xffffffffu : (uint32_t)i;
  if (i < 0) {
    for (int v = 0; v < V; ++v) {
      const int64_t r = j * V + v;
      dkey[r] = 0xffffffffu;
      tiles[r] = 0;
      rect[r] = make_ushort4(0, 0, 0, 0);
    }
    return;
  }
  GaussParams g;
  load_gaussian(sc, i, g);
  const float* shp = lsh + threadIdx.x * (3 * K + 1);  // this Gaussian's SH coefficients
  for (int v = 0; v < V; ++v) {
    const int64_t r = j * V + v;
    const ViewDev& w = views[v];
    ViewProj pr;
    bool ok = project_view(g, w, pr) && g.o >= (1.0 / 255.0);
    int x0 = 0, x1 = -1, y0 = 0, y1 = -1;
    if (ok) {
      // support box of d^T Q d <= 2 ln(255 o): half widths sqrt(K cov_xx), sqrt(K cov_yy);
      // or (radius_mode 1) the 3-sigma square, half width ceil(3 sqrt(lambda_max));
      // pixel px covers the centre px + 1/2
      double rx, ry;
      if (radius_mode == 1) {
        const double m = 0.5 * (pr.cov[0] + pr.cov[2]);
        const double lam = m + sqrt(fmax(0.0, m * m - pr.det));
        rx = ry = ceil(3.0 * sqrt(lam));
      } else {
        const double Kq = 2.0 * log(255.0 * g.o);
        rx = sqrt(Kq * pr.cov[0]);
        ry = sqrt(Kq * pr.cov[2]);
      }
      double fx0 = ceil((pr.u - rx) - 0.5), fx1 = floor((pr.u + rx) - 0.5);
      double fy0 = ceil((pr.v - ry) - 0.5), fy1 = floor((pr.v + ry) - 0.5);
      fx0 = fmax(fx0, 0.0);
      fy0 = fmax(fy0, 0.0);
      fx1 = fmin(fx1, (double)(w.width - 1));
      fy1 = fmin(fy1, (double)(w.height - 1));
      if (fx0 > fx1 || fy0 > fy1) {
        ok = false;
      } else {
        const int hl = 8 - w.tile_wl;  // tiles 2^tile_wl wide, 2^hl high
        x0 = (int)fx0 >> w.tile_wl;
        x1 = (int)fx1 >> w.tile_wl;
        y0 = (int)fy0 >> hl;
        y1 = (int)fy1 >> hl;
      }
    }
    if (!ok) {
      dkey[r] = 0xffffffffu;
      tiles[r] = 0;
      rect[r] = make_ushort4(0, 0, 0, 0);
      continue;
    }
    // colour
    double Y[16];
    sh_basis<DEG, double>(pr.dir[0], pr.dir[1], pr.dir[2], Y, nullptr);
    double col[3] = {0.5, 0.5, 0.5};
#pragma unroll
    for (int k = 0; k < K; ++k)
      for (int ch = 0; ch < 3; ++ch) col[ch] += Y[k] * (double)shp[3 * k + ch];
    // conic Q = cov^-1 = (a, b, c); factored exponent in log2 units:
    //   -1/2 d^T Q d = -1/2 a (dx + (b/a) dy)^2 - 1/2 dy^2 / cov_yy
    const double a = pr.cov[2] / pr.det;
    const double c = pr.cov[0] / pr.det;
    const double ratio = -pr.cov[1] / pr.cov[2];
    Record out;
    const float uh = (float)pr.u, vh = (float)pr.v;
    out.r0 = make_float4(uh, vh, (float)(pr.u - (double)uh), (float)(pr.v - (double)vh));
    out.r1 = make_float4((float)(-0.5 * a * kLog2e), (float)ratio, (float)(-0.5 / pr.cov[2] * kLog2e),
                         (float)(-0.125 * c * kLog2e));  // a quarter of the j^2 coefficient
    out.r2 = make_float4((float)g.o, (float)fmax(col[0], 0.0), (float)fmax(col[1], 0.0), (float)fmax(col[2], 0.0));
    rec[r] = out;
    if (grad_fx) {  // cleared for the backward's atomics: fixed-point sums, or FP32 sums
      ulonglong2* q = reinterpret_cast<ulonglong2*>(grad_fx + r * kGrad2D);
#pragma unroll
      for (int k = 0; k < kGrad2D / 2; ++k) q[k] = make_ulonglong2(0ull, 0ull);
    } else {
      float4* g4 = reinterpret_cast<float4*>(grad2d + r * kGrad2D);
      g4[0] = g4[1] = g4[2] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    dkey[r] = __float_as_uint((float)pr.tz);
    tiles[r] = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
    rect[r] = make_ushort4((unsigned short)x0, (unsigned short)x1, (unsigned short)y0, (unsigned short)y1);
  }
}

// Backward of the projection, geometric part: screen-space gradients (grad2d of
// every view) to the mean, log-scale, quaternion and opacity-logit gradients, in
// FP64. One thread per Gaussian in the caller's order; Gaussians that no view
// blends (including those of culled clusters) get zero. The SH coefficients and the
// colour's dependence on the mean through the view direction follow in k_sh_bwd.
// The projection backward's results for Gaussian i (compact slot j): the gradients,
// or, with the fused Adam, the Adam step of its log-scales, quaternion and opacity
// logit in place and its mean gradient, which k_sh_bwd completes, in dmean.
template <bool kAdam>
__device__ __forceinline__ void store_project_grads(const gsr_grads& gr, const AdamDev& adam, float* dmean, int64_t i,
                                                    int64_t j, const float (&gm)[3], const float (&gl)[3],
                                                    const float (&gq)[4], float go) {
  if constexpr (kAdam) {
    const AdamGroupDev& ql = adam.grp[1];
    const AdamGroupDev& qq = adam.grp[2];
    const AdamGroupDev& qo = adam.grp[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float p = ql.p[3 * i + a], m = ql.m[3 * i + a], v = ql.v[3 * i + a];
      adam_float(p, gl[a], m, v, ql.step_head, adam);
      ql.p[3 * i + a] = p, ql.m[3 * i + a] = m, ql.v[3 * i + a] = v;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      float p = qq.p[4 * i + a], m = qq.m[4 * i + a], v = qq.v[4 * i + a];
      adam_float(p, gq[a], m, v, qq.step_head, adam);
      qq.p[4 * i + a] = p, qq.m[4 * i + a] = m, qq.v[4 * i + a] = v;
    }
    {
      float p = qo.p[i], m = qo.m[i], v = qo.v[i];
      adam_float(p, go, m, v, qo.step_head, adam);
      qo.p[i] = p, qo.m[i] = m, qo.v[i] = v;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) dmean[3 * j + a] = gm[a];
  } else {
    // streaming stores but for the mean, to which the SH backward adds its term
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      gr.means[3 * i + a] = gm[a];
      __builtin_nontemporal_store(gl[a], gr.log_scales + 3 * i + a);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) __builtin_nontemporal_store(gq[a], gr.quats + 4 * i + a);
    __builtin_nontemporal_store(go, gr.opacity_logits + i);
  }
}

template <bool kAdam>
__global__ __launch_bounds__(kThreads) void k_project_bwd(
    gsr_scene sc, const ViewDev* __restrict__ views, int32_t V, const uint32_t* __restrict__ header,
    const uint32_t* __restrict__ visible, const uint32_t* __restrict__ cluster_offset,
    const uint32_t* __restrict__ tiles, float* __restrict__ grad2d, const unsigned long long* __restrict__ grad_fx,
    gsr_grads gr, float* __restrict__ S, float* __restrict__ Mst, uint32_t* __restrict__ Cst, AdamDev adam,
    float* __restrict__ dmean, int half) {
  if (frame_aborted(header)) return;  // the frame's scans may be garbage: nothing is written
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= sc.n) return;
  const int64_t c = i / GSR_CLUSTER;
  const bool vis = visible[c] != 0;
  const int64_t j = (int64_t)cluster_offset[c] * GSR_CLUSTER + (i % GSR_CLUSTER);
  double dm[3] = {0, 0, 0};
  double dlogit = 0.0;
  double GS[6] = {0, 0, 0, 0, 0, 0};  // gradient w.r.t. Sigma (packed like Sig)
  double sS = 0.0, sM = 0.0;
  uint32_t sC = 0;
  bool any = false;
  GaussParams g;
  if (vis) {
    for (int v = 0; v < V; ++v) {
      const int64_t r = j * V + v;
      float4* gg4 = reinterpret_cast<float4*>(grad2d + r * kGrad2D);
      if (tiles[r] == 0) {
        if (grad_fx) gg4[0] = gg4[1] = gg4[2] = make_float4(0.f, 0.f, 0.f, 0.f);
        continue;
      }
      float4 q0, q1, q2;
      if (grad_fx) {
        // the fixed-point sums of the deterministic backward, as the FP32 row that the
        // SH backward (and inspection) reads
        float x[kGrad2D];
        const ulonglong2* fq = reinterpret_cast<const ulonglong2*>(grad_fx + r * kGrad2D);
        const int E = grad_exponent(header);
#pragma unroll
        for (int k = 0; k < kGrad2D / 2; ++k) {
          const ulonglong2 w2 = fq[k];
          // slot 9: square sum (scale 2^(2E - 32)); slot 10: fragment count (2^-32)
          const int e0 = 2 * k == 10 ? -kFixedBits : E - kFixedBits;
          const int e1 = 2 * k + 1 == 9 ? 2 * E - kFixedBits : E - kFixedBits;
          x[2 * k] = (float)ldexp((double)(long long)w2.x, e0);
          x[2 * k + 1] = (float)ldexp((double)(long long)w2.y, e1);
        }
        q0 = make_float4(x[0], x[1], x[2], x[3]);
        q1 = make_float4(x[4], x[5], x[6], x[7]);
        q2 = make_float4(x[8], x[9], x[10], x[11]);
        gg4[0] = q0;
        gg4[1] = q1;
        gg4[2] = q2;
      } else {
        q0 = gg4[0];
        q1 = gg4[1];
        q2 = gg4[2];
        if (half) {
          // half_reduction: slots 6 and 7 hold (red, green) and (blue, opacity) as FP16
          // pairs; the FP32 row the SH backward (and inspection) reads is rewritten
          typedef _Float16 h2 __attribute__((ext_vector_type(2)));
          const h2 rg = __builtin_bit_cast(h2, q1.z), bo = __builtin_bit_cast(h2, q1.w);
          q1 = make_float4(q1.x, (float)bo.y, (float)rg.x, (float)rg.y);
          q2.x = (float)bo.x;
          gg4[1] = q1;
          gg4[2] = q2;
        }
      }
      const double du = q0.x, dv = q0.y, da = q0.z, db = q0.w, dc = q1.x, dop = q1.y;
      sS += q2.y;
      sM += dop;
      sC += (uint32_t)q2.z;
      if (!any) {
        load_gaussian(sc, i, g);
        any = true;
      }
      const ViewDev& w = views[v];
      ViewProj p;
      if (!project_view(g, w, p)) continue;
      dlogit += dop * g.o * (1.0 - g.o);
      // conic -> screen covariance: G_cov = -Q G_Q Q, G_Q = [[da, db/2], [db/2, dc]]
      // (one reciprocal per divisor; the products are within an FP64 ulp or two of the
      // quotients, far below the FP32 gradients they feed)
      const double idet = 1.0 / p.det;
      const double qa = p.cov[2] * idet, qb = -p.cov[1] * idet, qc = p.cov[0] * idet;
      const double h = 0.5 * db;
      const double t00 = da * qa + h * qb, t01 = da * qb + h * qc;
      const double t10 = h * qa + dc * qb, t11 = h * qb + dc * qc;
      const double g00 = -(qa * t00 + qb * t10);
      const double g01 = -(qa * t01 + qb * t11);
      const double g11 = -(qb * t01 + qc * t11);
      // cov = M Sigma M^T + 0.3 I: G_Sigma += M^T G_cov M, G_M = 2 G_cov M Sigma
      const double* M = p.M;
      double GM0[3], GM1[3];
      for (int k = 0; k < 3; ++k) {
        GM0[k] = g00 * M[k] + g01 * M[3 + k];
        GM1[k] = g01 * M[k] + g11 * M[3 + k];
      }
      int idx = 0;
      for (int r2 = 0; r2 < 3; ++r2)
        for (int c2 = r2; c2 < 3; ++c2) GS[idx++] += M[r2] * GM0[c2] + M[3 + r2] * GM1[c2];
      double GMf[6];
      for (int k = 0; k < 3; ++k) {
        GMf[k] = 2.0 * (GM0[0] * sig(g, 0, k) + GM0[1] * sig(g, 1, k) + GM0[2] * sig(g, 2, k));
        GMf[3 + k] = 2.0 * (GM1[0] * sig(g, 0, k) + GM1[1] * sig(g, 1, k) + GM1[2] * sig(g, 2, k));
      }
      // M = J W: G_J = G_M W^T; only J00, J02, J11, J12 depend on t
      const float* W = w.R;
      const double gJ00 = GMf[0] * W[0] + GMf[1] * W[1] + GMf[2] * W[2];
      const double gJ02 = GMf[0] * W[6] + GMf[1] * W[7] + GMf[2] * W[8];
      const double gJ11 = GMf[3] * W[3] + GMf[4] * W[4] + GMf[5] * W[5];
      const double gJ12 = GMf[3] * W[6] + GMf[4] * W[7] + GMf[5] * W[8];
      const double fx = w.fx, fy = w.fy, itz = 1.0 / p.tz, itz2 = itz * itz, itz3 = itz2 * itz;
      double dt[3] = {0, 0, 0};
      dt[2] += -gJ00 * fx * itz2 - gJ11 * fy * itz2;
      if (p.clx) {
        dt[2] += gJ02 * fx * p.xt * itz2;
      } else {
        dt[0] += -gJ02 * fx * itz2;
        dt[2] += gJ02 * 2.0 * fx * p.tx * itz3;
      }
      if (p.cly) {
        dt[2] += gJ12 * fy * p.yt * itz2;
      } else {
        dt[1] += -gJ12 * fy * itz2;
        dt[2] += gJ12 * 2.0 * fy * p.ty * itz3;
      }
      // screen mean
      dt[0] += du * fx * itz;
      dt[1] += dv * fy * itz;
      dt[2] += -du * fx * p.tx * itz2 - dv * fy * p.ty * itz2;
      for (int a = 0; a < 3; ++a) dm[a] += (double)W[a] * dt[0] + (double)W[3 + a] * dt[1] + (double)W[6 + a] * dt[2];
    }
  }
  if (kAdam && !vis) return;  // a culled cluster keeps its parameters and moments
  float gl[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f}, gm[3] = {0.f, 0.f, 0.f}, go = 0.f;
  if (!any) {
    store_project_grads<kAdam>(gr, adam, dmean, i, j, gm, gl, gq, go);
    return;
  }
  // Sigma = L L^T, L = R S: G_L = 2 G_Sigma L
  double GL[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int l = 0; l < 3; ++l) {
        const int a = r < l ? r : l, b = r < l ? l : r;
        const int base[3] = {0, 3, 5};
        acc += GS[base[a] + (b - a)] * g.R[3 * l + k] * g.s[k];
      }
      GL[3 * r + k] = 2.0 * acc;
    }
  double GR[9];
  for (int k = 0; k < 3; ++k) {
    double ds = 0.0;
    for (int r = 0; r < 3; ++r) ds += GL[3 * r + k] * g.R[3 * r + k];
    gl[k] = (float)(ds * g.s[k]);
    for (int r = 0; r < 3; ++r) GR[3 * r + k] = GL[3 * r + k] * g.s[k];
  }
  const double w = g.q[0], x = g.q[1], y = g.q[2], z = g.q[3];
  double dq[4];
  dq[0] = 2 * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
  dq[1] = 2 * (y * GR[1] + z * GR[2] + y * GR[3] - 2 * x * GR[4] - w * GR[5] + z * GR[6] + w * GR[7] - 2 * x * GR[8]);
  dq[2] = 2 * (-2 * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] + z * GR[7] - 2 * y * GR[8]);
  dq[3] = 2 * (-2 * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2 * z * GR[4] + y * GR[5] + x * GR[6] + y * GR[7]);
  const double qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
  const double iqn = 1.0 / g.qn;
  for (int a = 0; a < 4; ++a) gq[a] = (float)((dq[a] - g.q[a] * qd) * iqn);
  for (int a = 0; a < 3; ++a) gm[a] = (float)dm[a];
  go = (float)dlogit;
  store_project_grads<kAdam>(gr, adam, dmean, i, j, gm, gl, gq, go);
  if (S) {
    S[i] += (float)sS;
    Mst[i] += (float)sM;
    Cst[i] += sC;
  }
}

// Backward of the SH colour: colour = max(0, sum_k Y_k(dir) f_k + 1/2) per channel,
// dir = (mean - camera centre)/|mean - camera centre|. Writes the coefficient
// gradients and adds the direction term to the mean gradient that k_project_bwd
// wrote. The clamp decision is taken in FP64 like the projection's; the gradients
// accumulate in FP32.
template <int DEG, bool kAdam>
__global__ __launch_bounds__(kThreads) void k_sh_bwd(gsr_scene sc, const ViewDev* __restrict__ views, int32_t V,
                                                     const uint32_t* __restrict__ header,
                                                     const uint32_t* __restrict__ visible,
                                                     const uint32_t* __restrict__ cluster_offset,
                                                     const uint32_t* __restrict__ tiles,
                                                     const float* __restrict__ grad2d, gsr_grads gr, AdamDev adam,
                                                     const float* __restrict__ dmean) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  constexpr int R = 3 * K, S = R + 1;
  __shared__ float lsh[kThreads * S];  // the cluster's SH rows, then their gradients
  if (frame_aborted(header)) return;
  const int t = threadIdx.x;
  const int64_t c = blockIdx.x;  // one cluster per block
  const int64_t i0 = c * GSR_CLUSTER;
  const int nrows = (int)min<int64_t>(kThreads, sc.n - i0);
  float* osh = gr.sh + i0 * R;
  if (visible[c] == 0) {  // a culled cluster: its SH gradient rows are zero (written, not accumulated)
    if (!kAdam) zero_rows<R>(osh, nrows);  // or, with the fused Adam, its parameters stay as they are
    return;
  }
  rows_to_lds<R>(lsh, sc.sh + i0 * R, nrows);
  __syncthreads();
  const int64_t i = i0 + t;
  const float* f = lsh + t * S;  // this Gaussian's SH coefficients
  float gsh[R];
#pragma unroll
  for (int q = 0; q < R; ++q) gsh[q] = 0.0f;
  float dmu[3] = {0.f, 0.f, 0.f};
  bool written = false;
  if (t < nrows) {
    const int64_t j = (int64_t)cluster_offset[c] * GSR_CLUSTER + t;
    const double m0 = sc.means[3 * i], m1 = sc.means[3 * i + 1], m2 = sc.means[3 * i + 2];
    for (int v = 0; v < V; ++v) {
      const int64_t r = j * V + v;
      if (tiles[r] == 0) continue;
      const float4* gg4 = reinterpret_cast<const float4*>(grad2d + r * kGrad2D);
      const float4 q1 = gg4[1], q2 = gg4[2];
      const float dcol[3] = {q1.z, q1.w, q2.x};
      const ViewDev& w = views[v];
      const double d0 = m0 - w.campos[0], d1 = m1 - w.campos[1], d2 = m2 - w.campos[2];
      const double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      const double x = d0 / dist, y = d1 / dist, z = d2 / dist;
      float gc[3];
      {
        double Y[16];
        sh_basis<DEG, double>(x, y, z, Y, nullptr);
        double raw[3] = {0.5, 0.5, 0.5};
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) raw[ch] += Y[k] * (double)f[3 * k + ch];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) gc[ch] = raw[ch] < 0.0 ? 0.0f : dcol[ch];
      }
      const float xf = (float)x, yf = (float)y, zf = (float)z;
      float Yf[16];
      sh_basis<DEG, float>(xf, yf, zf, Yf, nullptr);
      // d colour / d f_k = Y_k, summed over the views
#pragma unroll
      for (int q = 0; q < R; ++q) gsh[q] += gc[q % 3] * Yf[q / 3];
      written = true;
      if constexpr (DEG > 0) {
        // d colour / d dir = grad of sum_k (sum_ch gc_ch f_k,ch) Y_k
        float wk[16];
#pragma unroll
        for (int k = 0; k < K; ++k) wk[k] = gc[0] * f[3 * k] + gc[1] * f[3 * k + 1] + gc[2] * f[3 * k + 2];
        float ddir[3];
        sh_weighted_grad<DEG>(xf, yf, zf, wk, ddir);
        const float dd = xf * ddir[0] + yf * ddir[1] + zf * ddir[2];
        const float inv = (float)(1.0 / dist);
        dmu[0] += (ddir[0] - xf * dd) * inv;
        dmu[1] += (ddir[1] - yf * dd) * inv;
        dmu[2] += (ddir[2] - zf * dd) * inv;
      }
    }
  }
  __syncthreads();  // every thread has read its coefficients: the rows now take the gradients
  float* orow = lsh + t * S;
#pragma unroll
  for (int q = 0; q < R; ++q) orow[q] = gsh[q];
  __syncthreads();
  if constexpr (kAdam) {
    // the cluster's SH slice, coalesced: gradient from LDS, parameter and moments from HBM
    const AdamGroupDev q = adam.grp[4];
    const int64_t base = i0 * R;
    for (int e = t; e < nrows * R; e += kThreads) {
      const int row = e / R, col = e - row * R;
      float pv = q.p[base + e], mv = q.m[base + e], vv = q.v[base + e];
      adam_float(pv, lsh[row * S + col], mv, vv, col < q.head ? q.step_head : q.step_rest, adam);
      q.p[base + e] = pv;
      q.m[base + e] = mv;
      q.v[base + e] = vv;
    }
    if (t < nrows) {  // the mean: the projection's part plus the colour's
      const int64_t j = (int64_t)cluster_offset[c] * GSR_CLUSTER + t;
      const AdamGroupDev qm = adam.grp[0];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        float gmv = dmean[3 * j + a];
        if (DEG > 0 && written) gmv += dmu[a];
        float pv = qm.p[3 * i + a], mv = qm.m[3 * i + a], vv = qm.v[3 * i + a];
        adam_float(pv, gmv, mv, vv, qm.step_head, adam);
        qm.p[3 * i + a] = pv;
        qm.m[3 * i + a] = mv;
        qm.v[3 * i + a] = vv;
      }
    }
  } else {
    rows_from_lds<R>(osh, lsh, nrows);
    if (DEG > 0 && written) {
      float* om = gr.means + 3 * i;
      om[0] += dmu[0];
      om[1] += dmu[1];
      om[2] += dmu[2];
    }
  }
}

__global__ void k_variance(const float* __restrict__ S, const float* __restrict__ M, const uint32_t* __restrict__ C,
                           int64_t n, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double c = (double)C[i];
  const double m = (double)M[i];
  out[i] = c > 0.0 ? (float)((double)S[i] - m * m / c) : 0.0f;
}

// Streaming loads and stores (non-temporal): every value is touched once, and the
// gradient planes are read back by the backward raster only after the caches have
// turned over.
__global__ void k_l1_grad(const f32x4* __restrict__ img, const f32x4* __restrict__ w,
                          const f32x4* __restrict__ gt, int64_t n4, f32x4* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
    const f32x4 a = __builtin_nontemporal_load(img + i), b = __builtin_nontemporal_load(w + i),
                c = __builtin_nontemporal_load(gt + i);
    f32x4 r;
    r.x = a.x > c.x ? b.x : (a.x < c.x ? -b.x : 0.0f);
    r.y = a.y > c.y ? b.y : (a.y < c.y ? -b.y : 0.0f);
    r.z = a.z > c.z ? b.z : (a.z < c.z ? -b.z : 0.0f);
    r.w = a.w > c.w ? b.w : (a.w < c.w ? -b.w : 0.0f);
    __builtin_nontemporal_store(r, out + i);
  }
}

__global__ void k_l1_grad_tail(const float* __restrict__ img, const float* __restrict__ w,
                               const float* __restrict__ gt, int64_t beg, int64_t n, float* __restrict__ out) {
  for (int64_t i = beg + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = img[i] > gt[i] ? w[i] : (img[i] < gt[i] ? -w[i] : 0.0f);
}

}  // namespace

void launch_l1_grad(const float* image, const float* w, const float* gt, int64_t n, float* out, hipStream_t s) {
  if (n <= 0) return;
  const bool aligned = (((uintptr_t)image | (uintptr_t)w | (uintptr_t)gt | (uintptr_t)out) & 15) == 0;
  const int64_t n4 = aligned ? n / 4 : 0;
  if (n4 > 0) {
    int64_t g = (n4 + 255) / 256;
    if (g > 8192) g = 8192;
    k_l1_grad<<<(unsigned)g, 256, 0, s>>>(reinterpret_cast<const f32x4*>(image), reinterpret_cast<const f32x4*>(w),
                                          reinterpret_cast<const f32x4*>(gt), n4, reinterpret_cast<f32x4*>(out));
  }
  const int64_t rest = n - 4 * n4;
  if (rest > 0) {
    int64_t g = (rest + 255) / 256;
    if (g > 8192) g = 8192;
    k_l1_grad_tail<<<(unsigned)g, 256, 0, s>>>(image, w, gt, 4 * n4, n, out);
  }
}

void launch_preprocess_fwd(const gsr_scene& sc, const Frame& f, hipStream_t s) {
  if (f.ncap <= 0) return;
  const unsigned grid = (unsigned)((f.ncap + kThreads - 1) / kThreads);
#define GSR_PRE_FWD(D)                                                                                          \
  k_preprocess_fwd<D><<<grid, kThreads, 0, s>>>(sc, f.views, f.V, f.ncap, f.header, f.cluster_list, f.compact2full, \
                                                f.rec, f.dkey, f.tiles_touched, f.rect, f.grad2d, f.grad2d_fx, \
                                                f.radius_mode)
  switch (sc.sh_degree) {
    case 0: GSR_PRE_FWD(0); break;
    case 1: GSR_PRE_FWD(1); break;
    case 2: GSR_PRE_FWD(2); break;
    default: GSR_PRE_FWD(3); break;
  }
#undef GSR_PRE_FWD
}

void launch_preprocess_bwd(const gsr_scene& sc, const Frame& f, const gsr_grads& g, const gsr_stats* stats,
                           const AdamDev* adam, bool half, hipStream_t s) {
  if (sc.n <= 0) return;
  const unsigned grid = (unsigned)((sc.n + kThreads - 1) / kThreads);
  const AdamDev none{};
  const AdamDev& a = adam ? *adam : none;
  if (adam)
    k_project_bwd<true><<<grid, kThreads, 0, s>>>(sc, f.views, f.V, f.header, f.cluster_visible, f.cluster_offset,
                                                  f.tiles_touched, f.grad2d, f.grad2d_fx, g,
                                                  stats ? stats->S : nullptr, stats ? stats->M : nullptr,
                                                  stats ? stats->C : nullptr, a, f.dmean, half ? 1 : 0);
  else
    k_project_bwd<false><<<grid, kThreads, 0, s>>>(sc, f.views, f.V, f.header, f.cluster_visible, f.cluster_offset,
                                                   f.tiles_touched, f.grad2d, f.grad2d_fx, g,
                                                   stats ? stats->S : nullptr, stats ? stats->M : nullptr,
                                                   stats ? stats->C : nullptr, a, f.dmean, half ? 1 : 0);
#define GSR_SH_BWD(D)                                                                                            \
  if (adam)                                                                                                      \
    k_sh_bwd<D, true><<<grid, kThreads, 0, s>>>(sc, f.views, f.V, f.header, f.cluster_visible, f.cluster_offset,           \
                                                f.tiles_touched, f.grad2d, g, a, f.dmean);                       \
  else                                                                                                           \
    k_sh_bwd<D, false><<<grid, kThreads, 0, s>>>(sc, f.views, f.V, f.header, f.cluster_visible, f.cluster_offset,          \
                                                 f.tiles_touched, f.grad2d, g, a, f.dmean)
  switch (sc.sh_degree) {
    case 0: GSR_SH_BWD(0); break;
    case 1: GSR_SH_BWD(1); break;
    case 2: GSR_SH_BWD(2); break;
    default: GSR_SH_BWD(3); break;
  }
#undef GSR_SH_BWD
}

void launch_variance(const float* S, const float* M, const uint32_t* C, int64_t n, float* out, hipStream_t s) {
  if (n <= 0) return;
  k_variance<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(S, M, C, n, out);
}

}  // namespace gsr
