// FP64 CPU reference ("the oracle") for the differentiable tile-based Gaussian
// rasterizer of LiteGS (arXiv 2503.01199).
//
// THIS IS TEST INFRASTRUCTURE. Only the test suite, the package's smoke check and
// the CPU-baseline leg of the benchmark load it. The GPU library never links,
// imports or calls anything here, and this file shares no code, header, table
// or constant generator with it.
//
// The file states the plain definition of what the rasterizer computes, in
// double precision, with no tiling, fusion or reordering beyond what the
// definition needs. Section references are to the paper:
//   Sec. 3, Eq. (1)  front-to-back alpha compositing with T_i = T_{i-1}(1-a_{i-1})
//   Sec. 3, Eq. (2)  2-D Gaussian G = exp(-1/2 d^T Q d), Q = inverse screen cov.
//   Sec. 3, Eq. (3)  dL/dc = sum over tiles and pixels of dL/dI * T * alpha
//   Sec. 3.2.1       Morton codes (normalise to unit cube, 2^21-1, interleave)
//   Sec. 3.2.2       clusters of 128 consecutive primitives with an AABB
//   Sec. 3.3         opacity-gradient statistic S_i, M_i, C_i and S - M^2/C
//   App. A.2, Eq. (7)-(9)  (a,b,c) form of the exponent and its scanline split
// Points on which the paper is silent (projection, pixel centres, alpha/T
// thresholds, support radius, ...) take one reading each, restated where it is
// used.
//
// Parity pins: every function here is pinned by tests under tests/ (closed
// forms, invariants, brute force, finite differences, library routines).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Constants fixed by the readings (not by the paper's text):
//   alpha skip below 1/255, alpha clamp at 0.99, stop when T would drop below
//   1e-4, screen-space low-pass dilation 0.3 px^2, Jacobian clamp 1.3 x half FoV.
constexpr double kAlphaMin = 1.0 / 255.0;
constexpr double kAlphaMax = 0.99;
constexpr double kTMin = 1e-4;
constexpr double kDilation = 0.3;
constexpr double kFovClamp = 1.3;
constexpr int kTilePixels = 256;  // pixels per tile: 16x16 by default, or 4x64, 8x32, 32x8, 64x4
constexpr double kPi = 3.14159265358979323846;

// Fragility tolerances: a discrete decision within this distance of its
// threshold may legitimately come out differently in FP32.
constexpr double kFragAlpha = 2e-5;   // |ln(255 * o * G)|
constexpr double kFragClamp = 2e-5;   // |o*G/0.99 - 1|
constexpr double kFragT = 1e-4;       // |T'/1e-4 - 1|
constexpr double kFragRect = 1e-9;    // pixels, distance of a rect edge to an integer

struct Camera {
  int W, H;
  double fx, fy, cx, cy;
  double R[9];  // world -> camera rotation, row-major
  double t[3];
  double near_plane;
  double bg[3];
  int radius_mode;  // tile membership: 0 the alpha >= 1/255 ellipse's box, 1 the 3-sigma square
  int tw, th;       // tile width and height in pixels (tw th = 256)
};

Camera unpack_camera(const double* c) {
  Camera k;
  k.W = (int)c[0];
  k.H = (int)c[1];
  k.fx = c[2]; k.fy = c[3]; k.cx = c[4]; k.cy = c[5];
  for (int i = 0; i < 9; ++i) k.R[i] = c[6 + i];
  for (int i = 0; i < 3; ++i) k.t[i] = c[15 + i];
  k.near_plane = c[18];
  for (int i = 0; i < 3; ++i) k.bg[i] = c[19 + i];
  k.radius_mode = (int)c[22];
  k.tw = c[23] > 0 ? (int)c[23] : 16;
  k.th = kTilePixels / k.tw;
  return k;
}

// ---------------------------------------------------------------------------
// Real spherical harmonics up to degree 3 (orthonormal on the unit sphere, no
// Condon-Shortley phase), index k = l*l + l + m. The normalisation constants are
// the closed forms sqrt((2l+1)/(4 pi) * (l-|m|)!/(l+|m|)!) * (2 for m != 0)^(1/2)
// written out per function. Each Y_k is given as a harmonic polynomial in
// (x, y, z) so that its gradient on R^3 is well defined; on the unit sphere the
// values are the textbook ones.
struct SH {
  double Y[16];
  double dY[16][3];
};

void sh_eval(int deg, double x, double y, double z, SH& s) {
  std::memset(&s, 0, sizeof(s));
  const double c0 = 0.5 * std::sqrt(1.0 / kPi);
  s.Y[0] = c0;
  if (deg < 1) return;
  const double c1 = std::sqrt(3.0 / (4.0 * kPi));
  s.Y[1] = c1 * y; s.dY[1][1] = c1;
  s.Y[2] = c1 * z; s.dY[2][2] = c1;
  s.Y[3] = c1 * x; s.dY[3][0] = c1;
  if (deg < 2) return;
  const double c2a = 0.5 * std::sqrt(15.0 / kPi);
  const double c2b = 0.25 * std::sqrt(5.0 / kPi);
  const double c2c = 0.25 * std::sqrt(15.0 / kPi);
  s.Y[4] = c2a * x * y;             s.dY[4][0] = c2a * y; s.dY[4][1] = c2a * x;
  s.Y[5] = c2a * y * z;             s.dY[5][1] = c2a * z; s.dY[5][2] = c2a * y;
  s.Y[6] = c2b * (2 * z * z - x * x - y * y);
  s.dY[6][0] = -2 * c2b * x; s.dY[6][1] = -2 * c2b * y; s.dY[6][2] = 4 * c2b * z;
  s.Y[7] = c2a * x * z;             s.dY[7][0] = c2a * z; s.dY[7][2] = c2a * x;
  s.Y[8] = c2c * (x * x - y * y);   s.dY[8][0] = 2 * c2c * x; s.dY[8][1] = -2 * c2c * y;
  if (deg < 3) return;
  const double c3a = 0.25 * std::sqrt(35.0 / (2.0 * kPi));
  const double c3b = 0.5 * std::sqrt(105.0 / kPi);
  const double c3c = 0.25 * std::sqrt(21.0 / (2.0 * kPi));
  const double c3d = 0.25 * std::sqrt(7.0 / kPi);
  const double c3e = 0.25 * std::sqrt(105.0 / kPi);
  // m = -3: y (3x^2 - y^2)
  s.Y[9] = c3a * y * (3 * x * x - y * y);
  s.dY[9][0] = c3a * 6 * x * y; s.dY[9][1] = c3a * (3 * x * x - 3 * y * y);
  // m = -2: x y z
  s.Y[10] = c3b * x * y * z;
  s.dY[10][0] = c3b * y * z; s.dY[10][1] = c3b * x * z; s.dY[10][2] = c3b * x * y;
  // m = -1: y (4z^2 - x^2 - y^2)
  s.Y[11] = c3c * y * (4 * z * z - x * x - y * y);
  s.dY[11][0] = c3c * (-2 * x * y);
  s.dY[11][1] = c3c * (4 * z * z - x * x - 3 * y * y);
  s.dY[11][2] = c3c * 8 * y * z;
  // m = 0: z (2z^2 - 3x^2 - 3y^2)
  s.Y[12] = c3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
  s.dY[12][0] = c3d * (-6 * x * z); s.dY[12][1] = c3d * (-6 * y * z);
  s.dY[12][2] = c3d * (6 * z * z - 3 * x * x - 3 * y * y);
  // m = 1: x (4z^2 - x^2 - y^2)
  s.Y[13] = c3c * x * (4 * z * z - x * x - y * y);
  s.dY[13][0] = c3c * (4 * z * z - 3 * x * x - y * y);
  s.dY[13][1] = c3c * (-2 * x * y);
  s.dY[13][2] = c3c * 8 * x * z;
  // m = 2: z (x^2 - y^2)
  s.Y[14] = c3e * z * (x * x - y * y);
  s.dY[14][0] = c3e * 2 * x * z; s.dY[14][1] = -c3e * 2 * y * z; s.dY[14][2] = c3e * (x * x - y * y);
  // m = 3: x (x^2 - 3y^2)
  s.Y[15] = c3a * x * (x * x - 3 * y * y);
  s.dY[15][0] = c3a * (3 * x * x - 3 * y * y); s.dY[15][1] = c3a * (-6 * x * y);
}

// ---------------------------------------------------------------------------
// Per (Gaussian, view) projected state: the screen-space primitive
// {x, y, Sigma_screen, c, o} of Sec. 3 plus what the backward needs.
struct Proj {
  int valid;          // passes near plane, det > 0, o >= 1/255 and has a non-empty footprint
  double o;           // sigmoid(opacity logit)
  double s[3];        // exp(log_scale)
  double q[4];        // normalised quaternion (w, x, y, z)
  double qnorm;
  double Rq[9];       // rotation of the quaternion
  double Sig[9];      // 3-D covariance R S^2 R^T
  double tcam[3];     // W mu + t
  double xt, yt;      // tx/tz and ty/tz after the Jacobian clamp
  int clampx, clampy; // 1 where the clamp was active
  double J[6];        // 2x3 EWA Jacobian
  double M[6];        // J W, 2x3
  double cov[3];      // screen covariance (a', b', c') incl. dilation
  double conic[3];    // (a, b, c) = inverse of cov
  double u, v;        // screen mean (pixel centres at integer + 1/2)
  double dir[3];      // unit view direction camera -> mean
  double dist;        // |mu - C|
  double rgb_raw[3];  // sum_k Y_k f_k + 1/2 before the clamp at 0
  double rgb[3];
  float depth32;      // t_z rounded to FP32: the depth ordering key
  int pxr[4];         // pixel footprint [x0, x1] x [y0, y1] inclusive, clipped
  int rect[4];        // tile rect [x0, x1] x [y0, y1] inclusive
  int tiles;          // tiles touched
  int rect_fragile;   // a footprint edge lies within kFragRect of a pixel-centre boundary
};

struct Scene {
  int64_t n;
  int deg, K;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* logits;
  const float* sh;
};

void quat_to_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

// Projection of one Gaussian into one view (Sec. 3: "the Gaussian primitive
// projected into screen space"). The EWA local-affine projection, dilation and
// clamp follow the 3DGS projection the paper builds on.
void project(const Scene& sc, int64_t i, const Camera& cam, Proj& p) {
  std::memset(&p, 0, sizeof(p));
  const float* mu = sc.means + 3 * i;
  const double mx = mu[0], my = mu[1], mz = mu[2];
  p.o = 1.0 / (1.0 + std::exp(-(double)sc.logits[i]));
  for (int k = 0; k < 3; ++k) p.s[k] = std::exp((double)sc.log_scales[3 * i + k]);
  double qn = 0;
  for (int k = 0; k < 4; ++k) qn += (double)sc.quats[4 * i + k] * (double)sc.quats[4 * i + k];
  qn = std::sqrt(qn);
  p.qnorm = qn;
  for (int k = 0; k < 4; ++k) p.q[k] = (double)sc.quats[4 * i + k] / qn;
  quat_to_rot(p.q, p.Rq);
  // Sigma = R S^2 R^T
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += p.Rq[3 * r + k] * p.s[k] * p.s[k] * p.Rq[3 * c + k];
      p.Sig[3 * r + c] = acc;
    }
  const double* W = cam.R;
  // Camera-space position. t_z is formed in this exact order so that its FP32
  // rounding (the depth key) is a reproducible function of the inputs.
  p.tcam[0] = ((W[0] * mx + W[1] * my) + W[2] * mz) + cam.t[0];
  p.tcam[1] = ((W[3] * mx + W[4] * my) + W[5] * mz) + cam.t[1];
  p.tcam[2] = ((W[6] * mx + W[7] * my) + W[8] * mz) + cam.t[2];
  p.depth32 = (float)p.tcam[2];
  const double tx = p.tcam[0], ty = p.tcam[1], tz = p.tcam[2];
  if (!(tz > cam.near_plane)) return;
  const double limx = kFovClamp * (double)cam.W / (2.0 * cam.fx);
  const double limy = kFovClamp * (double)cam.H / (2.0 * cam.fy);
  double xr = tx / tz, yr = ty / tz;
  p.clampx = (xr < -limx || xr > limx);
  p.clampy = (yr < -limy || yr > limy);
  p.xt = std::min(std::max(xr, -limx), limx);
  p.yt = std::min(std::max(yr, -limy), limy);
  p.J[0] = cam.fx / tz; p.J[1] = 0;            p.J[2] = -cam.fx * p.xt / tz;
  p.J[3] = 0;           p.J[4] = cam.fy / tz;  p.J[5] = -cam.fy * p.yt / tz;
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += p.J[3 * r + k] * W[3 * k + c];
      p.M[3 * r + c] = acc;
    }
  double cv[4] = {0, 0, 0, 0};
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      double acc = 0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc += p.M[3 * r + k] * p.Sig[3 * k + l] * p.M[3 * c + l];
      cv[2 * r + c] = acc;
    }
  p.cov[0] = cv[0] + kDilation;
  p.cov[1] = cv[1];
  p.cov[2] = cv[3] + kDilation;
  const double det = p.cov[0] * p.cov[2] - p.cov[1] * p.cov[1];
  if (!(det > 0)) return;
  p.conic[0] = p.cov[2] / det;
  p.conic[1] = -p.cov[1] / det;
  p.conic[2] = p.cov[0] / det;
  p.u = cam.fx * tx / tz + cam.cx;
  p.v = cam.fy * ty / tz + cam.cy;
  // View-dependent colour from the SH coefficients.
  const double C[3] = {-(W[0] * cam.t[0] + W[3] * cam.t[1] + W[6] * cam.t[2]),
                       -(W[1] * cam.t[0] + W[4] * cam.t[1] + W[7] * cam.t[2]),
                       -(W[2] * cam.t[0] + W[5] * cam.t[1] + W[8] * cam.t[2])};
  double d[3] = {mx - C[0], my - C[1], mz - C[2]};
  p.dist = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int k = 0; k < 3; ++k) p.dir[k] = d[k] / p.dist;
  SH s;
  sh_eval(sc.deg, p.dir[0], p.dir[1], p.dir[2], s);
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0;
    for (int k = 0; k < sc.K; ++k) acc += s.Y[k] * (double)sc.sh[(i * sc.K + k) * 3 + ch];
    p.rgb_raw[ch] = acc + 0.5;
    p.rgb[ch] = p.rgb_raw[ch] < 0 ? 0.0 : p.rgb_raw[ch];
  }
  if (p.o < kAlphaMin) return;
  auto near_int = [](double a) { return std::fabs(a - std::nearbyint(a)) < kFragRect; };
  // Support (App. A.1 tile culling: tiles where the Gaussian has decayed to almost
  // nothing are left out). radius_mode 0: alpha = min(0.99, o G) >= 1/255 exactly
  // where the quadratic form d^T Q d <= 2 ln(255 o); the axis-aligned box of that
  // ellipse has half widths sqrt(2 ln(255 o) cov_xx) and sqrt(2 ln(255 o) cov_yy).
  // radius_mode 1: the square of half width r = ceil(3 sqrt(lambda_max)), lambda_max
  // the larger eigenvalue of the screen covariance (the 3-sigma bound). A pixel
  // (px, py) has its centre at (px + 1/2, py + 1/2).
  double rx, ry;
  if (cam.radius_mode == 1) {
    const double m = 0.5 * (p.cov[0] + p.cov[2]);
    const double lam = m + std::sqrt(std::max(0.0, m * m - det));
    const double r3 = 3.0 * std::sqrt(lam);
    rx = ry = std::ceil(r3);
    p.rect_fragile = near_int(r3);
  } else {
    const double Kq = 2.0 * std::log(255.0 * p.o);
    rx = std::sqrt(Kq * p.cov[0]);
    ry = std::sqrt(Kq * p.cov[2]);
  }
  const double ex0 = p.u - rx - 0.5, ex1 = p.u + rx - 0.5;
  const double ey0 = p.v - ry - 0.5, ey1 = p.v + ry - 0.5;
  p.rect_fragile = p.rect_fragile || near_int(ex0) || near_int(ex1) || near_int(ey0) || near_int(ey1);
  double x0 = std::ceil(ex0), x1 = std::floor(ex1), y0 = std::ceil(ey0), y1 = std::floor(ey1);
  x0 = std::max(x0, 0.0); y0 = std::max(y0, 0.0);
  x1 = std::min(x1, (double)(cam.W - 1)); y1 = std::min(y1, (double)(cam.H - 1));
  if (x0 > x1 || y0 > y1) return;
  p.pxr[0] = (int)x0; p.pxr[1] = (int)x1; p.pxr[2] = (int)y0; p.pxr[3] = (int)y1;
  p.rect[0] = p.pxr[0] / cam.tw; p.rect[1] = p.pxr[1] / cam.tw;
  p.rect[2] = p.pxr[2] / cam.th; p.rect[3] = p.pxr[3] / cam.th;
  p.tiles = (p.rect[1] - p.rect[0] + 1) * (p.rect[3] - p.rect[2] + 1);
  p.valid = 1;
  if (cam.radius_mode == 1) {
    // The 3-sigma square can cut through the alpha >= 1/255 set, so membership is
    // no longer implied by alpha: the rasterizer evaluates a Gaussian at every
    // pixel of the tiles its rect covers, and nowhere else. The pixel footprint
    // becomes those tiles' pixels, which every candidate list below applies.
    p.pxr[0] = p.rect[0] * cam.tw;
    p.pxr[1] = std::min(p.rect[1] * cam.tw + cam.tw - 1, cam.W - 1);
    p.pxr[2] = p.rect[2] * cam.th;
    p.pxr[3] = std::min(p.rect[3] * cam.th + cam.th - 1, cam.H - 1);
  }
}

// Exponent of Eq. (2)/(7) at pixel (px, py): E = -1/2 (a dx^2 + 2 b dx dy + c dy^2),
// d = (u - px - 1/2, v - py - 1/2).
inline double exponent(const Proj& p, int px, int py, double& dx, double& dy) {
  dx = p.u - (px + 0.5);
  dy = p.v - (py + 0.5);
  return -0.5 * (p.conic[0] * dx * dx + 2 * p.conic[1] * dx * dy + p.conic[2] * dy * dy);
}

// One entry of a pixel's walk.
struct Frag {
  int64_t g;     // Gaussian index
  int pos;       // position in the list the pixel walks
  double G, a_raw, alpha, T;  // T before this fragment
  double dx, dy;
};

struct PixelResult {
  double rgb[3];
  double T;
  int n_contrib;    // position of the last blended entry + 1 (0 if none)
  int n_blended;
  int64_t last;     // Gaussian of the last blended entry (-1 if none)
  int64_t stop;     // Gaussian whose blend would have taken T below 1e-4 (-1 if the list ran out)
  std::vector<Frag> blended;
  std::vector<int64_t> fragile_at;  // Gaussians whose decision here is within rounding
};

bool depth_less(const std::vector<Proj>& P, int64_t a, int64_t b) {
  uint32_t da, db;
  std::memcpy(&da, &P[a].depth32, 4);
  std::memcpy(&db, &P[b].depth32, 4);
  if (da != db) return da < db;
  return a < b;
}

// Eq. (1) with the reading's thresholds: walk the depth-ordered list front to
// back; skip alpha < 1/255; clamp alpha at 0.99; the entry whose blend would
// take T below 1e-4 is not blended and ends the walk.
void composite(const std::vector<Proj>& P, const std::vector<int64_t>& list, int px, int py,
               const Camera& cam, bool keep, PixelResult& r) {
  r.rgb[0] = r.rgb[1] = r.rgb[2] = 0;
  r.T = 1.0;
  r.n_contrib = 0;
  r.n_blended = 0;
  r.last = -1;
  r.stop = -1;
  r.blended.clear();
  r.fragile_at.clear();
  for (int pos = 0; pos < (int)list.size(); ++pos) {
    const Proj& p = P[list[pos]];
    double dx, dy;
    const double E = exponent(p, px, py, dx, dy);
    const double G = std::exp(E);
    const double araw = p.o * G;
    bool frag = std::fabs(std::log(255.0 * araw)) < kFragAlpha;
    if (araw < kAlphaMin) {
      if (frag) r.fragile_at.push_back(list[pos]);
      continue;
    }
    frag = frag || std::fabs(araw / kAlphaMax - 1.0) < kFragClamp;
    const double alpha = araw <= kAlphaMax ? araw : kAlphaMax;
    const double Tn = r.T * (1.0 - alpha);
    frag = frag || std::fabs(Tn / kTMin - 1.0) < kFragT;
    if (frag) r.fragile_at.push_back(list[pos]);
    if (Tn < kTMin) {
      r.stop = list[pos];
      break;
    }
    if (keep) r.blended.push_back(Frag{list[pos], pos, G, araw, alpha, r.T, dx, dy});
    for (int ch = 0; ch < 3; ++ch) r.rgb[ch] += r.T * alpha * p.rgb[ch];
    r.T = Tn;
    r.n_contrib = pos + 1;
    r.n_blended++;
    r.last = list[pos];
  }
  for (int ch = 0; ch < 3; ++ch) r.rgb[ch] += r.T * cam.bg[ch];
}

// Candidate lists. mode 0: every valid Gaussian (brute force, no filter);
// mode 1: Gaussians whose pixel footprint contains the pixel (an exact superset
// of the alpha >= 1/255 set); mode 2: the pixel's tile list, i.e. every
// Gaussian whose tile rect covers the tile, in (depth, index) order. All three
// give the same image; mode 2 gives list positions comparable to a tiled walk.
struct Lists {
  int mode;
  bool membership;  // radius_mode 1: a Gaussian belongs to the pixels of its rect's tiles only
  std::vector<int64_t> all;                  // mode 0, depth-sorted
  std::vector<std::vector<int64_t>> rows;    // mode 1, per row (unsorted)
  std::vector<std::vector<int64_t>> tiles;   // mode 2, per tile, depth-sorted
  int tx, ty;  // mode 2: tiles per row and column
  int tw, th;  // mode 2: tile width and height in pixels
};

void build_lists(const std::vector<Proj>& P, const Camera& cam, int mode, int y_lo, int y_hi, Lists& L) {
  L.mode = mode;
  L.membership = cam.radius_mode == 1;
  const int64_t n = (int64_t)P.size();
  if (mode == 0) {
    for (int64_t i = 0; i < n; ++i)
      if (P[i].valid || (P[i].tcam[2] > cam.near_plane && P[i].o >= kAlphaMin && P[i].conic[0] > 0))
        L.all.push_back(i);
    std::sort(L.all.begin(), L.all.end(), [&](int64_t a, int64_t b) { return depth_less(P, a, b); });
  } else if (mode == 1) {
    L.rows.assign(cam.H, {});
    for (int64_t i = 0; i < n; ++i) {
      if (!P[i].valid) continue;
      for (int y = std::max(P[i].pxr[2], y_lo); y <= std::min(P[i].pxr[3], y_hi - 1); ++y)
        L.rows[y].push_back(i);
    }
  } else {
    L.tw = cam.tw;
    L.th = cam.th;
    L.tx = (cam.W + cam.tw - 1) / cam.tw;
    L.ty = (cam.H + cam.th - 1) / cam.th;
    L.tiles.assign((size_t)L.tx * L.ty, {});
    for (int64_t i = 0; i < n; ++i) {
      if (!P[i].valid) continue;
      for (int y = P[i].rect[2]; y <= P[i].rect[3]; ++y) {
        if ((y + 1) * cam.th <= y_lo || y * cam.th >= y_hi) continue;
        for (int x = P[i].rect[0]; x <= P[i].rect[1]; ++x) L.tiles[(size_t)y * L.tx + x].push_back(i);
      }
    }
    for (auto& t : L.tiles)
      std::sort(t.begin(), t.end(), [&](int64_t a, int64_t b) { return depth_less(P, a, b); });
  }
}

void pixel_list(const std::vector<Proj>& P, const Lists& L, int px, int py, std::vector<int64_t>& out) {
  out.clear();
  if (L.mode == 0) {
    if (!L.membership) {
      out = L.all;
    } else {  // the 3-sigma bound's tile membership applies to the brute force as well
      for (int64_t i : L.all)
        if (P[i].valid && P[i].pxr[0] <= px && px <= P[i].pxr[1] && P[i].pxr[2] <= py && py <= P[i].pxr[3])
          out.push_back(i);
    }
  } else if (L.mode == 1) {
    for (int64_t i : L.rows[py])
      if (P[i].pxr[0] <= px && px <= P[i].pxr[1]) out.push_back(i);
    std::sort(out.begin(), out.end(), [&](int64_t a, int64_t b) { return depth_less(P, a, b); });
  } else {
    out = L.tiles[(size_t)(py / L.th) * L.tx + px / L.tw];
  }
}

int n_threads(int req) {
  if (req > 0) return req;
  unsigned h = std::thread::hardware_concurrency();
  return h ? (int)h : 1;
}

template <class F>
void parallel_rows(int y0, int y1, int nt, F f) {
  std::atomic<int> next(y0);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (;;) {
        int y = next.fetch_add(1);
        if (y >= y1) break;
        f(t, y);
      }
    });
  for (auto& x : th) x.join();
}

Scene make_scene(int64_t n, int deg, const float* means, const float* ls, const float* q, const float* lo,
                 const float* sh) {
  Scene s{n, deg, (deg + 1) * (deg + 1), means, ls, q, lo, sh};
  return s;
}

void project_all(const Scene& sc, const Camera& cam, std::vector<Proj>& P) {
  P.resize(sc.n);
  for (int64_t i = 0; i < sc.n; ++i) project(sc, i, cam, P[i]);
}

// Per-Gaussian accumulators of the screen-space gradients (backward of Eq. (1)-(3)).
struct Grad2D {
  double u, v, a, b, c, o, rgb[3];
  double S, M;
  int64_t C;
};

// Backward through the 2-D quantities to the 3-D parameters (chain rule of the
// projection in `project`). Writes the 59-per-Gaussian (at SH3) gradient rows.
void chain_to_params(const Scene& sc, int64_t i, const Camera& cam, const Proj& p, const Grad2D& g,
                     double* dmu, double* dls, double* dq, double* dlogit, double* dsh) {
  const double* W = cam.R;
  // opacity: o = sigmoid(l)
  *dlogit += g.o * p.o * (1.0 - p.o);
  // colour: rgb = max(0, sum_k Y_k f_k + 1/2)
  SH s;
  sh_eval(sc.deg, p.dir[0], p.dir[1], p.dir[2], s);
  double ddir[3] = {0, 0, 0};
  for (int ch = 0; ch < 3; ++ch) {
    const double gc = p.rgb_raw[ch] < 0 ? 0.0 : g.rgb[ch];
    for (int k = 0; k < sc.K; ++k) {
      dsh[k * 3 + ch] += gc * s.Y[k];
      const double f = (double)sc.sh[(i * sc.K + k) * 3 + ch];
      for (int a = 0; a < 3; ++a) ddir[a] += gc * f * s.dY[k][a];
    }
  }
  // dir = (mu - C)/|mu - C|: d dir/d mu = (I - dir dir^T)/|mu - C|
  {
    const double dd = p.dir[0] * ddir[0] + p.dir[1] * ddir[1] + p.dir[2] * ddir[2];
    for (int a = 0; a < 3; ++a) dmu[a] += (ddir[a] - p.dir[a] * dd) / p.dist;
  }
  // conic (a,b,c) -> cov: G_cov = -Q G_Q Q with G_Q = [[da, db/2],[db/2, dc]]
  const double Q[4] = {p.conic[0], p.conic[1], p.conic[1], p.conic[2]};
  const double GQ[4] = {g.a, 0.5 * g.b, 0.5 * g.b, g.c};
  double T1[4], Gc[4];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) T1[2 * r + c] = GQ[2 * r + 0] * Q[0 + c] + GQ[2 * r + 1] * Q[2 + c];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) Gc[2 * r + c] = -(Q[2 * r + 0] * T1[0 + c] + Q[2 * r + 1] * T1[2 + c]);
  // cov = M Sig M^T + 0.3 I:  G_Sig = M^T G_cov M ;  G_M = 2 G_cov M Sig
  double GS[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 2; ++l) acc += p.M[3 * k + r] * Gc[2 * k + l] * p.M[3 * l + c];
      GS[3 * r + c] = acc;
    }
  double MS[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += p.M[3 * r + k] * p.Sig[3 * k + c];
      MS[3 * r + c] = acc;
    }
  double GM[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) GM[3 * r + c] = 2.0 * (Gc[2 * r + 0] * MS[0 + c] + Gc[2 * r + 1] * MS[3 + c]);
  // M = J W : G_J = G_M W^T
  double GJ[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += GM[3 * r + k] * W[3 * c + k];
      GJ[3 * r + c] = acc;
    }
  const double tx = p.tcam[0], ty = p.tcam[1], tz = p.tcam[2];
  const double fx = cam.fx, fy = cam.fy;
  double dt[3] = {0, 0, 0};
  // J00 = fx/tz, J11 = fy/tz
  dt[2] += GJ[0] * (-fx / (tz * tz)) + GJ[4] * (-fy / (tz * tz));
  // J02 = -fx xt/tz with xt = tx/tz unless clamped
  if (p.clampx) {
    dt[2] += GJ[2] * (fx * p.xt / (tz * tz));
  } else {
    dt[0] += GJ[2] * (-fx / (tz * tz));
    dt[2] += GJ[2] * (2.0 * fx * tx / (tz * tz * tz));
  }
  if (p.clampy) {
    dt[2] += GJ[5] * (fy * p.yt / (tz * tz));
  } else {
    dt[1] += GJ[5] * (-fy / (tz * tz));
    dt[2] += GJ[5] * (2.0 * fy * ty / (tz * tz * tz));
  }
  // screen mean u = fx tx/tz + cx, v = fy ty/tz + cy
  dt[0] += g.u * fx / tz;
  dt[1] += g.v * fy / tz;
  dt[2] += -g.u * fx * tx / (tz * tz) - g.v * fy * ty / (tz * tz);
  // t = W mu + t_w
  for (int a = 0; a < 3; ++a) dmu[a] += W[0 + a] * dt[0] + W[3 + a] * dt[1] + W[6 + a] * dt[2];
  // Sig = L L^T with L = R S:  G_L = 2 G_Sig L
  double Lm[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) Lm[3 * r + k] = p.Rq[3 * r + k] * p.s[k];
  double GL[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      double acc = 0;
      for (int l = 0; l < 3; ++l) acc += (GS[3 * r + l] + GS[3 * l + r]) * Lm[3 * l + k];
      GL[3 * r + k] = acc;
    }
  double GR[9];
  for (int k = 0; k < 3; ++k) {
    double ds = 0;
    for (int r = 0; r < 3; ++r) ds += GL[3 * r + k] * p.Rq[3 * r + k];
    dls[k] += ds * p.s[k];
    for (int r = 0; r < 3; ++r) GR[3 * r + k] = GL[3 * r + k] * p.s[k];
  }
  // R(q) with q = (w, x, y, z) normalised
  const double w = p.q[0], x = p.q[1], y = p.q[2], z = p.q[3];
  double dqh[4];
  dqh[0] = 2 * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
  dqh[1] = 2 * (y * GR[1] + z * GR[2] + y * GR[3] - 2 * x * GR[4] - w * GR[5] + z * GR[6] + w * GR[7] -
                2 * x * GR[8]);
  dqh[2] = 2 * (-2 * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] + z * GR[7] -
                2 * y * GR[8]);
  dqh[3] = 2 * (-2 * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2 * z * GR[4] + y * GR[5] + x * GR[6] +
                y * GR[7]);
  const double qd = w * dqh[0] + x * dqh[1] + y * dqh[2] + z * dqh[3];
  for (int k = 0; k < 4; ++k) dq[k] += (dqh[k] - p.q[k] * qd) / p.qnorm;
}

}  // namespace

// ===========================================================================
// C entry points (called through ctypes by the test suite).
extern "C" {

int orc_version() { return 1; }

// Real SH basis values and gradients at unit direction `dir` (pinned against
// scipy's complex spherical harmonics and by quadrature orthonormality).
void orc_sh_basis(int deg, const double* dir, double* Y, double* dY) {
  SH s;
  sh_eval(deg, dir[0], dir[1], dir[2], s);
  const int K = (deg + 1) * (deg + 1);
  for (int k = 0; k < K; ++k) {
    Y[k] = s.Y[k];
    for (int a = 0; a < 3; ++a) dY[3 * k + a] = s.dY[k][a];
  }
}

// Per-Gaussian projection for one view. Outputs (n rows each):
//   f64[n,16]: u, v, conic a, b, c, cov a', b', c', o, r, g, b, depth(f64), tx, ty, tz
//   i32[n,8] : valid, x0, x1, y0, y1 (tile rect, inclusive), tiles, rect_fragile
//   u32[n]   : FP32 bits of the depth key
void orc_preprocess(int64_t n, int deg, const float* means, const float* ls, const float* q, const float* lo,
                    const float* sh, const double* camp, double* f, int32_t* iv, uint32_t* depth_bits) {
  Scene sc = make_scene(n, deg, means, ls, q, lo, sh);
  Camera cam = unpack_camera(camp);
  for (int64_t i = 0; i < n; ++i) {
    Proj p;
    project(sc, i, cam, p);
    double* r = f + 16 * i;
    r[0] = p.u; r[1] = p.v; r[2] = p.conic[0]; r[3] = p.conic[1]; r[4] = p.conic[2];
    r[5] = p.cov[0]; r[6] = p.cov[1]; r[7] = p.cov[2]; r[8] = p.o;
    r[9] = p.rgb[0]; r[10] = p.rgb[1]; r[11] = p.rgb[2]; r[12] = p.tcam[2];
    r[13] = p.tcam[0]; r[14] = p.tcam[1]; r[15] = p.tcam[2];
    int32_t* k = iv + 8 * i;
    k[0] = p.valid; k[1] = p.rect[0]; k[2] = p.rect[1]; k[3] = p.rect[2]; k[4] = p.rect[3];
    k[5] = p.valid ? p.tiles : 0; k[6] = p.rect_fragile; k[7] = 0;
    std::memcpy(&depth_bits[i], &p.depth32, 4);
  }
}

// Forward render of the window [x_lo, x_hi) x [y_lo, y_hi) of one view (other pixels untouched).
//   image f64[3,H,W], T f64[H,W], n_contrib i32[H,W] (list position + 1 of the last
//   blended entry), n_blended i32[H,W], fragile u8[H,W].
void orc_render(int64_t n, int deg, const float* means, const float* ls, const float* q, const float* lo,
                const float* sh, const double* camp, int mode, int x_lo, int x_hi, int y_lo, int y_hi, int threads,
                double* image, double* T, int32_t* n_contrib, int32_t* n_blended, uint8_t* fragile) {
  Scene sc = make_scene(n, deg, means, ls, q, lo, sh);
  Camera cam = unpack_camera(camp);
  std::vector<Proj> P;
  project_all(sc, cam, P);
  Lists L;
  build_lists(P, cam, mode, y_lo, y_hi, L);
  const int W = cam.W, H = cam.H;
  parallel_rows(y_lo, y_hi, n_threads(threads), [&](int, int py) {
    std::vector<int64_t> list;
    PixelResult r;
    for (int px = x_lo; px < x_hi; ++px) {
      pixel_list(P, L, px, py, list);
      composite(P, list, px, py, cam, false, r);
      const size_t o = (size_t)py * W + px;
      for (int ch = 0; ch < 3; ++ch) image[(size_t)ch * H * W + o] = r.rgb[ch];
      T[o] = r.T;
      n_contrib[o] = r.n_contrib;
      n_blended[o] = r.n_blended;
      fragile[o] = (uint8_t)!r.fragile_at.empty();
    }
  });
}

// Backward of the render over the window [x_lo, x_hi) x [y_lo, y_hi) given dL/dI
// f64[3,H,W] (pixels outside the window contribute nothing). Outputs, all overwritten:
//   d_means f64[n,3], d_log_scales f64[n,3], d_quats f64[n,4], d_logits f64[n],
//   d_sh f64[n,K,3], g2d f64[n,9] (u, v, a, b, c, o, r, g, b),
//   S f64[n], M f64[n], C i64[n] (opacity-gradient statistic, Sec. 3.3),
//   gfrag u8[n] (1 if the Gaussian appears in the list of a fragile pixel),
//   C_slack i64[n] (by how much an FP32 walk may legitimately differ from C).
// The statistic sums over blended (pixel, Gaussian) pairs; the per-pixel
// gradient is taken w.r.t. the activated opacity o.
//
// C_slack: at a pixel with a fragile decision, an FP32 walk may take that decision
// the other way. An alpha test or a T-stop test that flips adds or removes its own
// entry. An alpha test or a 0.99 clamp that flips changes every later T of the
// pixel by at most a factor (1 - 1/255) or 1 +- 2e-3, which can move the pixel's
// stop by one entry: the last blended entry may become the stop, or the stop
// entry may be blended (the next visible entry then stops, its T being within
// rounding of 1e-4 times at most 1 - 1/255). Every other entry keeps its decision.
// So each fragile pixel adds 1 to the slack of each of its fragile subjects, of
// its last blended entry and of its stop entry (once per Gaussian per pixel).
void orc_backward(int64_t n, int deg, const float* means, const float* ls, const float* q, const float* lo,
                  const float* sh, const double* camp, int mode, int x_lo, int x_hi, int y_lo, int y_hi,
                  int threads, const double* dL_dI, double* d_means, double* d_ls, double* d_q, double* d_logit,
                  double* d_sh, double* g2d, double* S, double* M, int64_t* C, uint8_t* gfrag,
                  int64_t* C_slack) {
  Scene sc = make_scene(n, deg, means, ls, q, lo, sh);
  Camera cam = unpack_camera(camp);
  std::vector<Proj> P;
  project_all(sc, cam, P);
  Lists L;
  build_lists(P, cam, mode, y_lo, y_hi, L);
  const int W = cam.W, H = cam.H;
  const int nt = n_threads(threads);
  std::vector<std::vector<Grad2D>> acc(nt, std::vector<Grad2D>(n, Grad2D{0, 0, 0, 0, 0, 0, {0, 0, 0}, 0, 0, 0}));
  std::vector<std::vector<uint8_t>> fr(nt, std::vector<uint8_t>(n, 0));
  std::vector<std::vector<int64_t>> slack(nt, std::vector<int64_t>(n, 0));
  parallel_rows(y_lo, y_hi, nt, [&](int t, int py) {
    std::vector<int64_t> list;
    PixelResult r;
    std::vector<double> suffix;
    for (int px = x_lo; px < x_hi; ++px) {
      pixel_list(P, L, px, py, list);
      composite(P, list, px, py, cam, true, r);
      const size_t o = (size_t)py * W + px;
      // A decision within rounding of its threshold can change the gradients of the
      // Gaussian it concerns and of every Gaussian blended at this pixel.
      if (!r.fragile_at.empty()) {
        for (int64_t g : r.fragile_at) fr[t][g] = 1;
        for (const Frag& f : r.blended) fr[t][f.g] = 1;
        std::vector<int64_t> who(r.fragile_at);
        if (r.last >= 0) who.push_back(r.last);
        if (r.stop >= 0) who.push_back(r.stop);
        std::sort(who.begin(), who.end());
        who.erase(std::unique(who.begin(), who.end()), who.end());
        for (int64_t g : who) slack[t][g] += 1;
      }
      const double gI[3] = {dL_dI[o], dL_dI[(size_t)H * W + o], dL_dI[(size_t)2 * H * W + o]};
      const int nb = (int)r.blended.size();
      // suffix[k] = colour behind entry k: sum_{j>k} T_j a_j c_j + T_final bg
      suffix.assign(3 * (nb + 1), 0.0);
      for (int ch = 0; ch < 3; ++ch) suffix[3 * nb + ch] = r.T * cam.bg[ch];
      for (int k = nb - 1; k >= 0; --k) {
        const Frag& f = r.blended[k];
        const Proj& p = P[f.g];
        for (int ch = 0; ch < 3; ++ch)
          suffix[3 * k + ch] = suffix[3 * (k + 1) + ch] + f.T * f.alpha * p.rgb[ch];
      }
      for (int k = 0; k < nb; ++k) {
        const Frag& f = r.blended[k];
        const Proj& p = P[f.g];
        Grad2D& G = acc[t][f.g];
        // Eq. (3): dL/dc = dL/dI * T * alpha
        for (int ch = 0; ch < 3; ++ch) G.rgb[ch] += gI[ch] * f.T * f.alpha;
        // dI/dalpha_k = T_k c_k - (colour behind k)/(1 - alpha_k)
        double dA = 0;
        for (int ch = 0; ch < 3; ++ch)
          dA += gI[ch] * (f.T * p.rgb[ch] - suffix[3 * (k + 1) + ch] / (1.0 - f.alpha));
        // alpha = min(0.99, o G): zero derivative where the clamp is active
        const double dAr = f.a_raw <= kAlphaMax ? dA : 0.0;
        const double g_o = dAr * f.G;       // d/d o of this pixel's loss
        const double dE = dAr * p.o * f.G;  // d/d E (G = exp(E))
        G.o += g_o;
        G.S += g_o * g_o;
        G.M += g_o;
        G.C += 1;
        // E = -1/2 (a dx^2 + 2 b dx dy + c dy^2), dx = u - px - 1/2, dy = v - py - 1/2
        G.a += dE * (-0.5 * f.dx * f.dx);
        G.b += dE * (-f.dx * f.dy);
        G.c += dE * (-0.5 * f.dy * f.dy);
        G.u += dE * (-(p.conic[0] * f.dx + p.conic[1] * f.dy));
        G.v += dE * (-(p.conic[1] * f.dx + p.conic[2] * f.dy));
      }
    }
  });
  const int K = sc.K;
  std::memset(d_means, 0, sizeof(double) * 3 * n);
  std::memset(d_ls, 0, sizeof(double) * 3 * n);
  std::memset(d_q, 0, sizeof(double) * 4 * n);
  std::memset(d_logit, 0, sizeof(double) * n);
  std::memset(d_sh, 0, sizeof(double) * 3 * K * n);
  for (int64_t i = 0; i < n; ++i) {
    Grad2D g{0, 0, 0, 0, 0, 0, {0, 0, 0}, 0, 0, 0};
    uint8_t f = 0;
    C_slack[i] = 0;
    for (int t = 0; t < nt; ++t) {
      C_slack[i] += slack[t][i];
      const Grad2D& a = acc[t][i];
      g.u += a.u; g.v += a.v; g.a += a.a; g.b += a.b; g.c += a.c; g.o += a.o;
      for (int ch = 0; ch < 3; ++ch) g.rgb[ch] += a.rgb[ch];
      g.S += a.S; g.M += a.M; g.C += a.C;
      f |= fr[t][i];
    }
    double* r = g2d + 9 * i;
    r[0] = g.u; r[1] = g.v; r[2] = g.a; r[3] = g.b; r[4] = g.c; r[5] = g.o;
    r[6] = g.rgb[0]; r[7] = g.rgb[1]; r[8] = g.rgb[2];
    S[i] = g.S; M[i] = g.M; C[i] = g.C;
    gfrag[i] = f;
    if (g.C == 0) continue;
    chain_to_params(sc, i, cam, P[i], g, d_means + 3 * i, d_ls + 3 * i, d_q + 4 * i, d_logit + i,
                    d_sh + 3 * K * i);
  }
}

// Chain a given set of screen-space gradients g2d f64[n,9] (u, v, a, b, c, o, r,
// g, b) to the parameters, for one view. Used to pin the chain rule in isolation.
void orc_chain(int64_t n, int deg, const float* means, const float* ls, const float* q, const float* lo,
               const float* sh, const double* camp, const double* g2d, double* d_means, double* d_ls,
               double* d_q, double* d_logit, double* d_sh) {
  Scene sc = make_scene(n, deg, means, ls, q, lo, sh);
  Camera cam = unpack_camera(camp);
  const int K = sc.K;
  std::memset(d_means, 0, sizeof(double) * 3 * n);
  std::memset(d_ls, 0, sizeof(double) * 3 * n);
  std::memset(d_q, 0, sizeof(double) * 4 * n);
  std::memset(d_logit, 0, sizeof(double) * n);
  std::memset(d_sh, 0, sizeof(double) * 3 * K * n);
  for (int64_t i = 0; i < n; ++i) {
    Proj p;
    project(sc, i, cam, p);
    if (!(p.tcam[2] > cam.near_plane) || !(p.conic[0] > 0)) continue;
    const double* r = g2d + 9 * i;
    Grad2D g{r[0], r[1], r[2], r[3], r[4], r[5], {r[6], r[7], r[8]}, 0, 0, 0};
    chain_to_params(sc, i, cam, p, g, d_means + 3 * i, d_ls + 3 * i, d_q + 4 * i, d_logit + i, d_sh + 3 * K * i);
  }
}

// Morton codes (Sec. 3.2.1): per-axis min/max normalisation to [0,1]^3, scaling
// by 2^21 - 1, truncation to integers and interleaving bit k of x, y, z into bits
// 3k, 3k+1, 3k+2 of a 63-bit code. The arithmetic is FP64 on the FP32 inputs:
// u = clamp((p - lo)/(hi - lo), 0, 1), q = trunc(u * 2097151); a degenerate axis
// (hi == lo) maps to 0. perm = indices stably sorted by code.
void orc_morton(int64_t n, const float* means, uint64_t* codes, int64_t* perm) {
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = INFINITY;
    hi[a] = -INFINITY;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], (double)means[3 * i + a]);
      hi[a] = std::max(hi[a], (double)means[3 * i + a]);
    }
  for (int64_t i = 0; i < n; ++i) {
    uint64_t code = 0;
    for (int a = 0; a < 3; ++a) {
      double u = 0.0;
      if (hi[a] > lo[a]) u = ((double)means[3 * i + a] - lo[a]) / (hi[a] - lo[a]);
      u = std::min(std::max(u, 0.0), 1.0);
      const uint32_t qv = (uint32_t)(u * 2097151.0);
      for (int k = 0; k < 21; ++k)
        if ((qv >> k) & 1u) code |= (uint64_t)1 << (3 * k + a);
    }
    codes[i] = code;
  }
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  std::stable_sort(perm, perm + n, [&](int64_t a, int64_t b) { return codes[a] < codes[b]; });
}

// Cluster bounds (Sec. 3.2.2): clusters of `csize` consecutive primitives; per
// cluster the min and max of the means per axis and the largest log-scale.
// Output f32[nc, 8]: minx, miny, minz, maxx, maxy, maxz, max_log_scale, 0.
void orc_cluster_bounds(int64_t n, int csize, const float* means, const float* ls, float* out) {
  const int64_t nc = (n + csize - 1) / csize;
  for (int64_t c = 0; c < nc; ++c) {
    float b[8] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0f};
    for (int64_t i = c * csize; i < std::min(n, (c + 1) * csize); ++i) {
      for (int a = 0; a < 3; ++a) {
        b[a] = std::min(b[a], means[3 * i + a]);
        b[3 + a] = std::max(b[3 + a], means[3 * i + a]);
        b[6] = std::max(b[6], ls[3 * i + a]);
      }
    }
    std::memcpy(out + 8 * c, b, sizeof(b));
  }
}

// Binning, from per-Gaussian (valid, tile rect, depth bits) for V views with
// per-view tile grids. Emits one key per (Gaussian, covered tile) in Gaussian
// order then row-major tile order, key = (global tile id << 32) | depth bits,
// value = Gaussian index, stably sorts by key and derives per-tile ranges.
//   rects i32[V*n, 5] (valid, x0, x1, y0, y1), depth u32[V*n], tile_base i64[V+1],
//   tiles_x i32[V]. Outputs keys u64[M], vals i64[M] (view*n + i), ranges u32[2*T].
int64_t orc_bin(int64_t n, int V, const int32_t* rects, const uint32_t* depth, const int64_t* tile_base,
                const int32_t* tiles_x, uint64_t* keys, int64_t* vals, uint32_t* ranges) {
  std::vector<std::pair<uint64_t, int64_t>> kv;
  for (int v = 0; v < V; ++v)
    for (int64_t i = 0; i < n; ++i) {
      const int32_t* r = rects + 5 * (v * n + i);
      if (!r[0]) continue;
      for (int y = r[3]; y <= r[4]; ++y)
        for (int x = r[1]; x <= r[2]; ++x) {
          const uint64_t tile = (uint64_t)(tile_base[v] + (int64_t)y * tiles_x[v] + x);
          kv.emplace_back((tile << 32) | depth[v * n + i], v * n + i);
        }
    }
  std::stable_sort(kv.begin(), kv.end(),
                   [](const std::pair<uint64_t, int64_t>& a, const std::pair<uint64_t, int64_t>& b) {
                     return a.first < b.first;
                   });
  const int64_t T = tile_base[V];
  for (int64_t t = 0; t < 2 * T; ++t) ranges[t] = 0;
  for (size_t k = 0; k < kv.size(); ++k) {
    keys[k] = kv[k].first;
    vals[k] = kv[k].second;
    const uint64_t tile = kv[k].first >> 32;
    if (k == 0 || (kv[k - 1].first >> 32) != tile) ranges[2 * tile] = (uint32_t)k;
    ranges[2 * tile + 1] = (uint32_t)(k + 1);
  }
  return (int64_t)kv.size();
}

// Count of instances (sum of tiles touched) without materialising them.
int64_t orc_count_instances(int64_t n, int V, const int32_t* rects) {
  int64_t m = 0;
  for (int64_t k = 0; k < (int64_t)V * n; ++k) {
    const int32_t* r = rects + 5 * k;
    if (r[0]) m += (int64_t)(r[2] - r[1] + 1) * (r[4] - r[3] + 1);
  }
  return m;
}

// Variance metric of Sec. 3.3: C * Var = S - M^2 / C, 0 where C = 0.
void orc_variance(int64_t n, const double* S, const double* M, const int64_t* C, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = C[i] > 0 ? S[i] - M[i] * M[i] / (double)C[i] : 0.0;
}

}  // extern "C"
