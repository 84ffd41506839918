// CPU oracle for the differentiable Gaussian rasterizer.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product path links, loads or calls
// this file; only the test suite, the smoke check and the benchmark's CPU
// baseline do. It shares no code, header or constant table with the HIP
// library.
//
// What it computes (paper: Sec. II-A and II-B describe the map as anisotropic
// 3D Gaussians with mean, covariance, opacity and spherical-harmonic colour,
// optimised by a GPU renderer against keyframes, Fig. "GS_SLAM"; GS-SLAM may
// drop view-dependent colour, Sec. II-B). The paper prints no formula, so the
// rasterizer is the standard EWA-splatting image formation of the 3D Gaussian
// splatting work it cites: project every Gaussian to a 2D conic, order by
// camera depth, and composite front to back per pixel with alpha clamped to
// 0.99, alphas below 1/255 skipped and compositing stopped (exclusively)
// once transmittance would fall below 1e-4.
//
// Three scalar modes:
//   FP32        the reference for tile lists (bit-exact) and colour/depth.
//               Its projection follows a fixed sequence of IEEE-754 float
//               operations (no contraction; correctly rounded /, sqrt and
//               exp, the last being the library exp rounded to float) so that
//               an independent implementation of the same sequence
//               reproduces it bit for bit.
//   FP64 pinned the reference for gradients: values in double, every discrete
//               decision (cull, depth order, skip, clamp, stop) taken from the
//               FP32 recurrence evaluated alongside. A stricter variant also
//               takes the per-Gaussian screen-space values the compositing
//               uses (u, v, conic, opacity, colour, depth) rounded to FP32,
//               the precision the method runs in, and differentiates the
//               compositing and the projection in double from there.
//   FP64        values and decisions in double (for finite differences).
//
// Parity status: pinned by closed forms, library routines, invariants,
// torch autograd and finite differences in tests/test_oracle_*.py.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

// ---------------------------------------------------------------------------
// Constants of the method (float; promoted to double in the FP64 modes).
// ---------------------------------------------------------------------------
const float kAlphaMax = 0.99f;           // alpha clamp
const float kAlphaMin = 1.0f / 255.0f;   // skip threshold
const float kTransMin = 1e-4f;           // exclusive stop threshold on T
const float kDilation = 0.3f;            // low-pass dilation of the 2D covariance (px^2)
const float kClampFov = 1.3f;            // Jacobian clamp, multiple of the half-FoV tangent
// Squared Mahalanobis radius of the binning ellipse. alpha >= 1/255 with
// opacity <= 1 implies q <= 2 ln 255 = 11.0825; 11.2 leaves room for rounding.
const float kQMax = 11.2f;

// ---------------------------------------------------------------------------
// Exponential in the FP32 mode: exp(x) rounded to the nearest float (O1 uses
// it for the scales and the opacity). The library's double exp is rounded to
// float; that second rounding can only go wrong when the double result lies
// within its own error of a midpoint between two floats, so such results are
// recomputed from the library's long double exp (64 significant bits).
// exp32_tie_distance reports how close the long double result comes to a
// midpoint, so that tests can check that no input of the ranges in use is
// undecided even at that precision.
// ---------------------------------------------------------------------------
long double float_midpoint_near(float f, long double y) {
  // midpoint between f and its neighbour on y's side (exact in long double)
  const float nb = y >= (long double)f ? std::nextafter(f, INFINITY) : std::nextafter(f, -INFINITY);
  return 0.5L * ((long double)f + (long double)nb);
}
float exp32(float x) {
  const double y = std::exp((double)x);
  const float f = (float)y;
  if (!std::isfinite(f) || f == 0.0f) return f;
  const long double mid = float_midpoint_near(f, (long double)y);
  if (std::fabs((long double)y - mid) > 0x1p-50L * (long double)y) return f;
  return (float)std::exp((long double)x);
}
double exp32_tie_distance(float x) {
  const long double y = std::exp((long double)x);
  const float f = (float)y;
  if (!std::isfinite(f) || f == 0.0f) return INFINITY;
  return (double)(std::fabs(y - float_midpoint_near(f, y)) / y);
}
float exp_t(float x) { return exp32(x); }
double exp_t(double x) { return std::exp(x); }

template <class T> T sqrt_t(T x) { return std::sqrt(x); }

// ---------------------------------------------------------------------------
// Real spherical harmonics with the Condon-Shortley phase, any degree, as
// polynomials of the unit direction (x, y, z):
//   Y_l0  = N_l0 Pbar_l^0(z)
//   Y_lm  = sqrt2 N_lm Pbar_l^m(z) Re((x + i y)^m)      m > 0
//   Y_l-m = sqrt2 N_lm Pbar_l^m(z) Im((x + i y)^m)      m > 0
// where Pbar_l^m = P_l^m / (1 - z^2)^(m/2) (associated Legendre function with
// the (-1)^m phase, its sin^m factor moved into (x + i y)^m) and
// N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!). Index k = l^2 + l + m.
// Evaluated on a forward-mode dual number so the oracle's backward gets the
// exact gradient with respect to the direction.
// ---------------------------------------------------------------------------
struct Dual3 {
  double v, d[3];
  Dual3(double x = 0.0) : v(x) { d[0] = d[1] = d[2] = 0.0; }
};
inline Dual3 operator+(const Dual3& a, const Dual3& b) { Dual3 r(a.v + b.v); for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual3 operator-(const Dual3& a, const Dual3& b) { Dual3 r(a.v - b.v); for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual3 operator*(const Dual3& a, const Dual3& b) { Dual3 r(a.v * b.v); for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual3 operator*(double s, const Dual3& b) { Dual3 r(s * b.v); for (int i = 0; i < 3; ++i) r.d[i] = s * b.d[i]; return r; }

double factorial(int k) { double f = 1.0; for (int i = 2; i <= k; ++i) f *= i; return f; }

// out[k] = Y_k(dir) for k < (deg+1)^2; dir components are duals.
void sh_basis_dual(int deg, const Dual3 dir[3], Dual3* out) {
  const Dual3& x = dir[0];
  const Dual3& y = dir[1];
  const Dual3& z = dir[2];
  const double pi = 3.14159265358979323846;
  // (x + i y)^m for m = 0..deg
  std::vector<Dual3> re(deg + 1), im(deg + 1);
  re[0] = Dual3(1.0); im[0] = Dual3(0.0);
  for (int m = 1; m <= deg; ++m) {
    re[m] = re[m - 1] * x - im[m - 1] * y;
    im[m] = re[m - 1] * y + im[m - 1] * x;
  }
  for (int m = 0; m <= deg; ++m) {
    // Pbar_m^m = (-1)^m (2m-1)!!
    double dfact = 1.0;
    for (int i = 1; i <= 2 * m - 1; i += 2) dfact *= i;
    Dual3 p_mm((m % 2 ? -1.0 : 1.0) * dfact);
    Dual3 p_prev2, p_prev1 = p_mm;
    for (int l = m; l <= deg; ++l) {
      Dual3 p;
      if (l == m) p = p_mm;
      else if (l == m + 1) p = ((double)(2 * m + 1)) * (z * p_mm);
      else p = (1.0 / (l - m)) * (((double)(2 * l - 1)) * (z * p_prev1) - ((double)(l + m - 1)) * p_prev2);
      if (l > m) { p_prev2 = p_prev1; p_prev1 = p; }
      double N = std::sqrt((2.0 * l + 1.0) / (4.0 * pi) * factorial(l - m) / factorial(l + m));
      if (m == 0) {
        out[l * l + l] = N * p;
      } else {
        out[l * l + l + m] = (std::sqrt(2.0) * N) * (p * re[m]);
        out[l * l + l - m] = (std::sqrt(2.0) * N) * (p * im[m]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Camera
// ---------------------------------------------------------------------------
template <class T> struct Cam {
  T W[9], t[3], fx, fy, cx, cy;
  int width, height;
  T campos[3];   // camera centre in world: -W^T t
};
template <class T> Cam<T> make_cam(const float* c, int width, int height) {
  Cam<T> k;
  for (int i = 0; i < 9; ++i) k.W[i] = (T)c[i];
  for (int i = 0; i < 3; ++i) k.t[i] = (T)c[9 + i];
  k.fx = (T)c[12]; k.fy = (T)c[13]; k.cx = (T)c[14]; k.cy = (T)c[15];
  k.width = width; k.height = height;
  for (int j = 0; j < 3; ++j) {
    double s = 0.0;
    for (int i = 0; i < 3; ++i) s -= (double)c[i * 3 + j] * (double)c[9 + i];
    k.campos[j] = (T)s;
  }
  return k;
}

// ---------------------------------------------------------------------------
// Projection of one Gaussian (EWA splatting).
// ---------------------------------------------------------------------------
template <class T> struct Proj {
  Proj() { std::memset(static_cast<void*>(this), 0, sizeof(*this)); }
  bool vis;
  T u, v, z;
  T a, b, c;          // dilated screen-space covariance [[a, b], [b, c]]
  T det, A, B, C;     // conic = inverse covariance [[A, B], [B, C]]
  T o;                // opacity
  T col[3];
  T colraw[3];        // colour before the max(0, .) clamp
  T ex, ey;           // half-extents of the binning ellipse's bounding box (px)
  int px0, py0, px1, py1;   // pixel rectangle (inclusive)
  // intermediates for the backward
  T s[3], qn, qh[4], R[9], M[9], Sig[9], Tm[6];
  T tx, ty, tz, xi, yi; bool xclamp, yclamp;
  T J00, J02, J11, J12;
  T dir[3], dnorm;
};

template <class T> bool finite_t(T x) { return std::isfinite((double)x); }

// Projection in the fixed operation order described at the top of the file.
template <class T>
Proj<T> project_one(const float* P, int64_t stride, int64_t i, int deg, const Cam<T>& cam, T znear) {
  Proj<T> g;
  const float* raw[11];
  for (int k = 0; k < 11; ++k) raw[k] = P + k * stride + i;
  for (int k = 0; k < 11; ++k) if (!std::isfinite(*raw[k])) return g;
  const T mx = (T)*raw[0], my = (T)*raw[1], mz = (T)*raw[2];
  // O1 activations: scale = exp(log-scale), unit quaternion, rotation matrix
  for (int k = 0; k < 3; ++k) g.s[k] = exp_t((T)*raw[3 + k]);
  const T qw = (T)*raw[6], qx = (T)*raw[7], qy = (T)*raw[8], qz = (T)*raw[9];
  T ss = qw * qw + qx * qx;
  ss = ss + qy * qy;
  ss = ss + qz * qz;
  if (!(ss > (T)0) || !finite_t(ss)) return g;
  g.qn = sqrt_t(ss);
  const T w = qw / g.qn, x = qx / g.qn, y = qy / g.qn, z = qz / g.qn;
  g.qh[0] = w; g.qh[1] = x; g.qh[2] = y; g.qh[3] = z;
  T* R = g.R;
  R[0] = (T)1 - (T)2 * (y * y + z * z);
  R[1] = (T)2 * (x * y - w * z);
  R[2] = (T)2 * (x * z + w * y);
  R[3] = (T)2 * (x * y + w * z);
  R[4] = (T)1 - (T)2 * (x * x + z * z);
  R[5] = (T)2 * (y * z - w * x);
  R[6] = (T)2 * (x * z - w * y);
  R[7] = (T)2 * (y * z + w * x);
  R[8] = (T)1 - (T)2 * (x * x + y * y);
  // Sigma = M M^T with M = R diag(s)
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) g.M[r * 3 + k] = R[r * 3 + k] * g.s[k];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      T acc = g.M[r * 3 + 0] * g.M[k * 3 + 0] + g.M[r * 3 + 1] * g.M[k * 3 + 1];
      g.Sig[r * 3 + k] = acc + g.M[r * 3 + 2] * g.M[k * 3 + 2];
    }
  // O2 camera transform
  const T* W = cam.W;
  T tc[3];
  for (int r = 0; r < 3; ++r) {
    T acc = W[r * 3 + 0] * mx + W[r * 3 + 1] * my;
    acc = acc + W[r * 3 + 2] * mz;
    tc[r] = acc + cam.t[r];
  }
  g.tx = tc[0]; g.ty = tc[1]; g.tz = tc[2];
  if (!(g.tz >= znear)) return g;
  g.z = g.tz;
  // O3 EWA Jacobian with the tangent clamp
  const T limx = (T)kClampFov * (((T)0.5 * (T)cam.width) / cam.fx);
  const T limy = (T)kClampFov * (((T)0.5 * (T)cam.height) / cam.fy);
  T xr = g.tx / g.tz, yr = g.ty / g.tz;
  g.xclamp = (xr < -limx) || (xr > limx);
  g.yclamp = (yr < -limy) || (yr > limy);
  g.xi = std::fmin(std::fmax(xr, -limx), limx);
  g.yi = std::fmin(std::fmax(yr, -limy), limy);
  g.J00 = cam.fx / g.tz;
  g.J02 = -(cam.fx * g.xi) / g.tz;
  g.J11 = cam.fy / g.tz;
  g.J12 = -(cam.fy * g.yi) / g.tz;
  // T = J W (2x3)
  for (int k = 0; k < 3; ++k) {
    g.Tm[k] = g.J00 * W[0 * 3 + k] + g.J02 * W[2 * 3 + k];
    g.Tm[3 + k] = g.J11 * W[1 * 3 + k] + g.J12 * W[2 * 3 + k];
  }
  // U = T Sigma, Sigma' = U T^T + 0.3 I
  T U[6];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) {
      T acc = g.Tm[r * 3 + 0] * g.Sig[0 * 3 + k] + g.Tm[r * 3 + 1] * g.Sig[1 * 3 + k];
      U[r * 3 + k] = acc + g.Tm[r * 3 + 2] * g.Sig[2 * 3 + k];
    }
  T a = U[0] * g.Tm[0] + U[1] * g.Tm[1];
  a = a + U[2] * g.Tm[2];
  T b = U[0] * g.Tm[3] + U[1] * g.Tm[4];
  b = b + U[2] * g.Tm[5];
  T c = U[3] * g.Tm[3] + U[4] * g.Tm[4];
  c = c + U[5] * g.Tm[5];
  a = a + (T)kDilation;
  c = c + (T)kDilation;
  // O4 conic
  T det = a * c - b * b;
  if (!(det > (T)0) || !finite_t(det) || !finite_t(a) || !finite_t(b) || !finite_t(c)) return g;
  g.a = a; g.b = b; g.c = c; g.det = det;
  g.A = c / det;
  g.B = -(b / det);
  g.C = a / det;
  // projected mean
  g.u = (cam.fx * g.tx) / g.tz + cam.cx;
  g.v = (cam.fy * g.ty) / g.tz + cam.cy;
  if (!finite_t(g.u) || !finite_t(g.v)) return g;
  // O6 extents (opacity independent) and pixel rectangle
  g.ex = sqrt_t((T)kQMax * a);
  g.ey = sqrt_t((T)kQMax * c);
  T x0 = std::ceil((g.u - g.ex) - (T)0.5);
  T x1 = std::floor((g.u + g.ex) - (T)0.5);
  T y0 = std::ceil((g.v - g.ey) - (T)0.5);
  T y1 = std::floor((g.v + g.ey) - (T)0.5);
  x0 = std::fmax(x0, (T)0); y0 = std::fmax(y0, (T)0);
  x1 = std::fmin(x1, (T)(cam.width - 1)); y1 = std::fmin(y1, (T)(cam.height - 1));
  if (x0 > x1 || y0 > y1) return g;
  g.px0 = (int)x0; g.px1 = (int)x1; g.py0 = (int)y0; g.py1 = (int)y1;
  // O1 opacity = sigmoid(logit)
  g.o = (T)1 / ((T)1 + exp_t(-(T)*raw[10]));
  // O5 colour from spherical harmonics (evaluated in double)
  const int K = (deg + 1) * (deg + 1);
  Dual3 dd[3];
  double dnorm = 1.0;
  if (deg > 0) {
    double d0 = (double)mx - (double)cam.campos[0];
    double d1 = (double)my - (double)cam.campos[1];
    double d2 = (double)mz - (double)cam.campos[2];
    dnorm = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    dd[0] = Dual3(d0 / dnorm); dd[1] = Dual3(d1 / dnorm); dd[2] = Dual3(d2 / dnorm);
  }
  g.dnorm = (T)dnorm;
  for (int k = 0; k < 3; ++k) g.dir[k] = (T)dd[k].v;
  std::vector<Dual3> Y(K);
  sh_basis_dual(deg, dd, Y.data());
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc += (double)P[(11 + 3 * k + ch) * stride + i] * Y[k].v;
    acc += 0.5;
    g.colraw[ch] = (T)acc;
    g.col[ch] = std::fmax(g.colraw[ch], (T)0);
    if (!finite_t(g.col[ch])) return g;
  }
  g.vis = true;
  return g;
}

template <class T>
std::vector<Proj<T>> project_all(const float* P, int64_t n, int64_t stride, int deg, const Cam<T>& cam, T znear) {
  std::vector<Proj<T>> out(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = project_one<T>(P, stride, i, deg, cam, znear);
  return out;
}

uint32_t float_bits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }

// O8: visible Gaussians sorted by (raw bits of the FP32 depth, index).
std::vector<int64_t> depth_order(const std::vector<Proj<float>>& p32) {
  std::vector<int64_t> ord;
  for (int64_t i = 0; i < (int64_t)p32.size(); ++i) if (p32[i].vis) ord.push_back(i);
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    uint32_t za = float_bits(p32[a].z), zb = float_bits(p32[b].z);
    return za != zb ? za < zb : a < b;
  });
  return ord;
}

// ---------------------------------------------------------------------------
// Per-pixel compositing (O9, O10). TD is the type that takes the decisions,
// TV the type of the values. With TD == TV they are one computation.
// ---------------------------------------------------------------------------
struct Composited {      // one composited pair, FP64 values for the backward
  int64_t idx; bool clamped; double G, alpha, dx, dy;
};

template <class TD, class TV>
struct PixelResult {
  TV rgb[3], depth, T;
  int ncomp;
  double margin;
};

template <class T> T exp_blend(T x);
template <> float exp_blend<float>(float x) { return (float)std::exp((double)x); }
template <> double exp_blend<double>(double x) { return std::exp(x); }

template <class TD, class TV>
PixelResult<TD, TV> composite_pixel(const std::vector<Proj<TD>>& pd, const std::vector<Proj<TV>>& pv,
                                    const std::vector<int64_t>& order, const std::vector<Proj<float>>& rects,
                                    bool prefilter, int px, int py, const float* bg,
                                    std::vector<Composited>* trace) {
  PixelResult<TD, TV> res;
  TD Td = (TD)1;
  TV Tv = (TV)1;
  TV C[3] = {0, 0, 0}, D = 0;
  double margin = 1e30;
  int ncomp = 0;
  const TD xsd = (TD)px + (TD)0.5, ysd = (TD)py + (TD)0.5;
  const TV xsv = (TV)px + (TV)0.5, ysv = (TV)py + (TV)0.5;
  for (int64_t i : order) {
    if (prefilter) {
      const Proj<float>& r = rects[i];
      if (px < r.px0 || px > r.px1 || py < r.py0 || py > r.py1) continue;
    }
    const Proj<TD>& g = pd[i];
    TD dx = g.u - xsd, dy = g.v - ysd;
    TD qa = (g.A * dx) * dx, qc = (g.C * dy) * dy, qb = (g.B * dx) * dy;
    TD power = (TD)(-0.5) * (qa + qc) - qb;
    double pscale = std::fabs((double)qa) + std::fabs((double)qc) + std::fabs((double)qb) + 1e-30;
    margin = std::min(margin, std::fabs((double)power) / pscale);
    if (power > (TD)0) continue;
    TD G = exp_blend<TD>(power);
    TD araw = g.o * G;
    bool clamped = araw > (TD)kAlphaMax;
    TD alpha = clamped ? (TD)kAlphaMax : araw;
    margin = std::min(margin, std::fabs((double)araw - (double)kAlphaMax) / (double)kAlphaMax);
    margin = std::min(margin, std::fabs((double)alpha - (double)kAlphaMin) / (double)kAlphaMin);
    if (alpha < (TD)kAlphaMin) continue;
    TD Tn = Td * ((TD)1 - alpha);
    margin = std::min(margin, std::fabs((double)Tn - (double)kTransMin) / (double)kTransMin);
    if (Tn < (TD)kTransMin) break;
    // values
    const Proj<TV>& h = pv[i];
    TV dxv = h.u - xsv, dyv = h.v - ysv;
    TV powv = (TV)(-0.5) * ((h.A * dxv) * dxv + (h.C * dyv) * dyv) - (h.B * dxv) * dyv;
    TV Gv = exp_blend<TV>(powv);
    TV av = clamped ? (TV)kAlphaMax : h.o * Gv;
    TV wgt = av * Tv;
    for (int ch = 0; ch < 3; ++ch) C[ch] = C[ch] + wgt * h.col[ch];
    D = D + wgt * h.z;
    Tv = Tv * ((TV)1 - av);
    Td = Tn;
    ++ncomp;
    if (trace) trace->push_back({i, clamped, (double)Gv, (double)av, (double)dxv, (double)dyv});
  }
  for (int ch = 0; ch < 3; ++ch) res.rgb[ch] = C[ch] + Tv * (TV)bg[ch];
  res.depth = D;
  res.T = Tv;
  res.ncomp = ncomp;
  res.margin = margin;
  return res;
}

// The pixels a call covers: the window [x0, x1) x [y0, y1), every row_step-th
// row of it. The whole image by default. Restricting the pixels changes no
// pixel's value: each is composited on its own.
struct PixelSet {
  int x0, y0, x1, y1, row_step;
};
PixelSet pixel_set(const int32_t* win, int width, int height) {
  PixelSet s{0, 0, width, height, 1};
  if (win) {
    s.x0 = std::max(0, win[0]);
    s.y0 = std::max(0, win[1]);
    s.x1 = std::min(width, win[2]);
    s.y1 = std::min(height, win[3]);
    s.row_step = std::max(1, win[4]);
  }
  return s;
}

template <class TD, class TV>
void render_view(const float* P, int64_t n, int64_t stride, int deg, const float* camf, int width, int height,
                 float znear, const float* bg, bool prefilter, double* rgb, double* depth, double* alpha,
                 double* tfinal, int32_t* ncomp, double* margin, const PixelSet& ps) {
  Cam<float> c32 = make_cam<float>(camf, width, height);
  std::vector<Proj<float>> p32 = project_all<float>(P, n, stride, deg, c32, znear);
  std::vector<int64_t> order = depth_order(p32);
  std::vector<Proj<TD>> pd_own;
  std::vector<Proj<TV>> pv_own;
  const std::vector<Proj<TD>>* pd;
  const std::vector<Proj<TV>>* pv;
  if constexpr (std::is_same<TD, float>::value) pd = &p32;
  else { pd_own = project_all<TD>(P, n, stride, deg, make_cam<TD>(camf, width, height), (TD)znear); pd = &pd_own; }
  if constexpr (std::is_same<TV, float>::value) pv = &p32;
  else if constexpr (std::is_same<TV, TD>::value) pv = reinterpret_cast<const std::vector<Proj<TV>>*>(pd);
  else { pv_own = project_all<TV>(P, n, stride, deg, make_cam<TV>(camf, width, height), (TV)znear); pv = &pv_own; }
  if (!std::is_same<TD, float>::value) {
    // FP64 decisions: cull set and order from the FP64 projection itself
    std::vector<int64_t> ord;
    for (int64_t i = 0; i < n; ++i) if ((*pd)[i].vis) ord.push_back(i);
    std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
      double za = (double)(*pd)[a].z, zb = (double)(*pd)[b].z;
      return za != zb ? za < zb : a < b;
    });
    order.swap(ord);
    prefilter = false;
  }
  const int64_t HW = (int64_t)width * height;
#pragma omp parallel for schedule(dynamic, 1)
  for (int py = ps.y0; py < ps.y1; py += ps.row_step) {
    for (int px = ps.x0; px < ps.x1; ++px) {
      PixelResult<TD, TV> r = composite_pixel<TD, TV>(*pd, *pv, order, p32, prefilter, px, py, bg, nullptr);
      int64_t o = (int64_t)py * width + px;
      for (int ch = 0; ch < 3; ++ch) rgb[ch * HW + o] = (double)r.rgb[ch];
      depth[o] = (double)r.depth;
      alpha[o] = 1.0 - (double)r.T;
      if (std::is_same<TV, float>::value) alpha[o] = (double)(1.0f - (float)r.T);
      tfinal[o] = (double)r.T;
      ncomp[o] = r.ncomp;
      margin[o] = r.margin;
    }
  }
}

// ---------------------------------------------------------------------------
// Backward (O11 blend, O12 projection) in double.
// ---------------------------------------------------------------------------
enum { G2_U = 0, G2_V, G2_A, G2_B, G2_C, G2_O, G2_R, G2_G, G2_BL, G2_Z, G2_N };

// Chain rule from the per-Gaussian screen-space gradients to the parameters.
// With gcam (not null), also adds this Gaussian's part of the gradient with
// respect to the view's camera: gcam[0..8] = dL/dR (row-major), gcam[9..11] =
// dL/dt, for the world-to-camera transform x_cam = R x + t. R enters through
// the camera-space mean, through T = J R (the screen covariance J R Sigma
// R^T J^T) and, for view-dependent colour, through the camera centre -R^T t;
// t through the mean and the centre.
// grad[plane * gstride + gi] += ...; gi is the Gaussian's index in grad (its
// index i in the parameters unless the caller redirects the output).
void project_backward_one(const float* P, int64_t stride, int64_t i, int deg, const Cam<double>& cam,
                          const Proj<double>& g, const double* g2, double* grad, int64_t gstride,
                          double* gcam = nullptr, int64_t gi = -1) {
  if (gi < 0) gi = i;
  const double gu = g2[G2_U], gv = g2[G2_V], gA = g2[G2_A], gB = g2[G2_B], gC = g2[G2_C];
  const double gz = g2[G2_Z];
  double gcol[3] = {g2[G2_R], g2[G2_G], g2[G2_BL]};
  // opacity: o = sigmoid(l)
  grad[10 * gstride + gi] += g2[G2_O] * g.o * (1.0 - g.o);
  // colour: col = max(0, sum_k k_k Y_k(d) + 0.5)
  const int K = (deg + 1) * (deg + 1);
  Dual3 dd[3];
  for (int k = 0; k < 3; ++k) { dd[k] = Dual3(g.dir[k]); dd[k].d[k] = 1.0; }
  std::vector<Dual3> Y(K);
  sh_basis_dual(deg, dd, Y.data());
  double gdir[3] = {0, 0, 0};
  for (int ch = 0; ch < 3; ++ch) {
    if (g.colraw[ch] < 0.0) continue;
    for (int k = 0; k < K; ++k) {
      grad[(11 + 3 * k + ch) * gstride + gi] += gcol[ch] * Y[k].v;
      if (deg > 0) {
        double coef = (double)P[(11 + 3 * k + ch) * stride + i];
        for (int j = 0; j < 3; ++j) gdir[j] += gcol[ch] * coef * Y[k].d[j];
      }
    }
  }
  double gmean[3] = {0, 0, 0};
  double gview[3] = {0, 0, 0};   // dL/dv through the colour, v = mean - campos
  if (deg > 0) {
    // d = v/|v|, v = mean - campos:  dL/dv = (I - d d^T) dL/dd / |v|
    double dot = g.dir[0] * gdir[0] + g.dir[1] * gdir[1] + g.dir[2] * gdir[2];
    for (int j = 0; j < 3; ++j) gview[j] = (gdir[j] - g.dir[j] * dot) / g.dnorm;
    for (int j = 0; j < 3; ++j) gmean[j] += gview[j];
  }
  // conic (A, B, C) = (c, -b, a) / det,  det = a c - b^2
  const double a = g.a, b = g.b, c = g.c, det = g.det, d2 = det * det;
  const double ga = gA * (-c * c / d2) + gB * (b * c / d2) + gC * (-b * b / d2);
  const double gb = gA * (2.0 * b * c / d2) + gB * (-1.0 / det - 2.0 * b * b / d2) + gC * (2.0 * a * b / d2);
  const double gc = gA * (-b * b / d2) + gB * (a * b / d2) + gC * (-a * a / d2);
  // Sigma' = T Sigma T^T (+ dilation), rows T0, T1 of T = J W
  const double* T0 = g.Tm;
  const double* T1 = g.Tm + 3;
  const double* S = g.Sig;
  double ST0[3], ST1[3];
  for (int r = 0; r < 3; ++r) {
    ST0[r] = S[r * 3 + 0] * T0[0] + S[r * 3 + 1] * T0[1] + S[r * 3 + 2] * T0[2];
    ST1[r] = S[r * 3 + 0] * T1[0] + S[r * 3 + 1] * T1[1] + S[r * 3 + 2] * T1[2];
  }
  double gT0[3], gT1[3];
  for (int r = 0; r < 3; ++r) {
    gT0[r] = 2.0 * ga * ST0[r] + gb * ST1[r];
    gT1[r] = gb * ST0[r] + 2.0 * gc * ST1[r];
  }
  // dL/dSigma (full 3x3, as a function of independent entries)
  double gS[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k)
      gS[r * 3 + k] = ga * T0[r] * T0[k] + gb * T0[r] * T1[k] + gc * T1[r] * T1[k];
  // T = J W: J00, J02 in row 0, J11, J12 in row 1
  const double* W = cam.W;
  double gJ00 = 0, gJ02 = 0, gJ11 = 0, gJ12 = 0;
  for (int k = 0; k < 3; ++k) {
    gJ00 += gT0[k] * W[0 * 3 + k];
    gJ02 += gT0[k] * W[2 * 3 + k];
    gJ11 += gT1[k] * W[1 * 3 + k];
    gJ12 += gT1[k] * W[2 * 3 + k];
  }
  // J00 = fx/tz, J02 = -fx xi/tz with xi = clamp(tx/tz); same for y
  const double tx = g.tx, ty = g.ty, tz = g.tz, fx = cam.fx, fy = cam.fy;
  double gtx = 0, gty = 0, gtz = 0;
  gtz += gJ00 * (-fx / (tz * tz));
  gtz += gJ11 * (-fy / (tz * tz));
  gtz += gJ02 * (fx * g.xi / (tz * tz));
  gtz += gJ12 * (fy * g.yi / (tz * tz));
  if (!g.xclamp) {   // xi = tx/tz
    double gxi = gJ02 * (-fx / tz);
    gtx += gxi / tz;
    gtz += gxi * (-tx / (tz * tz));
  }
  if (!g.yclamp) {
    double gyi = gJ12 * (-fy / tz);
    gty += gyi / tz;
    gtz += gyi * (-ty / (tz * tz));
  }
  // u = fx tx/tz + cx, v = fy ty/tz + cy, z = tz
  gtx += gu * fx / tz;
  gtz += gu * (-fx * tx / (tz * tz));
  gty += gv * fy / tz;
  gtz += gv * (-fy * ty / (tz * tz));
  gtz += gz;
  // t = W mean + t_cw
  for (int j = 0; j < 3; ++j) gmean[j] += W[0 * 3 + j] * gtx + W[1 * 3 + j] * gty + W[2 * 3 + j] * gtz;
  for (int j = 0; j < 3; ++j) grad[j * gstride + gi] += gmean[j];
  if (gcam) {
    const double mu[3] = {(double)P[0 * stride + i], (double)P[1 * stride + i], (double)P[2 * stride + i]};
    const double gt[3] = {gtx, gty, gtz};
    // x_cam = W mu + t_cw
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) gcam[r * 3 + k] += gt[r] * mu[k];
      gcam[9 + r] += gt[r];
    }
    // T = J W with J = [[J00, 0, J02], [0, J11, J12]]: dL/dW = J^T dL/dT
    for (int k = 0; k < 3; ++k) {
      gcam[0 * 3 + k] += g.J00 * gT0[k];
      gcam[1 * 3 + k] += g.J11 * gT1[k];
      gcam[2 * 3 + k] += g.J02 * gT0[k] + g.J12 * gT1[k];
    }
    // campos = -W^T t_cw and v = mu - campos: dL/dcampos = -gview
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) gcam[r * 3 + k] += gview[k] * cam.t[r];
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += W[r * 3 + k] * gview[k];
      gcam[9 + r] += s;
    }
  }
  // Sigma = M M^T: dL/dM = (gS + gS^T) M
  double gM[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      double acc = 0;
      for (int j = 0; j < 3; ++j) acc += (gS[r * 3 + j] + gS[j * 3 + r]) * g.M[j * 3 + k];
      gM[r * 3 + k] = acc;
    }
  // M = R diag(s)
  double gR[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) gR[r * 3 + k] = gM[r * 3 + k] * g.s[k];
  for (int k = 0; k < 3; ++k) {
    double gs = gM[0 * 3 + k] * g.R[0 * 3 + k] + gM[1 * 3 + k] * g.R[1 * 3 + k] + gM[2 * 3 + k] * g.R[2 * 3 + k];
    grad[(3 + k) * gstride + gi] += gs * g.s[k];     // s = exp(log-scale)
  }
  // R(q^) for unit q^ = (w, x, y, z)
  const double w = g.qh[0], x = g.qh[1], y = g.qh[2], z = g.qh[3];
  double gw = 2.0 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
  double gx = 2.0 * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5] + z * gR[6] + w * gR[7] - 2.0 * x * gR[8]);
  double gy = 2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7] - 2.0 * y * gR[8]);
  double gzq = 2.0 * (-2.0 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0 * z * gR[4] + y * gR[5] + x * gR[6] + y * gR[7]);
  // q^ = q/|q|: dL/dq = (dL/dq^ - q^ (q^ . dL/dq^)) / |q|
  double dq[4] = {gw, gx, gy, gzq};
  double dot = w * gw + x * gx + y * gy + z * gzq;
  for (int k = 0; k < 4; ++k) grad[(6 + k) * gstride + gi] += (dq[k] - g.qh[k] * dot) / g.qn;
}

// Blend backward for one view: accumulates screen-space gradients g2[n][10].
// With `pinned`, decisions come from the FP32 recurrence, values from FP64;
// with `splats32` the compositing values are the FP32 projection's.
void blend_backward_view(const float* P, int64_t n, int64_t stride, int deg, const float* camf, int width, int height,
                         float znear, const float* bg, const float* grgb, const float* gdepth, const float* galpha,
                         bool pinned, bool splats32, std::vector<double>& g2out, std::vector<Proj<double>>& p64out,
                         const PixelSet& ps, std::vector<double>* absout = nullptr) {
  Cam<float> c32 = make_cam<float>(camf, width, height);
  Cam<double> c64 = make_cam<double>(camf, width, height);
  std::vector<Proj<float>> p32 = project_all<float>(P, n, stride, deg, c32, znear);
  std::vector<Proj<double>> p64 = project_all<double>(P, n, stride, deg, c64, (double)znear);
  // the chain rule to the parameters always uses the double projection
  std::vector<Proj<double>> blendv = p64;
  if (splats32)
    for (int64_t i = 0; i < n; ++i) {
      if (!p32[i].vis) continue;
      Proj<double>& d = blendv[i];
      const Proj<float>& f = p32[i];
      d.u = f.u; d.v = f.v; d.z = f.z; d.A = f.A; d.B = f.B; d.C = f.C; d.o = f.o;
      for (int ch = 0; ch < 3; ++ch) d.col[ch] = f.col[ch];
    }
  std::vector<int64_t> order;
  if (pinned) {
    order = depth_order(p32);
  } else {
    for (int64_t i = 0; i < n; ++i) if (p64[i].vis) order.push_back(i);
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      return p64[a].z != p64[b].z ? p64[a].z < p64[b].z : a < b;
    });
  }
  const int64_t HW = (int64_t)width * height;
  int nt = omp_get_max_threads();
  std::vector<std::vector<double>> acc(nt, std::vector<double>((size_t)n * G2_N, 0.0));
  std::vector<std::vector<double>> aacc(absout ? nt : 0, std::vector<double>((size_t)n * G2_N, 0.0));
#pragma omp parallel
  {
    std::vector<double>& mine = acc[omp_get_thread_num()];
    double* amine = absout ? aacc[omp_get_thread_num()].data() : nullptr;
    std::vector<Composited> trace;
#pragma omp for schedule(dynamic, 1)
    for (int py = ps.y0; py < ps.y1; py += ps.row_step) {
      for (int px = ps.x0; px < ps.x1; ++px) {
        trace.clear();
        double Tfin;
        if (pinned) {
          PixelResult<float, double> r = composite_pixel<float, double>(p32, blendv, order, p32, true, px, py, bg, &trace);
          Tfin = r.T;
        } else {
          PixelResult<double, double> r = composite_pixel<double, double>(p64, p64, order, p32, false, px, py, bg, &trace);
          Tfin = r.T;
        }
        const int64_t o = (int64_t)py * width + px;
        const double gc[3] = {grgb[o], grgb[HW + o], grgb[2 * HW + o]};
        const double gd = gdepth[o], ga = galpha[o];
        // reverse walk: recover T_k = T_{k+1} / (1 - alpha_k), suffix S
        double T = Tfin, S = 0.0;
        const double bgterm = ga - (gc[0] * bg[0] + gc[1] * bg[1] + gc[2] * bg[2]);
        for (int k = (int)trace.size() - 1; k >= 0; --k) {
          const Composited& e = trace[k];
          const Proj<double>& g = pinned ? blendv[e.idx] : p64[e.idx];
          const double al = e.alpha;
          T = T / (1.0 - al);
          const double xk = gc[0] * g.col[0] + gc[1] * g.col[1] + gc[2] * g.col[2] + gd * g.z;
          const double wgt = al * T;
          double* acc_i = &mine[(size_t)e.idx * G2_N];
          acc_i[G2_R] += wgt * gc[0];
          acc_i[G2_G] += wgt * gc[1];
          acc_i[G2_BL] += wgt * gc[2];
          acc_i[G2_Z] += wgt * gd;
          const double galpha_k = T * (xk - S) + Tfin * bgterm / (1.0 - al);
          // the magnitudes of the summands (for the bound on float summation
          // error): each term as the method forms it, in absolute value
          const double galpha_abs = T * (std::fabs(xk) + std::fabs(S)) + std::fabs(Tfin * bgterm / (1.0 - al));
          if (amine) {
            double* ai = amine + (size_t)e.idx * G2_N;
            ai[G2_R] += std::fabs(wgt * gc[0]);
            ai[G2_G] += std::fabs(wgt * gc[1]);
            ai[G2_BL] += std::fabs(wgt * gc[2]);
            ai[G2_Z] += std::fabs(wgt * gd);
            if (!e.clamped) {
              const double gp = galpha_abs * al, dx = std::fabs(e.dx), dy = std::fabs(e.dy);
              ai[G2_O] += galpha_abs * e.G;
              ai[G2_U] += gp * (std::fabs(g.A) * dx + std::fabs(g.B) * dy);
              ai[G2_V] += gp * (std::fabs(g.B) * dx + std::fabs(g.C) * dy);
              ai[G2_A] += 0.5 * gp * dx * dx;
              ai[G2_B] += gp * dx * dy;
              ai[G2_C] += 0.5 * gp * dy * dy;
            }
          }
          S = al * xk + (1.0 - al) * S;
          if (e.clamped) continue;
          // alpha = o exp(power)
          acc_i[G2_O] += galpha_k * e.G;
          const double gpow = galpha_k * al;
          const double dx = e.dx, dy = e.dy;
          acc_i[G2_U] += gpow * (-(g.A * dx + g.B * dy));
          acc_i[G2_V] += gpow * (-(g.B * dx + g.C * dy));
          acc_i[G2_A] += gpow * (-0.5 * dx * dx);
          acc_i[G2_B] += gpow * (-dx * dy);
          acc_i[G2_C] += gpow * (-0.5 * dy * dy);
        }
      }
    }
  }
  g2out.assign((size_t)n * G2_N, 0.0);
  for (int t = 0; t < nt; ++t)
    for (size_t k = 0; k < g2out.size(); ++k) g2out[k] += acc[t][k];
  if (absout) {
    absout->assign((size_t)n * G2_N, 0.0);
    for (int t = 0; t < nt; ++t)
      for (size_t k = 0; k < absout->size(); ++k) (*absout)[k] += aacc[t][k];
  }
  p64out.swap(p64);
}

}  // namespace

extern "C" {

int orc_num_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}

// The FP32-mode exponential and, if tie is not null, the relative distance
// of the long double exp from the nearest float rounding midpoint.
void orc_exp32(const float* x, float* y, double* tie, int64_t n) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    y[i] = exp32(x[i]);
    if (tie) tie[i] = exp32_tie_distance(x[i]);
  }
}

// The FP32-mode activations (O1): scale = exp(log-scale) and opacity =
// 1 / (1 + exp(-logit)) in float, element by element.
void orc_activations(const float* logscale, const float* logit, float* scale, float* opacity, int64_t n) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    if (scale) scale[i] = exp32(logscale[i]);
    if (opacity) opacity[i] = 1.0f / (1.0f + exp32(-logit[i]));
  }
}

// Real SH basis values Y_k(dir) for k < (deg+1)^2, dirs unit vectors [n][3].
void orc_sh_basis(int deg, const double* dirs, int64_t n, double* out, double* grad /* [n][K][3] or null */) {
  const int K = (deg + 1) * (deg + 1);
  std::vector<Dual3> Y(K);
  for (int64_t i = 0; i < n; ++i) {
    Dual3 d[3];
    for (int k = 0; k < 3; ++k) { d[k] = Dual3(dirs[i * 3 + k]); d[k].d[k] = 1.0; }
    sh_basis_dual(deg, d, Y.data());
    for (int k = 0; k < K; ++k) {
      out[i * K + k] = Y[k].v;
      if (grad) for (int j = 0; j < 3; ++j) grad[(i * K + k) * 3 + j] = Y[k].d[j];
    }
  }
}

// Projection of every Gaussian. prec = 32 or 64. out[n][17] =
// u v z a b c A B C o r g b ex ey det visible; rect[n][4] = px0 py0 px1 py1.
int orc_project(int prec, const float* params, int64_t n, int64_t stride, int deg, const float* cam,
                int width, int height, float znear, double* out, int32_t* rect) {
  auto fill = [&](auto const& ps) {
    for (int64_t i = 0; i < n; ++i) {
      const auto& g = ps[i];
      double* o = out + i * 17;
      for (int k = 0; k < 17; ++k) o[k] = 0.0;
      int32_t* r = rect + i * 4;
      r[0] = r[1] = 0; r[2] = r[3] = -1;
      if (!g.vis) continue;
      o[0] = g.u; o[1] = g.v; o[2] = g.z; o[3] = g.a; o[4] = g.b; o[5] = g.c;
      o[6] = g.A; o[7] = g.B; o[8] = g.C; o[9] = g.o;
      o[10] = g.col[0]; o[11] = g.col[1]; o[12] = g.col[2];
      o[13] = g.ex; o[14] = g.ey; o[15] = g.det; o[16] = 1.0;
      r[0] = g.px0; r[1] = g.py0; r[2] = g.px1; r[3] = g.py1;
    }
  };
  if (prec == 32) fill(project_all<float>(params, n, stride, deg, make_cam<float>(cam, width, height), znear));
  else if (prec == 64) fill(project_all<double>(params, n, stride, deg, make_cam<double>(cam, width, height), (double)znear));
  else return -1;
  return 0;
}

// O7/O8: sorted instance list over all views. Global tile id = view offset +
// ty * tiles_x + tx. Order (global tile, FP32 depth bits, Gaussian index).
// Writes at most `capacity` entries and returns the total count in *count.
int orc_tile_list(const float* params, int64_t n, int64_t stride, int deg, int num_views, const float* cams,
                  const int32_t* wh, int tile_w, int tile_h, float znear, int64_t capacity,
                  uint32_t* out_tile, uint32_t* out_gid, int64_t* count) {
  struct Inst { uint32_t tile, zb; uint32_t gid; };
  std::vector<Inst> all;
  uint32_t offset = 0;
  for (int v = 0; v < num_views; ++v) {
    const int W = wh[2 * v], H = wh[2 * v + 1];
    const int tiles_x = (W + tile_w - 1) / tile_w, tiles_y = (H + tile_h - 1) / tile_h;
    std::vector<Proj<float>> p = project_all<float>(params, n, stride, deg, make_cam<float>(cams + 16 * v, W, H), znear);
    for (int64_t i = 0; i < n; ++i) {
      if (!p[i].vis) continue;
      const int tx0 = p[i].px0 / tile_w, tx1 = p[i].px1 / tile_w;
      const int ty0 = p[i].py0 / tile_h, ty1 = p[i].py1 / tile_h;
      for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx)
          all.push_back({offset + (uint32_t)(ty * tiles_x + tx), float_bits(p[i].z), (uint32_t)i});
    }
    offset += (uint32_t)(tiles_x * tiles_y);
  }
  std::sort(all.begin(), all.end(), [](const Inst& a, const Inst& b) {
    if (a.tile != b.tile) return a.tile < b.tile;
    if (a.zb != b.zb) return a.zb < b.zb;
    return a.gid < b.gid;
  });
  *count = (int64_t)all.size();
  for (int64_t k = 0; k < std::min<int64_t>(capacity, (int64_t)all.size()); ++k) {
    out_tile[k] = all[k].tile;
    out_gid[k] = all[k].gid;
  }
  return 0;
}

// Brute-force render of one view. mode 0: FP32; 1: FP64 values with FP32
// decisions; 2: FP64 values and decisions. prefilter skips pairs outside the
// Gaussian's FP32 pixel rectangle (exact by containment; modes 0 and 1 only).
// window (x0, y0, x1, y1, row_step) or null: only those pixels are written.
int orc_render(int mode, int prefilter, const float* params, int64_t n, int64_t stride, int deg, const float* cam,
               int width, int height, float znear, const float* bg, double* rgb, double* depth, double* alpha,
               double* tfinal, int32_t* ncomp, double* margin, const int32_t* window) {
  const PixelSet ps = pixel_set(window, width, height);
  if (mode == 0)
    render_view<float, float>(params, n, stride, deg, cam, width, height, znear, bg, prefilter != 0, rgb, depth, alpha, tfinal, ncomp, margin, ps);
  else if (mode == 1)
    render_view<float, double>(params, n, stride, deg, cam, width, height, znear, bg, prefilter != 0, rgb, depth, alpha, tfinal, ncomp, margin, ps);
  else if (mode == 2)
    render_view<double, double>(params, n, stride, deg, cam, width, height, znear, bg, false, rgb, depth, alpha, tfinal, ncomp, margin, ps);
  else return -1;
  return 0;
}

// Analytic gradient of sum_v <dL/dimage_v, image_v> with respect to the
// parameters, summed over views. pinned: 0 = FP64 decisions and values;
// 1 = FP32 decisions, FP64 values; 2 = FP32 decisions and FP32 screen-space
// splat values, FP64 arithmetic. Images of view v start at the offsets
// img_off[v] (pixels) in grgb ([3][H][W] per view), gdepth and galpha
// ([H][W] per view). grad[P][n] is overwritten. If g2 is not null it
// receives the screen-space gradients [V][n][10] (u v A B C o r g b z).
// windows ([V][5] as orc_render's window, or null): only those pixels are
// walked, as if the upstream gradient were zero elsewhere. gcam ([V][12] or
// null) receives each view's camera gradient: dL/dR row-major, then dL/dt.
// gabs ([P][n] or null) receives, per parameter, the sum over the pairs of
// the magnitudes of the terms a float implementation adds up (each
// screen-space term in absolute value, carried through the projection's
// Jacobian in absolute value): a bound on the gradient (|grad| <= gabs) whose
// size, next to |grad|, says how much the sum cancels.
int orc_backward(int pinned, const float* params, int64_t n, int64_t stride, int deg, int num_views,
                 const float* cams, const int32_t* wh, float znear, const float* bg, const float* grgb,
                 const float* gdepth, const float* galpha, double* grad, double* g2, const int32_t* windows,
                 double* gcam, double* gabs) {
  const int P = 11 + 3 * (deg + 1) * (deg + 1);
  for (int64_t k = 0; k < (int64_t)P * n; ++k) grad[k] = 0.0;
  if (gcam)
    for (int k = 0; k < 12 * num_views; ++k) gcam[k] = 0.0;
  if (gabs)
    for (int64_t k = 0; k < (int64_t)P * n; ++k) gabs[k] = 0.0;
  int64_t off = 0;
  for (int v = 0; v < num_views; ++v) {
    const int W = wh[2 * v], H = wh[2 * v + 1];
    std::vector<double> g2v, absv;
    std::vector<Proj<double>> p64;
    blend_backward_view(params, n, stride, deg, cams + 16 * v, W, H, znear, bg, grgb + 3 * off, gdepth + off,
                        galpha + off, pinned != 0, pinned == 2, g2v, p64,
                        pixel_set(windows ? windows + 5 * v : nullptr, W, H), gabs ? &absv : nullptr);
    if (g2) std::memcpy(g2 + (size_t)v * n * G2_N, g2v.data(), sizeof(double) * n * G2_N);
    Cam<double> c64 = make_cam<double>(cams + 16 * v, W, H);
    const int nt = omp_get_max_threads();
    std::vector<double> gc((size_t)nt * 12, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      if (!p64[i].vis) continue;
      const double* gi = &g2v[(size_t)i * G2_N];
      bool any = false;
      for (int k = 0; k < G2_N; ++k) any = any || gi[k] != 0.0;
      if (!any) continue;
      project_backward_one(params, stride, i, deg, c64, p64[i], gi, grad, n,
                           gcam ? &gc[(size_t)omp_get_thread_num() * 12] : nullptr);
    }
    if (gcam)
      for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 12; ++k) gcam[v * 12 + k] += gc[(size_t)t * 12 + k];
    if (gabs) {
      // the summands' magnitudes carried to the parameters through the
      // projection's Jacobian in absolute value, column by column:
      // gabs += sum_k |J^T e_k| abs_k
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        if (!p64[i].vis) continue;
        const double* ai = &absv[(size_t)i * G2_N];
        std::vector<double> col(P);
        for (int k = 0; k < G2_N; ++k) {
          if (ai[k] == 0.0) continue;
          double unit[G2_N] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
          unit[k] = 1.0;
          std::fill(col.begin(), col.end(), 0.0);
          project_backward_one(params, stride, i, deg, c64, p64[i], unit, col.data(), 1, nullptr, 0);
          for (int q = 0; q < P; ++q) gabs[(int64_t)q * n + i] += std::fabs(col[q]) * ai[k];
        }
      }
    }
    off += (int64_t)W * H;
  }
  return 0;
}

}  // extern "C"
