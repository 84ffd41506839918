// EWA projection of 3D Gaussians to screen-space conics, and its backward.
//
// Compiled with -ffp-contract=off and correctly rounded float division and
// square root: the forward is a fixed sequence of IEEE-754 float operations
// (see the projection contract in the design notes), so that binning and the
// depth keys are reproducible bit for bit by an independent implementation
// of the same sequence.
//
// Image formation (paper Sec. II-A: anisotropic 3D Gaussians with mean,
// covariance and opacity, colour from spherical harmonics; Sec. II-B: the
// renderer that drives mapping): Sigma = R diag(s)^2 R^T from the unit
// quaternion and exp(log-scale); camera-space mean t = W mean + t_cw;
// screen covariance Sigma' = J W Sigma W^T J^T + 0.3 I with the pinhole
// Jacobian J taken at the mean (direction clamped to 1.3x the half field of
// view); conic = inverse of Sigma'. Binning uses the opacity-independent
// bounding box of the ellipse q = 11.2 (q = squared Mahalanobis distance):
// alpha >= 1/255 with opacity <= 1 requires q <= 2 ln 255 < 11.2, so no
// contributing pixel lies outside its Gaussian's tiles.

#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr float kDilation = 0.3f;
constexpr float kClampFov = 1.3f;
constexpr float kQMax = 11.2f;
constexpr int kLdsViews = 64;           // views per chunk of the several-view projection (descriptors in LDS)
constexpr int kProjHist = 4 * 256;      // depth-key digit counters of the projection (four 8-bit digits)
constexpr bool kStageCoef = true;       // several views: colour coefficients staged in LDS once per Gaussian

__device__ __forceinline__ bool finitef(float x) { return __builtin_isfinite(x); }

// ---------------------------------------------------------------------------
// exp(x) correctly rounded to float, for the scales and the opacity.
//
// The device's double-precision exp (a few ulp of double at most) is rounded
// to float. That is the correctly rounded result unless the double lies so
// close to a midpoint between two neighbouring floats that its own error
// could put it on the wrong side; only then is exp evaluated again in
// double-double arithmetic (about 100 significant bits) and the side of that
// midpoint decided from it. Every float input gets the float nearest to its
// exact exponential.
// ---------------------------------------------------------------------------
struct DD {
  double hi, lo;
};

// hi + lo exactly, for |a| >= |b| or a == 0
__device__ __forceinline__ DD dd_fast(double a, double b) {
  const double s = a + b;
  return DD{s, b - (s - a)};
}
// a + b exactly, any order of magnitude
__device__ __forceinline__ DD dd_sum(double a, double b) {
  const double s = a + b;
  const double bv = s - a;
  return DD{s, (a - (s - bv)) + (b - bv)};
}
__device__ __forceinline__ DD dd_add(DD a, DD b) {
  DD s = dd_sum(a.hi, b.hi);
  return dd_fast(s.hi, s.lo + (a.lo + b.lo));
}
__device__ __forceinline__ DD dd_mul(DD a, DD b) {
  const double p = a.hi * b.hi;
  const double e = fma(a.hi, b.hi, -p);          // exact low part of a.hi * b.hi
  return dd_fast(p, e + (a.hi * b.lo + a.lo * b.hi));
}
__device__ __forceinline__ DD dd_div_small(DD a, double k) {
  const double q = a.hi / k;
  const double r = fma(-q, k, a.hi);             // exact remainder
  return dd_fast(q, (r + a.lo) / k);
}

// exp(x) as hi + lo for a float x with a finite, nonzero float exponential.
// x = n ln2 + r with |r| <= ln2/2 (ln2 in two doubles whose sum is within
// 2^-106 of it; n ln2_hi formed exactly with an fma), then e^r from its
// Taylor series summed to 24 terms (the remainder is below 2^-110), scaled
// by 2^n.
__device__ __noinline__ DD exp_dd(float xf) {
  const double ln2_hi = 0x1.62e42fefa39efp-1;
  const double ln2_lo = 0x1.abc9e3b39803fp-56;
  const double x = (double)xf;
  const double n = rint(x * 0x1.71547652b82fep+0);
  const double p = n * ln2_hi;
  const double pe = fma(n, ln2_hi, -p);
  DD r = dd_sum(x, -p);
  r = dd_add(r, dd_sum(-pe, -(n * ln2_lo)));
  DD term{1.0, 0.0}, sum{1.0, 0.0};
  for (int k = 1; k <= 24; ++k) {
    term = dd_div_small(dd_mul(term, r), (double)k);
    sum = dd_add(sum, term);
  }
  const int e = (int)n;
  return DD{ldexp(sum.hi, e), ldexp(sum.lo, e)};
}

__device__ __forceinline__ float exp32_rn(float x) {
  const double y = exp((double)x);
  const float f = (float)y;
  if (!finitef(f)) return f;                     // overflow to inf, or a NaN input
  const double fd = (double)f;
  const uint32_t fb = __float_as_uint(f);        // f >= 0
  // the neighbour of f on y's side and the midpoint between them (exact)
  double nb;
  if (y >= fd) nb = (double)__uint_as_float(fb + 1u);
  else nb = f == 0.0f ? -0x1p-149 : (double)__uint_as_float(fb - 1u);
  const double mid = 0.5 * (fd + nb);
  if (fabs(y - mid) > 0x1p-48 * y) return f;
  const DD e = exp_dd(x);
  const double side = (e.hi - mid) + e.lo;       // e.hi - mid is exact (Sterbenz)
  const double lo = fmin(fd, nb), hi = fmax(fd, nb);
  if (side > 0.0) return (float)hi;
  if (side < 0.0) return (float)lo;
  return (__float_as_uint((float)lo) & 1u) ? (float)hi : (float)lo;   // exact tie: even
}

// Opacity = sigmoid(logit): one correctly rounded float operation per step.
__device__ __forceinline__ float opacity_of(float logit) { return 1.0f / (1.0f + exp32_rn(-logit)); }


// Correctly rounded square root. The hardware square root is within one ulp;
// the result is moved to the neighbour whose rounding interval contains the
// exact root, decided by comparing x with the squares of the midpoints
// between neighbouring floats (exact in double: 25-bit midpoints square to at
// most 50 bits, and no float is the square of a midpoint).
__device__ __forceinline__ float sqrt_rn(float x) {
  float y = __builtin_sqrtf(x);
  if (!(x > 0.0f) || !finitef(x)) return y;
  const double xd = (double)x;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const float up = __uint_as_float(__float_as_uint(y) + 1u);   // y > 0: neighbours by bit pattern
    const float dn = __uint_as_float(__float_as_uint(y) - 1u);
    const double mu = 0.5 * ((double)y + (double)up);
    const double md = 0.5 * ((double)y + (double)dn);
    if (mu * mu < xd) y = up;
    else if (md * md > xd) y = dn;
  }
  return y;
}

// Real spherical harmonics (Condon-Shortley phase) up to degree 3 as
// polynomials of the unit direction, normalisations sqrt((2l+1)/(4pi)
// (l-m)!/(l+m)!) (times sqrt 2 for m != 0) folded into the constants.
constexpr float SH_C0 = 0.28209479177387814f;
constexpr float SH_C1 = 0.4886025119029199f;
constexpr float SH_C2a = 1.0925484305920792f;
constexpr float SH_C2b = 0.31539156525252005f;
constexpr float SH_C2c = 0.5462742152960396f;
constexpr float SH_K0 = 0.5900435899266435f;
constexpr float SH_K1 = 2.890611442640554f;
constexpr float SH_K2 = 0.4570457994644658f;
constexpr float SH_K3 = 0.3731763325901154f;
constexpr float SH_K5 = 1.445305721320277f;

__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* Y) {
  Y[0] = SH_C0;
  if (deg < 1) return;
  Y[1] = -SH_C1 * y;
  Y[2] = SH_C1 * z;
  Y[3] = -SH_C1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = SH_C2a * (x * y);
  Y[5] = -SH_C2a * (y * z);
  Y[6] = SH_C2b * (2.0f * zz - xx - yy);
  Y[7] = -SH_C2a * (x * z);
  Y[8] = SH_C2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -SH_K0 * y * (3.0f * xx - yy);
  Y[10] = SH_K1 * (x * y) * z;
  Y[11] = -SH_K2 * y * (4.0f * zz - xx - yy);
  Y[12] = SH_K3 * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -SH_K2 * x * (4.0f * zz - xx - yy);
  Y[14] = SH_K5 * z * (xx - yy);
  Y[15] = -SH_K0 * x * (xx - 3.0f * yy);
}

// A Gaussian the projection can never draw for its values alone: a
// non-finite mean, log-scale, rotation or opacity logit, or a rotation
// quaternion of zero (or non-finite) norm. Such Gaussians are culled in
// every view and counted once per render.
__device__ __forceinline__ bool degenerate_gaussian(const float* __restrict__ P, int64_t stride, int64_t i) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 11; ++k) ok = ok && finitef(P[k * stride + i]);
  if (!ok) return true;
  const float qw = P[6 * stride + i], qx = P[7 * stride + i], qy = P[8 * stride + i], qz = P[9 * stride + i];
  float ss = qw * qw + qx * qx;
  ss = ss + qy * qy;
  ss = ss + qz * qz;
  return !(ss > 0.0f) || !finitef(ss);
}

// The part of a Gaussian's projection that no view changes: its mean and its
// world covariance Sigma = R diag(s)^2 R^T from the unit quaternion and
// exp(log-scale). Computed once per Gaussian however many views see it.
struct GaussLocal {
  float mx, my, mz;
  float Sig[9];
};

// False if the Gaussian cannot be drawn (a non-finite value among planes
// 0..10, a zero quaternion).
__device__ __forceinline__ bool gaussian_local(const float* __restrict__ P, int64_t stride, int64_t i,
                                               GaussLocal& L) {
  float raw[11];
#pragma unroll
  for (int k = 0; k < 11; ++k) raw[k] = P[k * stride + i];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 11; ++k) ok = ok && finitef(raw[k]);
  if (!ok) return false;
  L.mx = raw[0];
  L.my = raw[1];
  L.mz = raw[2];
  float sc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) sc[k] = exp32_rn(raw[3 + k]);
  const float qw = raw[6], qx = raw[7], qy = raw[8], qz = raw[9];
  float ss = qw * qw + qx * qx;
  ss = ss + qy * qy;
  ss = ss + qz * qz;
  if (!(ss > 0.0f) || !finitef(ss)) return false;
  const float qn = sqrt_rn(ss);
  const float w = __fdiv_rn(qw, qn), x = __fdiv_rn(qx, qn), y = __fdiv_rn(qy, qn), z = __fdiv_rn(qz, qn);
  float R[9], M[9];
  R[0] = 1.0f - 2.0f * (y * y + z * z);
  R[1] = 2.0f * (x * y - w * z);
  R[2] = 2.0f * (x * z + w * y);
  R[3] = 2.0f * (x * y + w * z);
  R[4] = 1.0f - 2.0f * (x * x + z * z);
  R[5] = 2.0f * (y * z - w * x);
  R[6] = 2.0f * (x * z - w * y);
  R[7] = 2.0f * (y * z + w * x);
  R[8] = 1.0f - 2.0f * (x * x + y * y);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[r * 3 + k] = R[r * 3 + k] * sc[k];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float acc = M[r * 3 + 0] * M[k * 3 + 0] + M[r * 3 + 1] * M[k * 3 + 1];
      L.Sig[r * 3 + k] = acc + M[r * 3 + 2] * M[k * 3 + 2];
    }
  return true;
}

// Everything the projection computes for one (view, Gaussian).
struct ProjState {
  float Sig[9];
  float tx, ty, tz, xi, yi;
  bool xclamp, yclamp;
  float J00, J02, J11, J12, Tm[6];
  float a, b, c, det, A, B, C;
  float u, v;
  int x0, y0, x1, y1;
};

// The view part of the projection contract: returns false if the Gaussian is
// culled in this view.
__device__ __forceinline__ bool project_view(const GaussLocal& L, const ViewDesc& V, float znear, ProjState& g) {
  const float mx = L.mx, my = L.my, mz = L.mz;
#pragma unroll
  for (int k = 0; k < 9; ++k) g.Sig[k] = L.Sig[k];
  const float* W = V.R;
  float tc[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    float acc = W[r * 3 + 0] * mx + W[r * 3 + 1] * my;
    acc = acc + W[r * 3 + 2] * mz;
    tc[r] = acc + V.t[r];
  }
  g.tx = tc[0]; g.ty = tc[1]; g.tz = tc[2];
  if (!(g.tz >= znear)) return false;
  const float limx = kClampFov * __fdiv_rn(0.5f * (float)V.width, V.fx);
  const float limy = kClampFov * __fdiv_rn(0.5f * (float)V.height, V.fy);
  const float xr = __fdiv_rn(g.tx, g.tz), yr = __fdiv_rn(g.ty, g.tz);
  g.xclamp = (xr < -limx) || (xr > limx);
  g.yclamp = (yr < -limy) || (yr > limy);
  g.xi = fminf(fmaxf(xr, -limx), limx);
  g.yi = fminf(fmaxf(yr, -limy), limy);
  g.J00 = __fdiv_rn(V.fx, g.tz);
  g.J02 = __fdiv_rn(-(V.fx * g.xi), g.tz);
  g.J11 = __fdiv_rn(V.fy, g.tz);
  g.J12 = __fdiv_rn(-(V.fy * g.yi), g.tz);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g.Tm[k] = g.J00 * W[0 * 3 + k] + g.J02 * W[2 * 3 + k];
    g.Tm[3 + k] = g.J11 * W[1 * 3 + k] + g.J12 * W[2 * 3 + k];
  }
  float U[6];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float acc = g.Tm[r * 3 + 0] * g.Sig[0 * 3 + k] + g.Tm[r * 3 + 1] * g.Sig[1 * 3 + k];
      U[r * 3 + k] = acc + g.Tm[r * 3 + 2] * g.Sig[2 * 3 + k];
    }
  float a = U[0] * g.Tm[0] + U[1] * g.Tm[1];
  a = a + U[2] * g.Tm[2];
  float b = U[0] * g.Tm[3] + U[1] * g.Tm[4];
  b = b + U[2] * g.Tm[5];
  float c = U[3] * g.Tm[3] + U[4] * g.Tm[4];
  c = c + U[5] * g.Tm[5];
  a = a + kDilation;
  c = c + kDilation;
  const float det = a * c - b * b;
  if (!(det > 0.0f) || !finitef(det) || !finitef(a) || !finitef(b) || !finitef(c)) return false;
  g.a = a; g.b = b; g.c = c; g.det = det;
  g.A = __fdiv_rn(c, det);
  g.B = -__fdiv_rn(b, det);
  g.C = __fdiv_rn(a, det);
  g.u = __fdiv_rn(V.fx * g.tx, g.tz) + V.cx;
  g.v = __fdiv_rn(V.fy * g.ty, g.tz) + V.cy;
  if (!finitef(g.u) || !finitef(g.v)) return false;
  const float ex = sqrt_rn(kQMax * a);
  const float ey = sqrt_rn(kQMax * c);
  float x0 = ceilf((g.u - ex) - 0.5f);
  float x1 = floorf((g.u + ex) - 0.5f);
  float y0 = ceilf((g.v - ey) - 0.5f);
  float y1 = floorf((g.v + ey) - 0.5f);
  x0 = fmaxf(x0, 0.0f);
  y0 = fmaxf(y0, 0.0f);
  x1 = fminf(x1, (float)(V.width - 1));
  y1 = fminf(y1, (float)(V.height - 1));
  if (x0 > x1 || y0 > y1) return false;
  g.x0 = (int)x0; g.x1 = (int)x1; g.y0 = (int)y0; g.y1 = (int)y1;
  return true;
}

// The whole projection contract of one (view, Gaussian).
__device__ __forceinline__ bool project_geometry(const float* __restrict__ P, int64_t stride, int64_t i,
                                                 const ViewDesc& V, float znear, ProjState& g) {
  GaussLocal L;
  return gaussian_local(P, stride, i, L) && project_view(L, V, znear, g);
}

// Conservative early cull from the mean and the largest scale only: true
// when the Gaussian is surely behind the near plane or surely projects
// outside the image, so the full projection (which reads and transforms the
// rotation and does the correctly rounded arithmetic) can be skipped. The
// near-plane test repeats the projection's own float operations, so it takes
// the same decision; the lateral test bounds the extent from above
//   a <= |row 0 of J|^2 s_max^2 + 0.3 <= (fx / z)^2 (1 + lim_x^2) s_max^2 + 0.3
// (W is a rotation) and keeps a margin of 1% and a pixel for rounding.
// mx, my, mz: the mean; lmax: the largest log-scale.
__device__ __forceinline__ bool surely_culled_at(float mx, float my, float mz, float lmax, const ViewDesc& V,
                                                 float znear) {
  const float* W = V.R;
  float tc[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    float acc = W[r * 3 + 0] * mx + W[r * 3 + 1] * my;
    acc = acc + W[r * 3 + 2] * mz;
    tc[r] = acc + V.t[r];
  }
  if (!(tc[2] >= znear)) return finitef(tc[2]);         // exactly the projection's near-plane cull
  if (!finitef(lmax) || lmax > 20.0f) return false;
  const float smax = __expf(lmax) * 1.01f;    // a bound: 1 % covers the fast exp's error
  const float iz = 1.0f / tc[2];
  const float limx = kClampFov * 0.5f * (float)V.width / V.fx, limy = kClampFov * 0.5f * (float)V.height / V.fy;
  const float jx = V.fx * iz, jy = V.fy * iz;
  const float ax = jx * jx * (1.0f + limx * limx) * smax * smax + kDilation;
  const float ay = jy * jy * (1.0f + limy * limy) * smax * smax + kDilation;
  const float exb = sqrtf(kQMax * ax) * 1.01f + 1.0f, eyb = sqrtf(kQMax * ay) * 1.01f + 1.0f;
  const float u = V.fx * tc[0] * iz + V.cx, v = V.fy * tc[1] * iz + V.cy;
  if (!finitef(u) || !finitef(v) || !finitef(exb) || !finitef(eyb)) return false;
  return (u + exb < 0.0f) || (u - exb > (float)V.width) || (v + eyb < 0.0f) || (v - eyb > (float)V.height);
}

__device__ __forceinline__ float largest_log_scale(const float* __restrict__ P, int64_t stride, int64_t i) {
  return fmaxf(fmaxf(P[3 * stride + i], P[4 * stride + i]), P[5 * stride + i]);
}

// The colour coefficients of one Gaussian, plane j = 3 k + channel of the
// parameter rows 11.. : read from the parameter array ...
struct GlobalCoef {
  const float* __restrict__ P;
  int64_t stride, i;
  __device__ __forceinline__ float operator()(int j) const { return P[(11 + j) * stride + i]; }
};
// ... or from registers (an array of them) ...
struct ArrayCoef {
  const float* c;
  __device__ __forceinline__ float operator()(int j) const { return c[j]; }
};
// Sums of the SH coefficients' gradient terms over views, in registers.
struct ArraySink {
  float* g;
  __device__ __forceinline__ void operator()(int j, bool passed, float t) const {
    if (passed) g[j] += t;
  }
};
// ... or, where one thread projects a Gaussian into several views, the
// constant terms from registers and the rest from the thread's own column of
// an LDS array that it filled once (3 (K - 1) rows of `pitch` words).
struct StagedCoef {
  float dc[3];
  const float* col;
  int pitch;
  __device__ __forceinline__ float operator()(int j) const { return j < 3 ? dc[j] : col[(j - 3) * pitch]; }
};

// Colour of one Gaussian of mean (mx, my, mz) seen from the view (before and
// after max(0, .)).
template <class Coef>
__device__ __forceinline__ void project_colour(float mx, float my, float mz, const Coef& coef, int deg,
                                               const ViewDesc& V, float* raw, float* col) {
  float Y[16];
  float dx = 0.0f, dy = 0.0f, dz = 0.0f;
  if (deg > 0) {
    dx = mx - V.campos[0];
    dy = my - V.campos[1];
    dz = mz - V.campos[2];
    const float nrm = sqrtf(dx * dx + dy * dy + dz * dz);
    const float inv = 1.0f / nrm;
    dx *= inv; dy *= inv; dz *= inv;
  }
  sh_basis(deg, dx, dy, dz, Y);
  const int K = (deg + 1) * (deg + 1);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = SH_C0 * coef(ch);
    for (int k = 1; k < K; ++k) acc = acc + Y[k] * coef(3 * k + ch);
    raw[ch] = acc + 0.5f;
    col[ch] = fmaxf(raw[ch], 0.0f);
  }
}

// Projection of one (view, Gaussian) splat s into its records; returns
// whether it is visible (and then its depth key).
// L, good, o: the Gaussian's view-independent part, whether it can be drawn
// at all, and its opacity.
// coef: its colour coefficients.
template <class Coef>
__device__ __forceinline__ bool project_splat(const Coef& coef, int deg, int64_t s, const ViewDesc& V, int tile_w,
                                              int tile_h, float znear, bool skip_geometry, const GaussLocal& L,
                                              bool good, float o, Splat* __restrict__ splats,
                                              int4* __restrict__ rect, uint32_t* __restrict__ ntiles,
                                              uint32_t* __restrict__ zkey, uint32_t* key_out) {
  ProjState g;
  bool vis = !skip_geometry && good && project_view(L, V, znear, g);
  float raw[3], col[3];
  if (vis) {
    project_colour(L.mx, L.my, L.mz, coef, deg, V, raw, col);
    vis = finitef(col[0]) && finitef(col[1]) && finitef(col[2]);
  }
  if (!vis) {
    // a tile count of zero marks the splat as not listed; its other records
    // are never read
    ntiles[s] = 0u;
    return false;
  }
  const int tx0 = g.x0 / tile_w, tx1 = g.x1 / tile_w, ty0 = g.y0 / tile_h, ty1 = g.y1 / tile_h;
  Splat sp;
  sp.w0 = make_float4(g.u, g.v, g.tz, o);
  // spare words: the tile rectangle for the emission (first global tile id;
  // width | the view's tile pitch << 16)
  sp.w1 = make_float4(g.A, g.B, g.C, __uint_as_float((uint32_t)(V.tile_offset + ty0 * V.tiles_x + tx0)));
  sp.w2 = make_float4(col[0], col[1], col[2], __uint_as_float((uint32_t)(tx1 - tx0 + 1) | ((uint32_t)V.tiles_x << 16)));
  splats[s] = sp;
  rect[s] = make_int4(g.x0, g.y0, g.x1, g.y1);
  ntiles[s] = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
  const uint32_t key = __float_as_uint(g.tz);
  zkey[s] = key;
  *key_out = key;
  return true;
}

// One view: one thread per Gaussian. Several views: one thread per Gaussian,
// in two phases per chunk of up to kLdsViews views. First the conservative
// cull of every view of the chunk with all lanes on the same view, so that
// the empty records of the culled views are written coalesced; it leaves each
// lane a mask of the views it must project. Then each lane walks its own
// mask, so that the full projection runs with the wavefront's lanes busy even
// where most of the views are culled.
// MULTI: the several-view form (a separate instantiation, so that each form
// gets the registers of its own body). Its dynamic LDS holds the chunk's view
// descriptors (read per lane in the second phase) and, when `stage` is set,
// each thread's colour coefficients past the constant terms, loaded once per
// Gaussian rather than once per view it is projected into.
template <bool MULTI>
__global__ void __launch_bounds__(256) project_kernel(const float* __restrict__ P, int64_t n, int64_t stride, int deg,
                                                      int num_views, const ViewDesc* __restrict__ views, int tile_w,
                                                      int tile_h, float znear, Splat* __restrict__ splats,
                                                      int4* __restrict__ rect, uint32_t* __restrict__ ntiles,
                                                      uint32_t* __restrict__ zkey, uint32_t* __restrict__ zhist,
                                                      int zrb, int zpasses, uint32_t* __restrict__ nonfinite,
                                                      bool stage) {
  // digit histograms of the visible splats' depth keys for the radix sort
  // that follows (zpasses digits of zrb bits; zpasses * 2^zrb <= kProjHist)
  __shared__ uint32_t s_hist[kProjHist];
  const int zR = 1 << zrb;
  if (zhist)
    for (int e = threadIdx.x; e < zpasses * zR; e += blockDim.x) s_hist[e] = 0u;
  auto count_key = [&](uint32_t key) {
    if (zhist)
      for (int p = 0; p < zpasses; ++p) atomicAdd(&s_hist[p * zR + ((key >> (zrb * p)) & (zR - 1))], 1u);
  };
  extern __shared__ float s_dyn[];
  ViewDesc* s_views = reinterpret_cast<ViewDesc*>(s_dyn);
  const int chunk_views = min(num_views, kLdsViews);
  float* s_sh = s_dyn + chunk_views * (int)(sizeof(ViewDesc) / 4) + threadIdx.x;
  const int nsh = stage ? 3 * ((deg + 1) * (deg + 1) - 1) : 0;
  auto load_views = [&](int first, int count) {
    const int words = (int)(sizeof(ViewDesc) / 4) * count;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(views + first);
    for (int e = threadIdx.x; e < words; e += blockDim.x) reinterpret_cast<uint32_t*>(s_dyn)[e] = src[e];
  };
  const bool views_resident = num_views <= kLdsViews;
  if (MULTI && views_resident) load_views(0, num_views);   // else per chunk, in the loop
  __syncthreads();
  const int64_t stride_t = (int64_t)gridDim.x * blockDim.x;
  // the loop runs the same number of times on every lane (and every wave of
  // the block), so the wave-wide votes and the block barriers below see all
  // lanes
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x; i0 < n; i0 += stride_t) {
    const int64_t i = i0 + threadIdx.x;
    const bool mine = i < n;
    if (nonfinite) {
      const unsigned long long bad = __ballot(mine && degenerate_gaussian(P, stride, i));
      if (bad && (threadIdx.x & 63) == 0) atomicAdd(nonfinite, (uint32_t)__popcll(bad));
    }
    if (!MULTI) {
      uint32_t key;
      if (mine) {
        const bool skip = surely_culled_at(P[0 * stride + i], P[1 * stride + i], P[2 * stride + i],
                                           largest_log_scale(P, stride, i), views[0], znear);
        GaussLocal L;
        bool good = false;
        float o = 0.0f;
        if (!skip) {
          good = gaussian_local(P, stride, i, L);
          o = opacity_of(P[10 * stride + i]);
        }
        if (project_splat(GlobalCoef{P, stride, i}, deg, i, views[0], tile_w, tile_h, znear, skip, L, good, o,
                          splats, rect, ntiles, zkey, &key))
          count_key(key);
      }
      continue;
    }
    float mx = 0.0f, my = 0.0f, mz = 0.0f, lmax = 0.0f;
    if (mine) {
      mx = P[0 * stride + i];
      my = P[1 * stride + i];
      mz = P[2 * stride + i];
      lmax = largest_log_scale(P, stride, i);
    }
    // phase one over views [vb, vb + nv), whose descriptors are in LDS
    auto cull_chunk = [&](int vb, int nv) {
      uint64_t keep = 0;
      for (int v = 0; v < nv; ++v) {
        if (!mine) continue;
        if (surely_culled_at(mx, my, mz, lmax, s_views[v], znear))
          ntiles[(int64_t)(vb + v) * n + i] = 0u;
        else
          keep |= 1ull << v;
      }
      return keep;
    };
    if (!views_resident) {
      __syncthreads();                       // every lane is done with the previous Gaussian's last chunk
      load_views(0, chunk_views);
      __syncthreads();
    }
    uint64_t keep = cull_chunk(0, chunk_views);
    // the Gaussian's view-independent part (and its staged coefficients),
    // formed once, out of the view walk, so that the walk's body holds no
    // exponential; skipped where the first chunk culls every view
    bool good = false;
    GaussLocal L;
    float o = 0.0f;
    StagedCoef sc;
    sc.col = s_sh;
    sc.pitch = blockDim.x;
    if (mine && (keep || !views_resident)) {
      good = gaussian_local(P, stride, i, L);
      o = opacity_of(P[10 * stride + i]);
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) sc.dc[ch] = P[(11 + ch) * stride + i];
      for (int j = 0; j < nsh; ++j) s_sh[j * (int)blockDim.x] = P[(14 + j) * stride + i];
    }
    for (int vb = 0;;) {
      // phase two: each lane walks its own kept views
      while (__any(keep != 0)) {
        if (keep) {
          const int v = __builtin_ctzll(keep);
          keep &= keep - 1;
          const int64_t s = (int64_t)(vb + v) * n + i;
          uint32_t key;
          const bool vis = stage ? project_splat(sc, deg, s, s_views[v], tile_w, tile_h, znear, false, L, good, o,
                                                 splats, rect, ntiles, zkey, &key)
                                 : project_splat(GlobalCoef{P, stride, i}, deg, s, s_views[v], tile_w, tile_h,
                                                 znear, false, L, good, o, splats, rect, ntiles, zkey, &key);
          if (vis) count_key(key);
        }
      }
      vb += kLdsViews;
      if (vb >= num_views) break;
      const int nv = min(kLdsViews, num_views - vb);
      __syncthreads();                       // every lane is done with the previous chunk
      load_views(vb, nv);
      __syncthreads();
      keep = cull_chunk(vb, nv);
    }
  }
  if (zhist) {
    __syncthreads();
    uint32_t* dst = zhist + (size_t)(blockIdx.x % kHistCopies) * (zpasses * zR);
    for (int e = threadIdx.x; e < zpasses * zR; e += blockDim.x) {
      const uint32_t c = s_hist[e];
      if (c) atomicAdd(dst + e, c);
    }
  }
}

// Projection intermediates in double for the backward chain rule (the chain
// rule is cheap next to the blend, and double keeps its cancellations -- the
// conic inverse, the Jacobian terms of the depth -- out of the gradient).
// The Gaussian's view-independent part: scales, unit quaternion, rotation,
// M = R diag(s), Sigma = M M^T, opacity.
struct LocalD {
  double s[3], qn, qh[4], R[9], M[9], Sig[9], o;
};
// Its part in one view.
struct ViewD {
  double tx, ty, tz, xi, yi;
  bool xclamp, yclamp;
  double Tm[6];
  double a, b, c, det;
};

__device__ __forceinline__ void local_f64(const float* __restrict__ P, int64_t stride, int64_t i, LocalD& g) {
#pragma unroll
  for (int k = 0; k < 3; ++k) g.s[k] = exp((double)P[(3 + k) * stride + i]);
  const double qw = P[6 * stride + i], qx = P[7 * stride + i], qy = P[8 * stride + i], qz = P[9 * stride + i];
  g.qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const double w = qw / g.qn, x = qx / g.qn, y = qy / g.qn, z = qz / g.qn;
  g.qh[0] = w; g.qh[1] = x; g.qh[2] = y; g.qh[3] = z;
  double* R = g.R;
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) g.M[r * 3 + k] = R[r * 3 + k] * g.s[k];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      g.Sig[r * 3 + k] = g.M[r * 3 + 0] * g.M[k * 3 + 0] + g.M[r * 3 + 1] * g.M[k * 3 + 1] +
                         g.M[r * 3 + 2] * g.M[k * 3 + 2];
  g.o = 1.0 / (1.0 + exp(-(double)P[10 * stride + i]));
}

// Sigma of local_f64 alone (what the per-view chain rule needs; the rest of
// the local part is formed again once the views are summed, rather than held
// in registers across the view loop).
__device__ __forceinline__ void sigma_f64(const float* __restrict__ P, int64_t stride, int64_t i, double* Sig) {
  LocalD L;
  local_f64(P, stride, i, L);
#pragma unroll
  for (int k = 0; k < 9; ++k) Sig[k] = L.Sig[k];
}

__device__ __forceinline__ void view_f64(const double* Sig, double mx, double my, double mz, const ViewDesc& V,
                                         ViewD& g) {
  const float* W = V.R;
  g.tx = W[0] * mx + W[1] * my + W[2] * mz + V.t[0];
  g.ty = W[3] * mx + W[4] * my + W[5] * mz + V.t[1];
  g.tz = W[6] * mx + W[7] * my + W[8] * mz + V.t[2];
  const double limx = (double)kClampFov * (0.5 * (double)V.width / (double)V.fx);
  const double limy = (double)kClampFov * (0.5 * (double)V.height / (double)V.fy);
  const double xr = g.tx / g.tz, yr = g.ty / g.tz;
  g.xclamp = (xr < -limx) || (xr > limx);
  g.yclamp = (yr < -limy) || (yr > limy);
  g.xi = fmin(fmax(xr, -limx), limx);
  g.yi = fmin(fmax(yr, -limy), limy);
  const double J00 = V.fx / g.tz, J02 = -(V.fx * g.xi) / g.tz;
  const double J11 = V.fy / g.tz, J12 = -(V.fy * g.yi) / g.tz;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g.Tm[k] = J00 * W[k] + J02 * W[6 + k];
    g.Tm[3 + k] = J11 * W[3 + k] + J12 * W[6 + k];
  }
  double U[6];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      U[r * 3 + k] = g.Tm[r * 3 + 0] * Sig[k] + g.Tm[r * 3 + 1] * Sig[3 + k] + g.Tm[r * 3 + 2] * Sig[6 + k];
  g.a = U[0] * g.Tm[0] + U[1] * g.Tm[1] + U[2] * g.Tm[2] + (double)kDilation;
  g.b = U[0] * g.Tm[3] + U[1] * g.Tm[4] + U[2] * g.Tm[5];
  g.c = U[3] * g.Tm[3] + U[4] * g.Tm[4] + U[5] * g.Tm[5] + (double)kDilation;
  g.det = g.a * g.c - g.b * g.b;
}

__device__ __forceinline__ void sh_basis_d(int deg, double x, double y, double z, double* Y) {
  Y[0] = 0.28209479177387814;
  if (deg < 1) return;
  const double c1 = 0.4886025119029199;
  Y[1] = -c1 * y; Y[2] = c1 * z; Y[3] = -c1 * x;
  if (deg < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  Y[4] = 1.0925484305920792 * x * y;
  Y[5] = -1.0925484305920792 * y * z;
  Y[6] = 0.31539156525252005 * (2.0 * zz - xx - yy);
  Y[7] = -1.0925484305920792 * x * z;
  Y[8] = 0.5462742152960396 * (xx - yy);
  if (deg < 3) return;
  Y[9] = -0.5900435899266435 * y * (3.0 * xx - yy);
  Y[10] = 2.890611442640554 * x * y * z;
  Y[11] = -0.4570457994644658 * y * (4.0 * zz - xx - yy);
  Y[12] = 0.3731763325901154 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
  Y[13] = -0.4570457994644658 * x * (4.0 * zz - xx - yy);
  Y[14] = 1.445305721320277 * z * (xx - yy);
  Y[15] = -0.5900435899266435 * x * (xx - 3.0 * yy);
}

// d/d(x, y, z) of sum_k c_k Y_k for the polynomials above.
// One colour channel's SH coefficients, read from the interleaved float array
// coef[3 k + ch] and widened at each use (no double copy held in registers).
struct ChannelCoef {
  const float* coef;
  int ch;
  __device__ __forceinline__ double operator[](int k) const { return (double)coef[3 * k + ch]; }
};

template <class C>
__device__ __forceinline__ void sh_dir_grad_d(int deg, double x, double y, double z, const C& c, double* g) {
  g[0] = g[1] = g[2] = 0.0;
  if (deg < 1) return;
  const double C1 = 0.4886025119029199, C2a = 1.0925484305920792, C2b = 0.31539156525252005,
               C2c = 0.5462742152960396, K0 = 0.5900435899266435, K1 = 2.890611442640554,
               K2 = 0.4570457994644658, K3 = 0.3731763325901154, K5 = 1.445305721320277;
  g[1] -= C1 * c[1];
  g[2] += C1 * c[2];
  g[0] -= C1 * c[3];
  if (deg < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  g[0] += C2a * y * c[4];            g[1] += C2a * x * c[4];
  g[1] -= C2a * z * c[5];            g[2] -= C2a * y * c[5];
  g[0] -= 2.0 * C2b * x * c[6];      g[1] -= 2.0 * C2b * y * c[6];     g[2] += 4.0 * C2b * z * c[6];
  g[0] -= C2a * z * c[7];            g[2] -= C2a * x * c[7];
  g[0] += 2.0 * C2c * x * c[8];      g[1] -= 2.0 * C2c * y * c[8];
  if (deg < 3) return;
  g[0] -= 6.0 * K0 * x * y * c[9];   g[1] -= K0 * (3.0 * xx - 3.0 * yy) * c[9];
  g[0] += K1 * y * z * c[10];        g[1] += K1 * x * z * c[10];      g[2] += K1 * x * y * c[10];
  g[0] += 2.0 * K2 * x * y * c[11];  g[1] -= K2 * (4.0 * zz - xx - 3.0 * yy) * c[11];  g[2] -= 8.0 * K2 * y * z * c[11];
  g[0] -= 6.0 * K3 * x * z * c[12];  g[1] -= 6.0 * K3 * y * z * c[12];  g[2] += K3 * (6.0 * zz - 3.0 * xx - 3.0 * yy) * c[12];
  g[0] -= K2 * (4.0 * zz - 3.0 * xx - yy) * c[13];  g[1] += 2.0 * K2 * x * y * c[13];  g[2] -= 8.0 * K2 * x * z * c[13];
  g[0] += 2.0 * K5 * x * z * c[14];  g[1] -= 2.0 * K5 * y * z * c[14];  g[2] += K5 * (xx - yy) * c[14];
  g[0] -= K0 * (3.0 * xx - 3.0 * yy) * c[15];  g[1] += 6.0 * K0 * x * y * c[15];
}

// Chain rule of one (view, Gaussian) pair from its screen-space gradient G:
// adds to the mean and SH gradients, and to the sums over views of dL/dSigma
// (gSig, 3x3) and dL/dopacity (gO), which finish_local turns into the scale,
// rotation and opacity-logit gradients once per Gaussian (the maps from
// Sigma and from the opacity are the same in every view). POSE: also adds
// the pair's part of the gradient with respect to the view's camera to
// gpose[12]: dL/dR (row-major) and dL/dt of x_cam = R x + t. R acts through
// the camera-space mean, through T = J R and, for view-dependent colour,
// through the camera centre -R^T t.
// The colour part of one (view, Gaussian) pair's chain rule: from the colour
// gradients gcol[3] to the SH coefficients (gsh(j, passed, term): the term of
// plane j, passed false where the clamp stops it) and, for DEG > 0, to
// dL/d(mean - camera centre) through the viewing direction (gview, =).
// Real SH basis function k at the unit direction (x, y, z) and its gradient
// with respect to (x, y, z) as a polynomial (the same functions as sh_basis_d
// and sh_dir_grad_d, one at a time; k is a constant after unrolling).
__device__ __forceinline__ double sh_term_d(int k, double x, double y, double z, double* d) {
  const double C0 = 0.28209479177387814, C1 = 0.4886025119029199, C2a = 1.0925484305920792,
               C2b = 0.31539156525252005, C2c = 0.5462742152960396, K0 = 0.5900435899266435,
               K1 = 2.890611442640554, K2 = 0.4570457994644658, K3 = 0.3731763325901154,
               K5 = 1.445305721320277;
  const double xx = x * x, yy = y * y, zz = z * z;
  switch (k) {
    case 0: d[0] = 0.0; d[1] = 0.0; d[2] = 0.0; return C0;
    case 1: d[0] = 0.0; d[1] = -C1; d[2] = 0.0; return -C1 * y;
    case 2: d[0] = 0.0; d[1] = 0.0; d[2] = C1; return C1 * z;
    case 3: d[0] = -C1; d[1] = 0.0; d[2] = 0.0; return -C1 * x;
    case 4: d[0] = C2a * y; d[1] = C2a * x; d[2] = 0.0; return C2a * x * y;
    case 5: d[0] = 0.0; d[1] = -C2a * z; d[2] = -C2a * y; return -C2a * y * z;
    case 6: d[0] = -2.0 * C2b * x; d[1] = -2.0 * C2b * y; d[2] = 4.0 * C2b * z; return C2b * (2.0 * zz - xx - yy);
    case 7: d[0] = -C2a * z; d[1] = 0.0; d[2] = -C2a * x; return -C2a * x * z;
    case 8: d[0] = 2.0 * C2c * x; d[1] = -2.0 * C2c * y; d[2] = 0.0; return C2c * (xx - yy);
    case 9: d[0] = -6.0 * K0 * x * y; d[1] = -K0 * (3.0 * xx - 3.0 * yy); d[2] = 0.0;
      return -K0 * y * (3.0 * xx - yy);
    case 10: d[0] = K1 * y * z; d[1] = K1 * x * z; d[2] = K1 * x * y; return K1 * x * y * z;
    case 11: d[0] = 2.0 * K2 * x * y; d[1] = -K2 * (4.0 * zz - xx - 3.0 * yy); d[2] = -8.0 * K2 * y * z;
      return -K2 * y * (4.0 * zz - xx - yy);
    case 12: d[0] = -6.0 * K3 * x * z; d[1] = -6.0 * K3 * y * z; d[2] = K3 * (6.0 * zz - 3.0 * xx - 3.0 * yy);
      return K3 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    case 13: d[0] = -K2 * (4.0 * zz - 3.0 * xx - yy); d[1] = 2.0 * K2 * x * y; d[2] = -8.0 * K2 * x * z;
      return -K2 * x * (4.0 * zz - xx - yy);
    case 14: d[0] = 2.0 * K5 * x * z; d[1] = -2.0 * K5 * y * z; d[2] = K5 * (xx - yy); return K5 * z * (xx - yy);
    default: d[0] = -K0 * (3.0 * xx - 3.0 * yy); d[1] = 6.0 * K0 * x * y; d[2] = 0.0;
      return -K0 * x * (xx - 3.0 * yy);
  }
}

// The colour part of one (view, Gaussian) pair's chain rule: from the colour
// gradients gcol[3] to the SH coefficients (gsh(j, passed, term): the term of
// plane j, passed false where the clamp stops it) and, for DEG > 0, to
// dL/d(mean - camera centre) through the viewing direction (gview, =). Two
// walks over the basis: the raw colours (for the clamp), then the gradients,
// each basis function formed where it is used (few registers at degree 3).
template <int DEG, class Coef, class Sink>
__device__ __forceinline__ void colour_chain(const float* __restrict__ P, int64_t stride, int64_t i,
                                             const ViewDesc& V, const float* gcol, const Coef& coef, const Sink& gsh,
                                             double* gview) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  double dir[3] = {0.0, 0.0, 0.0}, dnorm = 1.0;
  if (DEG > 0) {
    dir[0] = (double)P[0 * stride + i] - (double)V.campos[0];
    dir[1] = (double)P[1 * stride + i] - (double)V.campos[1];
    dir[2] = (double)P[2 * stride + i] - (double)V.campos[2];
    dnorm = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    dir[0] /= dnorm; dir[1] /= dnorm; dir[2] /= dnorm;
  }
  double raw[3] = {0.5, 0.5, 0.5};
  auto first_walk = [&](int k) {
    double d[3];
    const double Yk = sh_term_d(k, dir[0], dir[1], dir[2], d);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) raw[ch] += (double)coef(3 * k + ch) * Yk;
  };
#pragma unroll
  for (int k = 0; k < K; ++k) first_walk(k);
  // the clamp at zero passes no gradient
  double gc[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) gc[ch] = raw[ch] < 0.0 ? 0.0 : (double)gcol[ch];
  double gdir[3] = {0.0, 0.0, 0.0};
  // the second walk forms the basis again rather than keeping the first
  // walk's values (an empty asm hides that the direction is the same)
  double ux = dir[0], uy = dir[1], uz = dir[2];
  asm volatile("" : "+v"(ux), "+v"(uy), "+v"(uz));
  auto second_walk = [&](int k) {
    double d[3];
    const double Yk = sh_term_d(k, ux, uy, uz, d);
    double w = 0.0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      gsh(3 * k + ch, !(raw[ch] < 0.0), (float)(gc[ch] * Yk));
      w += gc[ch] * (double)coef(3 * k + ch);
    }
    if (DEG > 0) {
      gdir[0] += w * d[0];
      gdir[1] += w * d[1];
      gdir[2] += w * d[2];
    }
  };
#pragma unroll
  for (int k = 0; k < K; ++k) second_walk(k);
#pragma unroll
  for (int j = 0; j < 3; ++j) gview[j] = 0.0;
  if (DEG > 0) {
    const double dot = dir[0] * gdir[0] + dir[1] * gdir[1] + dir[2] * gdir[2];
#pragma unroll
    for (int j = 0; j < 3; ++j) gview[j] = (gdir[j] - dir[j] * dot) / dnorm;
  }
}

// COLOUR false: the colour part is left out (sh_backward_kernel forms it).
template <int DEG, bool POSE = false, bool COLOUR = true>
__device__ __forceinline__ void chain_view(const float* __restrict__ P, int64_t stride, int64_t i, const ViewDesc& V,
                                           const double* Sig, const float* G, const float* coef, double* gmean,
                                           double* gSig, double& gO, float* gsh, double* gpose = nullptr) {
  ViewD g;
  view_f64(Sig, (double)P[0 * stride + i], (double)P[1 * stride + i], (double)P[2 * stride + i], V, g);
  gO += (double)G[G2_O];
  double gview[3] = {0.0, 0.0, 0.0};   // dL/d(mean - camera centre) through the colour
  if (COLOUR) {
    colour_chain<DEG>(P, stride, i, V, G + G2_R, ArrayCoef{coef}, ArraySink{gsh}, gview);
#pragma unroll
    for (int j = 0; j < 3; ++j) gmean[j] += gview[j];
  }
  // conic (A, B, C) = (c, -b, a) / det
  const double a = g.a, b = g.b, c = g.c, det = g.det;
  const double id = 1.0 / det, id2 = id * id;
  const double gA = (double)G[G2_A], gB = (double)G[G2_B], gC = (double)G[G2_C];
  const double ga = (-gA * c * c + gB * b * c - gC * b * b) * id2;
  const double gb = (2.0 * gA * b * c - 2.0 * gB * b * b + 2.0 * gC * a * b) * id2 - gB * id;
  const double gc_ = (-gA * b * b + gB * a * b - gC * a * a) * id2;
  // Sigma' = T Sigma T^T
  const double* T0 = g.Tm;
  const double* T1 = g.Tm + 3;
  const double* S = Sig;
  double ST0[3], ST1[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    ST0[r] = S[r * 3 + 0] * T0[0] + S[r * 3 + 1] * T0[1] + S[r * 3 + 2] * T0[2];
    ST1[r] = S[r * 3 + 0] * T1[0] + S[r * 3 + 1] * T1[1] + S[r * 3 + 2] * T1[2];
  }
  double gT0[3], gT1[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    gT0[r] = 2.0 * ga * ST0[r] + gb * ST1[r];
    gT1[r] = gb * ST0[r] + 2.0 * gc_ * ST1[r];
  }
  double gSS[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      gSS[r * 3 + k] = 2.0 * ga * T0[r] * T0[k] + gb * (T0[r] * T1[k] + T1[r] * T0[k]) +
                       2.0 * gc_ * T1[r] * T1[k];
  const float* W = V.R;
  double gJ00 = 0, gJ02 = 0, gJ11 = 0, gJ12 = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    gJ00 += gT0[k] * W[k];
    gJ02 += gT0[k] * W[6 + k];
    gJ11 += gT1[k] * W[3 + k];
    gJ12 += gT1[k] * W[6 + k];
  }
  const double tx = g.tx, ty = g.ty, tz = g.tz, fx = V.fx, fy = V.fy;
  const double itz = 1.0 / tz, itz2 = itz * itz;
  double gtx = 0, gty = 0, gtz = 0;
  gtz += -gJ00 * fx * itz2 - gJ11 * fy * itz2 + gJ02 * fx * g.xi * itz2 + gJ12 * fy * g.yi * itz2;
  if (!g.xclamp) {
    const double gxi = -gJ02 * fx * itz;
    gtx += gxi * itz;
    gtz += -gxi * tx * itz2;
  }
  if (!g.yclamp) {
    const double gyi = -gJ12 * fy * itz;
    gty += gyi * itz;
    gtz += -gyi * ty * itz2;
  }
  const double gu = (double)G[G2_U], gv = (double)G[G2_V];
  gtx += gu * fx * itz;
  gtz += -gu * fx * tx * itz2;
  gty += gv * fy * itz;
  gtz += -gv * fy * ty * itz2;
  gtz += (double)G[G2_Z];
#pragma unroll
  for (int j = 0; j < 3; ++j) gmean[j] += W[j] * gtx + W[3 + j] * gty + W[6 + j] * gtz;
  if (POSE) {
    const double mu[3] = {(double)P[0 * stride + i], (double)P[1 * stride + i], (double)P[2 * stride + i]};
    const double gt[3] = {gtx, gty, gtz};
    const double J00 = fx * itz, J02 = -(fx * g.xi) * itz, J11 = fy * itz, J12 = -(fy * g.yi) * itz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      // x_cam = R mu + t; T = J R with J's rows (J00, 0, J02), (0, J11, J12);
      // centre c = -R^T t and dL/dc = -gview
      gpose[0 * 3 + k] += gt[0] * mu[k] + J00 * gT0[k] + gview[k] * (double)V.t[0];
      gpose[1 * 3 + k] += gt[1] * mu[k] + J11 * gT1[k] + gview[k] * (double)V.t[1];
      gpose[2 * 3 + k] += gt[2] * mu[k] + J02 * gT0[k] + J12 * gT1[k] + gview[k] * (double)V.t[2];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
      gpose[9 + r] += gt[r] + (double)W[r * 3 + 0] * gview[0] + (double)W[r * 3 + 1] * gview[1] +
                      (double)W[r * 3 + 2] * gview[2];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) gSig[k] += gSS[k];
}

// From the view sums of dL/dSigma and dL/dopacity to the gradients of the
// log-scales, the (unnormalised) quaternion and the opacity logit.
__device__ __forceinline__ void finish_local(const LocalD& L, const double* gSig, double gO, double* gls, double* gq,
                                             double& glogit) {
  glogit += gO * L.o * (1.0 - L.o);
  // Sigma = M M^T, M = R diag(s)
  double gM[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      gM[r * 3 + k] = gSig[r * 3 + 0] * L.M[k] + gSig[r * 3 + 1] * L.M[3 + k] + gSig[r * 3 + 2] * L.M[6 + k];
  double gR[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) gR[r * 3 + k] = gM[r * 3 + k] * L.s[k];
#pragma unroll
  for (int k = 0; k < 3; ++k)
    gls[k] += (gM[k] * L.R[k] + gM[3 + k] * L.R[3 + k] + gM[6 + k] * L.R[6 + k]) * L.s[k];
  const double w = L.qh[0], x = L.qh[1], y = L.qh[2], z = L.qh[3];
  const double gw = 2.0 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
  const double gx = 2.0 * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5] + z * gR[6] +
                           w * gR[7] - 2.0 * x * gR[8]);
  const double gy = 2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
                           z * gR[7] - 2.0 * y * gR[8]);
  const double gz = 2.0 * (-2.0 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0 * z * gR[4] +
                           y * gR[5] + x * gR[6] + y * gR[7]);
  const double dot = w * gw + x * gx + y * gy + z * gz;
  gq[0] += (gw - w * dot) / L.qn;
  gq[1] += (gx - x * dot) / L.qn;
  gq[2] += (gy - y * dot) / L.qn;
  gq[3] += (gz - z * dot) / L.qn;
}

// The backward's per-lane view walks read the view descriptors from LDS
// (up to kLdsViews of them; else from global memory). Called by every thread
// of the workgroup, before any early exit.
__device__ __forceinline__ const ViewDesc* stage_views(const ViewDesc* __restrict__ views, int num_views,
                                                       ViewDesc* s_views) {
  if (num_views > kLdsViews) return views;
  const int words = (int)(sizeof(ViewDesc) / 4) * num_views;
  for (int e = threadIdx.x; e < words; e += blockDim.x)
    reinterpret_cast<uint32_t*>(s_views)[e] = reinterpret_cast<const uint32_t*>(views)[e];
  __syncthreads();
  return s_views;
}

// Bit v set for each view vb + v (v < 64) that lists Gaussian i.
__device__ __forceinline__ uint64_t listed_views(const uint32_t* __restrict__ ntiles, int64_t n, int64_t i, int vb,
                                                 int num_views) {
  uint64_t m = 0;
  const int nv = min(64, num_views - vb);
  for (int v = 0; v < nv; ++v)
    if (ntiles[(int64_t)(vb + v) * n + i] != 0u) m |= 1ull << v;
  return m;
}

// Chain rule from the screen-space gradients (u, v, conic, opacity, colour,
// depth) of every view to the parameters, summed over views, in double.
// One thread per Gaussian, so the parameter gradients need no atomics. For
// DEG > 0 the colour part (the SH coefficients and the mean's share through
// the viewing direction) is left to sh_backward_kernel, launched after this
// one: the two halves each fit in fewer registers than the whole (for SH
// degree 3, 256 VGPRs and one wave per SIMD together).
template <int DEG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) project_backward_kernel(const float* __restrict__ P, int64_t n, int64_t stride,
                                                               int num_views, const ViewDesc* __restrict__ views,
                                                               float* __restrict__ g2,
                                                               const uint32_t* __restrict__ ntiles,
                                                               float* __restrict__ grad, bool overwrite,
                                                               bool zero_g2, IterCounters counters) {
  constexpr bool kColour = DEG == 0;
  constexpr int K = kColour ? 1 : 0;
  if (counters.stats && blockIdx.x == 0 && threadIdx.x == 0) count_iteration(counters);
  __shared__ ViewDesc s_views[kLdsViews];
  const ViewDesc* vsrc = stage_views(views, num_views, s_views);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double gmean[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, glogit = 0.0;
    float gsh[3 * K + 1];      // SH gradients (degree 0 only): one term per view, float is enough
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) gsh[k] = 0.0f;
    float coef[3 * K + 1];     // SH coefficients, read once
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) coef[k] = P[(11 + k) * stride + i];
    bool touched = false;
    double Sig[9];             // formed at the first view that passes the Gaussian a gradient
    double gSig[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gO = 0.0;
    // each lane walks the views that list its Gaussian, in view order
    for (int vb = 0; vb < num_views; vb += 64) {
     for (uint64_t seen = listed_views(ntiles, n, i, vb, num_views); seen; seen &= seen - 1) {
      const int cur = vb + __builtin_ctzll(seen);
      float* gv = g2 + ((int64_t)cur * n + i) * G2_N;
      float G[G2_N];
      bool any = false;
#pragma unroll
      for (int k = 0; k < G2_N; ++k) {
        G[k] = gv[k];
        any = any || (G[k] != 0.0f);
      }
      if (!any) continue;
      // the mapping iteration leaves the accumulators clean for its next
      // replay: only rows of splats with tiles ever receive gradients (the
      // colour half clears them where it runs)
      if (zero_g2 && kColour) {
#pragma unroll
        for (int k = 0; k < G2_N; ++k) gv[k] = 0.0f;
      }
      if (!touched) sigma_f64(P, stride, i, Sig);
      touched = true;
      chain_view<DEG, false, kColour>(P, stride, i, vsrc[cur], Sig, G, coef, gmean, gSig, gO, gsh);
     }
    }
    if (touched) {
      LocalD L;
      local_f64(P, stride, i, L);
      finish_local(L, gSig, gO, gls, gq, glogit);
    }
    if (overwrite) {
      // every plane is written (zero for a Gaussian no view composited)
#pragma unroll
      for (int j = 0; j < 3; ++j) grad[(0 + j) * stride + i] = (float)gmean[j];
#pragma unroll
      for (int j = 0; j < 3; ++j) grad[(3 + j) * stride + i] = (float)gls[j];
#pragma unroll
      for (int j = 0; j < 4; ++j) grad[(6 + j) * stride + i] = (float)gq[j];
      grad[10 * stride + i] = (float)glogit;
#pragma unroll
      for (int k = 0; k < 3 * K; ++k) grad[(11 + k) * stride + i] = gsh[k];
      continue;
    }
    if (!touched) continue;
#pragma unroll
    for (int j = 0; j < 3; ++j) grad[(0 + j) * stride + i] += (float)gmean[j];
#pragma unroll
    for (int j = 0; j < 3; ++j) grad[(3 + j) * stride + i] += (float)gls[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) grad[(6 + j) * stride + i] += (float)gq[j];
    grad[10 * stride + i] += (float)glogit;
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) grad[(11 + k) * stride + i] += gsh[k];
  }
}

// Waves per SIMD asked of the compiler for the colour half, whose
// higher-order SH coefficients sit in LDS (degree 3: 45 KB of them per
// workgroup, so three workgroups per CU).
template <int DEG>
constexpr int kShBackwardWaves = DEG == 3 ? 2 : 4;

// The colour half of the chain rule for DEG > 0 (after
// project_backward_kernel, which left it out): per Gaussian, over its views,
// the SH coefficients' gradient and the mean's share through the viewing
// direction, written (overwrite: every SH plane) or added (mean planes: always
// added, after the geometry half). Clears the screen-space gradient rows it
// reads when zero_g2. The coefficients past degree 0 are read once into the
// thread's own column of LDS (registers hold the gradient sums).
template <int DEG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kShBackwardWaves<DEG>))) sh_backward_kernel(const float* __restrict__ P, int64_t n, int64_t stride,
                                                          int num_views, const ViewDesc* __restrict__ views,
                                                          float* __restrict__ g2,
                                                          const uint32_t* __restrict__ ntiles,
                                                          float* __restrict__ grad, bool overwrite, bool zero_g2) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  static_assert(DEG > 0, "the colour half exists for view-dependent colour only");
  __shared__ ViewDesc s_views[kLdsViews];
  __shared__ float s_sh[3 * (K - 1) * 256];
  const ViewDesc* vsrc = stage_views(views, num_views, s_views);
  StagedCoef coef;
  coef.col = s_sh + threadIdx.x;
  coef.pitch = 256;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float gsh[3 * K];
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) gsh[k] = 0.0f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) coef.dc[ch] = P[(11 + ch) * stride + i];
#pragma unroll
    for (int j = 0; j < 3 * (K - 1); ++j) s_sh[j * 256 + threadIdx.x] = P[(14 + j) * stride + i];
    double gmean[3] = {0, 0, 0};
    bool touched = false;
    for (int vb = 0; vb < num_views; vb += 64) {
     for (uint64_t seen = listed_views(ntiles, n, i, vb, num_views); seen; seen &= seen - 1) {
      const int cur = vb + __builtin_ctzll(seen);
      float* gv = g2 + ((int64_t)cur * n + i) * G2_N;
      float G[G2_N];
      bool any = false;
#pragma unroll
      for (int k = 0; k < G2_N; ++k) {
        G[k] = gv[k];
        any = any || (G[k] != 0.0f);
      }
      if (!any) continue;
      if (zero_g2) {
#pragma unroll
        for (int k = 0; k < G2_N; ++k) gv[k] = 0.0f;
      }
      if (G[G2_R] == 0.0f && G[G2_G] == 0.0f && G[G2_BL] == 0.0f) continue;
      double gview[3];
      colour_chain<DEG>(P, stride, i, vsrc[cur], G + G2_R, coef, ArraySink{gsh}, gview);
      touched = true;
#pragma unroll
      for (int j = 0; j < 3; ++j) gmean[j] += gview[j];
     }
    }
    if (overwrite) {
#pragma unroll
      for (int k = 0; k < 3 * K; ++k) grad[(11 + k) * stride + i] = gsh[k];
    } else if (touched) {
#pragma unroll
      for (int k = 0; k < 3 * K; ++k) grad[(11 + k) * stride + i] += gsh[k];
    }
    if (touched) {
#pragma unroll
      for (int j = 0; j < 3; ++j) grad[j * stride + i] += (float)gmean[j];
    }
  }
}

// Camera gradient of every view: per (view, Gaussian) the chain rule of
// chain_view with the pose terms, summed over each workgroup (in double) and
// added with one atomic per (workgroup, view, component). gcam[v][12] += dL/dR
// (row-major), dL/dt; twist[v][6] (if not null) += the gradient with respect
// to a left perturbation exp(xi^) [R | t] of the pose, xi = (rho, phi): dL/drho
// = dL/dt and dL/dphi = the axial vector of A - A^T, A = dL/dR R^T + dL/dt t^T.
// The loops are uniform over each workgroup (every thread reaches every
// reduction).
template <int DEG>
__global__ void __launch_bounds__(256) pose_backward_kernel(const float* __restrict__ P, int64_t n, int64_t stride,
                                                            int num_views, const ViewDesc* __restrict__ views,
                                                            const float* __restrict__ g2,
                                                            const uint32_t* __restrict__ ntiles,
                                                            double* __restrict__ gcam, double* __restrict__ twist) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  __shared__ double red[4][12];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    const bool mine = i < n;
    float coef[3 * K];
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) coef[k] = mine ? P[(11 + k) * stride + i] : 0.0f;
    double Sig[9];
    bool haveS = false;
    for (int cur = 0; cur < num_views; ++cur) {
      double gp[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) gp[k] = 0.0;
      if (mine && ntiles[(int64_t)cur * n + i] != 0u) {
        const float* gv = g2 + ((int64_t)cur * n + i) * G2_N;
        float G[G2_N];
        bool any = false;
#pragma unroll
        for (int k = 0; k < G2_N; ++k) {
          G[k] = gv[k];
          any = any || (G[k] != 0.0f);
        }
        if (any) {
          if (!haveS) sigma_f64(P, stride, i, Sig);
          haveS = true;
          double gmean[3] = {0, 0, 0}, gSig[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gO = 0.0;
          float gsh[3 * K];
#pragma unroll
          for (int k = 0; k < 3 * K; ++k) gsh[k] = 0.0f;
          chain_view<DEG, true>(P, stride, i, views[cur], Sig, G, coef, gmean, gSig, gO, gsh, gp);
        }
      }
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        double x = gp[k];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
        if (lane == 0) red[wave][k] = x;
      }
      __syncthreads();
      if (threadIdx.x < 12) {
        const int k = threadIdx.x;
        const double sum = red[0][k] + red[1][k] + red[2][k] + red[3][k];
        if (sum != 0.0) atomicAdd(gcam + cur * 12 + k, sum);
      }
      if (twist && threadIdx.x == 0) {
        double Gs[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) Gs[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
        const ViewDesc& V = views[cur];
        double A[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            A[r * 3 + c] = Gs[r * 3 + 0] * (double)V.R[c * 3 + 0] + Gs[r * 3 + 1] * (double)V.R[c * 3 + 1] +
                           Gs[r * 3 + 2] * (double)V.R[c * 3 + 2] + Gs[9 + r] * (double)V.t[c];
        const double tw[6] = {Gs[9], Gs[10], Gs[11], A[7] - A[5], A[2] - A[6], A[3] - A[1]};
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (tw[k] != 0.0) atomicAdd(twist + cur * 6 + k, tw[k]);
      }
      __syncthreads();
    }
  }
}

// Inspection copy of one view's splats; the screen covariance (a, b, c) is
// not kept by the forward, so it is recomputed here by the same projection.
__global__ void export_splats_kernel(const float* __restrict__ P, int64_t n, int64_t stride,
                                     const ViewDesc* __restrict__ view, float znear, const Splat* __restrict__ splats,
                                     const int4* __restrict__ rect, const uint32_t* __restrict__ ntiles,
                                     float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float* o = out + i * 16;
    const bool vis = ntiles[i] != 0u;
    const int4 r = vis ? rect[i] : make_int4(0, 0, -1, -1);
    Splat s;
    if (vis) {
      s = splats[i];
    } else {
      s.w0 = make_float4(0.f, 0.f, 0.f, 0.f);
      s.w1 = s.w0;
      s.w2 = s.w0;
    }
    ProjState g;
    const bool geo = vis && project_geometry(P, stride, i, *view, znear, g);
    o[0] = s.w0.x; o[1] = s.w0.y; o[2] = s.w0.z;
    o[3] = geo ? g.a : 0.f;
    o[4] = geo ? g.b : 0.f;
    o[5] = geo ? g.c : 0.f;
    o[6] = s.w1.x; o[7] = s.w1.y; o[8] = s.w1.z;
    o[9] = s.w0.w;
    o[10] = s.w2.x; o[11] = s.w2.y; o[12] = s.w2.z;
    o[13] = vis ? (float)r.x : 0.f;
    o[14] = vis ? (float)r.y : 0.f;
    o[15] = vis ? (float)r.z : -1.f;
  }
}

// The activations of O1 as the projection computes them: scale[k][n] =
// exp(log-scale k) and opacity[n] = sigmoid(logit), each correctly rounded
// where the projection's float operations are.
__global__ void __launch_bounds__(256) activations_kernel(const float* __restrict__ P, int64_t n, int64_t stride,
                                                          float* __restrict__ scale, float* __restrict__ opacity) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (scale) {
#pragma unroll
      for (int k = 0; k < 3; ++k) scale[k * n + i] = exp32_rn(P[(3 + k) * stride + i]);
    }
    if (opacity) opacity[i] = opacity_of(P[10 * stride + i]);
  }
}

int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

}  // namespace

void launch_project(const float* params, int64_t n, int64_t stride, int deg, int num_views, const ViewDesc* views,
                    int tile_w, int tile_h, float znear, Splat* splats, int4* rect, uint32_t* ntiles,
                    uint32_t* zkey, uint32_t* zhist, int zrb, int zpasses, uint32_t* nonfinite, hipStream_t st) {
  if (n == 0 || num_views == 0) return;
  if (zpasses * (1 << zrb) > kProjHist) zhist = nullptr;
  if (num_views == 1) {
    project_kernel<false><<<grid_for(n, 256), 256, 0, st>>>(params, n, stride, deg, num_views, views, tile_w, tile_h,
                                                            znear, splats, rect, ntiles, zkey, zhist, zrb, zpasses,
                                                            nonfinite, false);
    return;
  }
  // the chunk's view descriptors and (staged) 3 (K - 1) coefficient rows per
  // thread: at most 64 * 108 B + 45 * 256 * 4 B = 52 KB of dynamic LDS
  const bool stage = kStageCoef && deg > 0;
  const size_t lds = (size_t)std::min(num_views, kLdsViews) * sizeof(ViewDesc) +
                     (stage ? (size_t)3 * ((deg + 1) * (deg + 1) - 1) * 256 * sizeof(float) : 0);
  project_kernel<true><<<grid_for(n, 256), 256, lds, st>>>(params, n, stride, deg, num_views, views, tile_w, tile_h,
                                                           znear, splats, rect, ntiles, zkey, zhist, zrb, zpasses,
                                                           nonfinite, stage);
}

void launch_activations(const float* params, int64_t n, int64_t stride, float* scale, float* opacity,
                        hipStream_t st) {
  if (n == 0 || (!scale && !opacity)) return;
  activations_kernel<<<grid_for(n, 256), 256, 0, st>>>(params, n, stride, scale, opacity);
}

void launch_project_backward(const float* params, int64_t n, int64_t stride, int deg, int num_views,
                             const ViewDesc* views, float znear, float* g2, const uint32_t* ntiles, float* grad,
                             bool overwrite, bool zero_g2, const IterCounters* counters, hipStream_t st) {
  (void)znear;
  if (n == 0) return;
  const IterCounters ic = counters ? *counters : IterCounters{nullptr, nullptr, nullptr, 0};
  const int gsz = grid_for(n, 256);
  switch (deg) {
    case 0:
      project_backward_kernel<0><<<gsz, 256, 0, st>>>(params, n, stride, num_views, views, g2, ntiles, grad, overwrite,
                                                          zero_g2, ic);
      break;
    case 1:
      project_backward_kernel<1><<<gsz, 256, 0, st>>>(params, n, stride, num_views, views, g2, ntiles, grad, overwrite,
                                                          zero_g2, ic);
      sh_backward_kernel<1><<<gsz, 256, 0, st>>>(params, n, stride, num_views, views, g2, ntiles, grad, overwrite,
                                                     zero_g2);
      break;
    case 2:
      project_backward_kernel<2><<<gsz, 256, 0, st>>>(params, n, stride, num_views, views, g2, ntiles, grad, overwrite,
                                                          zero_g2, ic);
      sh_backward_kernel<2><<<gsz, 256, 0, st>>>(params, n, stride, num_views, views, g2, ntiles, grad, overwrite,
                                                     zero_g2);
      break;
    default:
      project_backward_kernel<3><<<gsz, 256, 0, st>>>(params, n, stride, num_views, views, g2, ntiles, grad, overwrite,
                                                          zero_g2, ic);
      sh_backward_kernel<3><<<gsz, 256, 0, st>>>(params, n, stride, num_views, views, g2, ntiles, grad, overwrite,
                                                     zero_g2);
      break;
  }
}

void launch_pose_backward(const float* params, int64_t n, int64_t stride, int deg, int num_views,
                          const ViewDesc* views, const float* g2, const uint32_t* ntiles, double* gcam, double* twist,
                          hipStream_t st) {
  if (n == 0) return;
  const int gsz = grid_for(n, 256);
  switch (deg) {
    case 0: pose_backward_kernel<0><<<gsz, 256, 0, st>>>(params, n, stride, num_views, views, g2, ntiles, gcam, twist); break;
    case 1: pose_backward_kernel<1><<<gsz, 256, 0, st>>>(params, n, stride, num_views, views, g2, ntiles, gcam, twist); break;
    case 2: pose_backward_kernel<2><<<gsz, 256, 0, st>>>(params, n, stride, num_views, views, g2, ntiles, gcam, twist); break;
    default: pose_backward_kernel<3><<<gsz, 256, 0, st>>>(params, n, stride, num_views, views, g2, ntiles, gcam, twist); break;
  }
}

void launch_export_splats(const float* params, int64_t n, int64_t stride, const ViewDesc* view, float znear,
                          const Splat* splats, const int4* rect, const uint32_t* ntiles, float* out,
                          hipStream_t st) {
  if (n == 0) return;
  export_splats_kernel<<<grid_for(n, 256), 256, 0, st>>>(params, n, stride, view, znear, splats, rect, ntiles, out);
}

}  // namespace gsr
