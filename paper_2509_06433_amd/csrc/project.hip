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

// Exponential by Cody-Waite reduction: x = n ln2 + r, ln2 split into a head
// with 15 significant bits (so n * head is exact) and a tail; e^r by its
// degree-7 Taylor polynomial in Horner form; result scaled by 2^n.
__device__ __forceinline__ float exp_cw(float x) {
  x = fminf(fmaxf(x, -87.0f), 88.0f);
  const float n = rintf(x * 1.44269504088896341f);
  float r = x - n * 0.693145751953125f;
  r = r - n * 1.4286068203094173e-06f;
  float p = 1.98412698412698413e-4f;
  p = p * r + 1.38888888888888889e-3f;
  p = p * r + 8.33333333333333333e-3f;
  p = p * r + 4.16666666666666667e-2f;
  p = p * r + 1.66666666666666667e-1f;
  p = p * r + 0.5f;
  p = p * r + 1.0f;
  p = p * r + 1.0f;
  return ldexpf(p, (int)n);
}

__device__ __forceinline__ bool finitef(float x) { return __builtin_isfinite(x); }

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

// Gradient of sum_k c_k Y_k with respect to the (unnormalised) direction,
// treating each Y_k as the polynomial above.
__device__ __forceinline__ void sh_dir_grad(int deg, float x, float y, float z, const float* c, float* g) {
  g[0] = g[1] = g[2] = 0.0f;
  if (deg < 1) return;
  g[1] += -SH_C1 * c[1];
  g[2] += SH_C1 * c[2];
  g[0] += -SH_C1 * c[3];
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  g[0] += SH_C2a * y * c[4];
  g[1] += SH_C2a * x * c[4];
  g[1] += -SH_C2a * z * c[5];
  g[2] += -SH_C2a * y * c[5];
  g[0] += -2.0f * SH_C2b * x * c[6];
  g[1] += -2.0f * SH_C2b * y * c[6];
  g[2] += 4.0f * SH_C2b * z * c[6];
  g[0] += -SH_C2a * z * c[7];
  g[2] += -SH_C2a * x * c[7];
  g[0] += 2.0f * SH_C2c * x * c[8];
  g[1] += -2.0f * SH_C2c * y * c[8];
  if (deg < 3) return;
  g[0] += -6.0f * SH_K0 * x * y * c[9];
  g[1] += -SH_K0 * (3.0f * xx - 3.0f * yy) * c[9];
  g[0] += SH_K1 * y * z * c[10];
  g[1] += SH_K1 * x * z * c[10];
  g[2] += SH_K1 * x * y * c[10];
  g[0] += 2.0f * SH_K2 * x * y * c[11];
  g[1] += -SH_K2 * (4.0f * zz - xx - 3.0f * yy) * c[11];
  g[2] += -8.0f * SH_K2 * y * z * c[11];
  g[0] += -6.0f * SH_K3 * x * z * c[12];
  g[1] += -6.0f * SH_K3 * y * z * c[12];
  g[2] += SH_K3 * (6.0f * zz - 3.0f * xx - 3.0f * yy) * c[12];
  g[0] += -SH_K2 * (4.0f * zz - 3.0f * xx - yy) * c[13];
  g[1] += 2.0f * SH_K2 * x * y * c[13];
  g[2] += -8.0f * SH_K2 * x * z * c[13];
  g[0] += 2.0f * SH_K5 * x * z * c[14];
  g[1] += -2.0f * SH_K5 * y * z * c[14];
  g[2] += SH_K5 * (xx - yy) * c[14];
  g[0] += -SH_K0 * (3.0f * xx - 3.0f * yy) * c[15];
  g[1] += 6.0f * SH_K0 * x * y * c[15];
}

// Everything the projection computes for one (view, Gaussian).
struct ProjState {
  float s[3], qn, qh[4], R[9], M[9], Sig[9];
  float tx, ty, tz, xi, yi;
  bool xclamp, yclamp;
  float J00, J02, J11, J12, Tm[6];
  float a, b, c, det, A, B, C;
  float u, v;
  int x0, y0, x1, y1;
};

// The projection contract: returns false if the Gaussian is culled.
__device__ __forceinline__ bool project_geometry(const float* __restrict__ P, int64_t stride, int64_t i,
                                                 const ViewDesc& V, float znear, ProjState& g) {
  float raw[11];
#pragma unroll
  for (int k = 0; k < 11; ++k) raw[k] = P[k * stride + i];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 11; ++k) ok = ok && finitef(raw[k]);
  if (!ok) return false;
  const float mx = raw[0], my = raw[1], mz = raw[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) g.s[k] = exp_cw(raw[3 + k]);
  const float qw = raw[6], qx = raw[7], qy = raw[8], qz = raw[9];
  float ss = qw * qw + qx * qx;
  ss = ss + qy * qy;
  ss = ss + qz * qz;
  if (!(ss > 0.0f) || !finitef(ss)) return false;
  g.qn = __fsqrt_rn(ss);
  const float w = __fdiv_rn(qw, g.qn), x = __fdiv_rn(qx, g.qn), y = __fdiv_rn(qy, g.qn), z = __fdiv_rn(qz, g.qn);
  g.qh[0] = w; g.qh[1] = x; g.qh[2] = y; g.qh[3] = z;
  float* R = g.R;
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
    for (int k = 0; k < 3; ++k) g.M[r * 3 + k] = R[r * 3 + k] * g.s[k];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float acc = g.M[r * 3 + 0] * g.M[k * 3 + 0] + g.M[r * 3 + 1] * g.M[k * 3 + 1];
      g.Sig[r * 3 + k] = acc + g.M[r * 3 + 2] * g.M[k * 3 + 2];
    }
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
  const float ex = __fsqrt_rn(kQMax * a);
  const float ey = __fsqrt_rn(kQMax * c);
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

// Colour of one Gaussian seen from the view (before and after max(0, .)).
__device__ __forceinline__ void project_colour(const float* __restrict__ P, int64_t stride, int64_t i, int deg,
                                               const ViewDesc& V, float* raw, float* col, float* dir,
                                               float* dnorm) {
  float Y[16];
  float dx = 0.0f, dy = 0.0f, dz = 0.0f, nrm = 1.0f;
  if (deg > 0) {
    dx = P[0 * stride + i] - V.campos[0];
    dy = P[1 * stride + i] - V.campos[1];
    dz = P[2 * stride + i] - V.campos[2];
    nrm = sqrtf(dx * dx + dy * dy + dz * dz);
    const float inv = 1.0f / nrm;
    dx *= inv; dy *= inv; dz *= inv;
  }
  dir[0] = dx; dir[1] = dy; dir[2] = dz;
  *dnorm = nrm;
  sh_basis(deg, dx, dy, dz, Y);
  const int K = (deg + 1) * (deg + 1);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = SH_C0 * P[(11 + ch) * stride + i];
    for (int k = 1; k < K; ++k) acc = acc + Y[k] * P[(11 + 3 * k + ch) * stride + i];
    raw[ch] = acc + 0.5f;
    col[ch] = fmaxf(raw[ch], 0.0f);
  }
}

__global__ void __launch_bounds__(256) project_kernel(const float* __restrict__ P, int64_t n, int64_t stride, int deg,
                                                      int num_views, const ViewDesc* __restrict__ views, int tile_w,
                                                      int tile_h, float znear, Splat* __restrict__ splats,
                                                      int4* __restrict__ rect, uint32_t* __restrict__ ntiles,
                                                      uint32_t* __restrict__ zkey, uint32_t* __restrict__ svals) {
  const int64_t total = n * (int64_t)num_views;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < total; s += (int64_t)gridDim.x * blockDim.x) {
    const int view = (int)(s / n);
    const int64_t i = s - (int64_t)view * n;
    const ViewDesc& V = views[view];
    ProjState g;
    bool vis = project_geometry(P, stride, i, V, znear, g);
    float raw[3], col[3], dir[3], dnorm;
    float o = 0.0f;
    if (vis) {
      o = 1.0f / (1.0f + exp_cw(-P[10 * stride + i]));
      project_colour(P, stride, i, deg, V, raw, col, dir, &dnorm);
      vis = finitef(col[0]) && finitef(col[1]) && finitef(col[2]);
    }
    svals[s] = (uint32_t)s;
    if (!vis) {
      Splat z;
      z.w0 = make_float4(0.f, 0.f, 0.f, 0.f);
      z.w1 = z.w0;
      z.w2 = z.w0;
      splats[s] = z;
      rect[s] = make_int4(0, 0, -1, -1);
      ntiles[s] = 0u;
      zkey[s] = 0xFFFFFFFFu;
      continue;
    }
    Splat sp;
    sp.w0 = make_float4(g.u, g.v, g.tz, o);
    sp.w1 = make_float4(g.A, g.B, g.C, 0.0f);
    sp.w2 = make_float4(col[0], col[1], col[2], 0.0f);
    splats[s] = sp;
    rect[s] = make_int4(g.x0, g.y0, g.x1, g.y1);
    const int tx0 = g.x0 / tile_w, tx1 = g.x1 / tile_w, ty0 = g.y0 / tile_h, ty1 = g.y1 / tile_h;
    ntiles[s] = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
    zkey[s] = __float_as_uint(g.tz);
  }
}

// Chain rule from the screen-space gradients (u, v, conic, opacity, colour,
// depth) of every view to the parameters, summed over views. One thread per
// Gaussian, so the parameter gradients need no atomics.
__global__ void __launch_bounds__(256) project_backward_kernel(const float* __restrict__ P, int64_t n, int64_t stride,
                                                               int deg, int num_views,
                                                               const ViewDesc* __restrict__ views, float znear,
                                                               const float* __restrict__ g2,
                                                               float* __restrict__ grad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int K = (deg + 1) * (deg + 1);
    float gmean[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
    float glogit = 0.f;
    float gsh[48];
    for (int k = 0; k < 3 * K; ++k) gsh[k] = 0.f;
    bool touched = false;
    for (int view = 0; view < num_views; ++view) {
      const float* gv = g2 + ((int64_t)view * n + i) * G2_N;
      float G[G2_N];
#pragma unroll
      for (int k = 0; k < G2_N; ++k) G[k] = gv[k];
      bool any = false;
#pragma unroll
      for (int k = 0; k < G2_N; ++k) any = any || (G[k] != 0.0f);
      if (!any) continue;
      const ViewDesc& V = views[view];
      ProjState g;
      if (!project_geometry(P, stride, i, V, znear, g)) continue;
      touched = true;
      // opacity
      const float o = 1.0f / (1.0f + exp_cw(-P[10 * stride + i]));
      glogit += G[G2_O] * o * (1.0f - o);
      // colour
      float raw[3], col[3], dir[3], dnorm;
      project_colour(P, stride, i, deg, V, raw, col, dir, &dnorm);
      float Y[16];
      sh_basis(deg, dir[0], dir[1], dir[2], Y);
      float gdir[3] = {0.f, 0.f, 0.f};
      for (int ch = 0; ch < 3; ++ch) {
        if (raw[ch] < 0.0f) continue;
        const float gc = G[G2_R + ch];
        for (int k = 0; k < K; ++k) gsh[3 * k + ch] += gc * Y[k];
        if (deg > 0) {
          float coef[16], gd[3];
          for (int k = 0; k < K; ++k) coef[k] = P[(11 + 3 * k + ch) * stride + i];
          sh_dir_grad(deg, dir[0], dir[1], dir[2], coef, gd);
          gdir[0] += gc * gd[0];
          gdir[1] += gc * gd[1];
          gdir[2] += gc * gd[2];
        }
      }
      if (deg > 0) {
        const float dot = dir[0] * gdir[0] + dir[1] * gdir[1] + dir[2] * gdir[2];
        for (int j = 0; j < 3; ++j) gmean[j] += (gdir[j] - dir[j] * dot) / dnorm;
      }
      // conic (A, B, C) = (c, -b, a) / det
      const float a = g.a, b = g.b, c = g.c, det = g.det;
      const float id = 1.0f / det, id2 = id * id;
      const float gA = G[G2_A], gB = G[G2_B], gC = G[G2_C];
      const float ga = (-gA * c * c + gB * b * c - gC * b * b) * id2;
      const float gb = (2.0f * gA * b * c - 2.0f * gB * b * b + 2.0f * gC * a * b) * id2 - gB * id;
      const float gc_ = (-gA * b * b + gB * a * b - gC * a * a) * id2;
      // Sigma' = T Sigma T^T
      const float* T0 = g.Tm;
      const float* T1 = g.Tm + 3;
      const float* S = g.Sig;
      float ST0[3], ST1[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        ST0[r] = S[r * 3 + 0] * T0[0] + S[r * 3 + 1] * T0[1] + S[r * 3 + 2] * T0[2];
        ST1[r] = S[r * 3 + 0] * T1[0] + S[r * 3 + 1] * T1[1] + S[r * 3 + 2] * T1[2];
      }
      float gT0[3], gT1[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        gT0[r] = 2.0f * ga * ST0[r] + gb * ST1[r];
        gT1[r] = gb * ST0[r] + 2.0f * gc_ * ST1[r];
      }
      // symmetric part of dL/dSigma, doubled: gS + gS^T
      float gSS[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          gSS[r * 3 + k] = 2.0f * ga * T0[r] * T0[k] + gb * (T0[r] * T1[k] + T1[r] * T0[k]) +
                           2.0f * gc_ * T1[r] * T1[k];
      const float* W = V.R;
      float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        gJ00 += gT0[k] * W[0 * 3 + k];
        gJ02 += gT0[k] * W[2 * 3 + k];
        gJ11 += gT1[k] * W[1 * 3 + k];
        gJ12 += gT1[k] * W[2 * 3 + k];
      }
      const float tx = g.tx, ty = g.ty, tz = g.tz, fx = V.fx, fy = V.fy;
      const float itz = 1.0f / tz, itz2 = itz * itz;
      float gtx = 0.f, gty = 0.f, gtz = 0.f;
      gtz += -gJ00 * fx * itz2 - gJ11 * fy * itz2 + gJ02 * fx * g.xi * itz2 + gJ12 * fy * g.yi * itz2;
      if (!g.xclamp) {
        const float gxi = -gJ02 * fx * itz;
        gtx += gxi * itz;
        gtz += -gxi * tx * itz2;
      }
      if (!g.yclamp) {
        const float gyi = -gJ12 * fy * itz;
        gty += gyi * itz;
        gtz += -gyi * ty * itz2;
      }
      gtx += G[G2_U] * fx * itz;
      gtz += -G[G2_U] * fx * tx * itz2;
      gty += G[G2_V] * fy * itz;
      gtz += -G[G2_V] * fy * ty * itz2;
      gtz += G[G2_Z];
#pragma unroll
      for (int j = 0; j < 3; ++j) gmean[j] += W[0 * 3 + j] * gtx + W[1 * 3 + j] * gty + W[2 * 3 + j] * gtz;
      // Sigma = M M^T, M = R diag(s)
      float gM[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          gM[r * 3 + k] = gSS[r * 3 + 0] * g.M[0 * 3 + k] + gSS[r * 3 + 1] * g.M[1 * 3 + k] +
                          gSS[r * 3 + 2] * g.M[2 * 3 + k];
      float gR[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) gR[r * 3 + k] = gM[r * 3 + k] * g.s[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float gs = gM[0 * 3 + k] * g.R[0 * 3 + k] + gM[1 * 3 + k] * g.R[1 * 3 + k] + gM[2 * 3 + k] * g.R[2 * 3 + k];
        gls[k] += gs * g.s[k];
      }
      const float w = g.qh[0], x = g.qh[1], y = g.qh[2], z = g.qh[3];
      const float gw = 2.0f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
      const float gx = 2.0f * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0f * x * gR[4] - w * gR[5] + z * gR[6] +
                               w * gR[7] - 2.0f * x * gR[8]);
      const float gy = 2.0f * (-2.0f * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] +
                               z * gR[7] - 2.0f * y * gR[8]);
      const float gz = 2.0f * (-2.0f * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0f * z * gR[4] +
                               y * gR[5] + x * gR[6] + y * gR[7]);
      const float dot = w * gw + x * gx + y * gy + z * gz;
      const float iqn = 1.0f / g.qn;
      gq[0] += (gw - w * dot) * iqn;
      gq[1] += (gx - x * dot) * iqn;
      gq[2] += (gy - y * dot) * iqn;
      gq[3] += (gz - z * dot) * iqn;
    }
    if (!touched) continue;
#pragma unroll
    for (int j = 0; j < 3; ++j) grad[(0 + j) * stride + i] += gmean[j];
#pragma unroll
    for (int j = 0; j < 3; ++j) grad[(3 + j) * stride + i] += gls[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) grad[(6 + j) * stride + i] += gq[j];
    grad[10 * stride + i] += glogit;
    for (int k = 0; k < 3 * K; ++k) grad[(11 + k) * stride + i] += gsh[k];
  }
}

// Inspection copy of one view's splats; the screen covariance (a, b, c) is
// not kept by the forward, so it is recomputed here by the same projection.
__global__ void export_splats_kernel(const float* __restrict__ P, int64_t n, int64_t stride,
                                     const ViewDesc* __restrict__ view, float znear, const Splat* __restrict__ splats,
                                     const int4* __restrict__ rect, float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const Splat s = splats[i];
    const int4 r = rect[i];
    float* o = out + i * 16;
    const bool vis = r.z >= r.x;
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

int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

}  // namespace

void launch_project(const float* params, int64_t n, int64_t stride, int deg, int num_views, const ViewDesc* views,
                    int tile_w, int tile_h, float znear, Splat* splats, int4* rect, uint32_t* ntiles,
                    uint32_t* zkey, uint32_t* svals, hipStream_t st) {
  const int64_t total = n * num_views;
  if (total == 0) return;
  project_kernel<<<grid_for(total, 256), 256, 0, st>>>(params, n, stride, deg, num_views, views, tile_w, tile_h,
                                                       znear, splats, rect, ntiles, zkey, svals);
}

void launch_project_backward(const float* params, int64_t n, int64_t stride, int deg, int num_views,
                             const ViewDesc* views, float znear, const float* g2, float* grad, hipStream_t st) {
  if (n == 0) return;
  project_backward_kernel<<<grid_for(n, 256), 256, 0, st>>>(params, n, stride, deg, num_views, views, znear, g2,
                                                            grad);
}

void launch_export_splats(const float* params, int64_t n, int64_t stride, const ViewDesc* view, float znear,
                          const Splat* splats, const int4* rect, float* out, hipStream_t st) {
  if (n == 0) return;
  export_splats_kernel<<<grid_for(n, 256), 256, 0, st>>>(params, n, stride, view, znear, splats, rect, out);
}

}  // namespace gsr
