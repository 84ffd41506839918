// Driver for a sanitizer build of the oracle (AddressSanitizer and
// UndefinedBehaviorSanitizer, host code only). Test infrastructure: it calls
// every entry point of oracle.cpp on small seeded scenes -- each render mode,
// windows, the tile list, the projection, the backward in each mode with
// every optional output -- including Gaussians the projection must cull
// (non-finite values, a zero quaternion, behind the camera, a huge one), so
// that an out-of-bounds access or undefined operation anywhere in the
// oracle's own code stops the run with a report. Exit status 0 = clean.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <vector>

extern "C" {
int orc_num_threads(int n);
void orc_exp32(const float* x, float* y, double* tie, int64_t n);
void orc_activations(const float* logscale, const float* logit, float* scale, float* opacity, int64_t n);
void orc_sh_basis(int deg, const double* dirs, int64_t n, double* out, double* grad);
int orc_project(int prec, const float* params, int64_t n, int64_t stride, int deg, const float* cam, int width,
                int height, float znear, double* out, int32_t* rect);
int orc_tile_list(const float* params, int64_t n, int64_t stride, int deg, int num_views, const float* cams,
                  const int32_t* wh, int tile_w, int tile_h, float znear, int64_t capacity, uint32_t* out_tile,
                  uint32_t* out_gid, int64_t* count);
int orc_render(int mode, int prefilter, const float* params, int64_t n, int64_t stride, int deg, const float* cam,
               int width, int height, float znear, const float* bg, double* rgb, double* depth, double* alpha,
               double* tfinal, int32_t* ncomp, double* margin, const int32_t* window);
int orc_backward(int pinned, const float* params, int64_t n, int64_t stride, int deg, int num_views,
                 const float* cams, const int32_t* wh, float znear, const float* bg, const float* grgb,
                 const float* gdepth, const float* galpha, double* grad, double* g2, const int32_t* windows,
                 double* gcam, double* gabs);
}

namespace {

// xorshift64*: seeded uniform numbers for the inputs (no part of the method)
struct Rng {
  uint64_t s;
  double uniform() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return (double)((s * 2685821657736338717ull) >> 11) * 0x1p-53;
  }
  double range(double a, double b) { return a + (b - a) * uniform(); }
};

int failures = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

// [P][stride] parameters of n Gaussians (stride > n: padded planes), the
// last five of them degenerate or culled on purpose.
std::vector<float> scene(Rng& r, int n, int64_t stride, int deg, float focal, int W, int H) {
  const int P = 11 + 3 * (deg + 1) * (deg + 1);
  std::vector<float> p((size_t)P * stride, 0.0f);
  for (int i = 0; i < n; ++i) {
    const double z = r.range(1.0, 4.0);
    p[0 * stride + i] = (float)((r.range(-0.1, 1.1) * W - W / 2.0) / focal * z);
    p[1 * stride + i] = (float)((r.range(-0.1, 1.1) * H - H / 2.0) / focal * z);
    p[2 * stride + i] = (float)z;
    for (int k = 3; k < 6; ++k) p[k * stride + i] = (float)r.range(-3.5, -1.5);
    for (int k = 6; k < 10; ++k) p[k * stride + i] = (float)r.range(-1.0, 1.0);
    p[10 * stride + i] = (float)r.range(-2.0, 3.0);
    for (int k = 11; k < P; ++k) p[k * stride + i] = (float)r.range(-0.5, 0.5);
  }
  const float nan = std::numeric_limits<float>::quiet_NaN(), inf = std::numeric_limits<float>::infinity();
  p[0 * stride + (n - 1)] = nan;                                           // non-finite mean
  p[4 * stride + (n - 2)] = inf;                                           // infinite log-scale
  for (int k = 6; k < 10; ++k) p[k * stride + (n - 3)] = 0.0f;             // zero quaternion
  p[2 * stride + (n - 4)] = -2.0f;                                         // behind the camera
  for (int k = 3; k < 6; ++k) p[k * stride + (n - 5)] = 1.5f;              // larger than the view
  return p;
}

std::vector<float> camera(float focal, int W, int H, double yaw) {
  std::vector<float> c(16, 0.0f);
  const double cy = std::cos(yaw), sy = std::sin(yaw);
  const double R[9] = {cy, 0, sy, 0, 1, 0, -sy, 0, cy};
  for (int k = 0; k < 9; ++k) c[k] = (float)R[k];
  c[9] = 0.05f;
  c[10] = -0.02f;
  c[11] = 0.1f;
  c[12] = focal;
  c[13] = focal * 1.1f;
  c[14] = W / 2.0f;
  c[15] = H / 2.0f;
  return c;
}

void run_case(Rng& r, int deg, int n, int64_t stride, int nv) {
  const int P = 11 + 3 * (deg + 1) * (deg + 1);
  const float focal = 30.0f;
  const int Ws[2] = {37, 29}, Hs[2] = {29, 18};
  std::vector<float> p = scene(r, n, stride, deg, focal, Ws[0], Hs[0]);
  std::vector<float> cams;
  std::vector<int32_t> wh;
  for (int v = 0; v < nv; ++v) {
    std::vector<float> c = camera(focal, Ws[v], Hs[v], 0.1 * v);
    cams.insert(cams.end(), c.begin(), c.end());
    wh.push_back(Ws[v]);
    wh.push_back(Hs[v]);
  }
  const float bg[3] = {0.1f, 0.2f, 0.3f};
  const float znear = 0.2f;

  // projection, both precisions
  for (int prec : {32, 64}) {
    std::vector<double> out((size_t)n * 17);
    std::vector<int32_t> rect((size_t)n * 4);
    expect(orc_project(prec, p.data(), n, stride, deg, cams.data(), Ws[0], Hs[0], znear, out.data(),
                       rect.data()) == 0, "project");
    expect(out[(size_t)(n - 1) * 17 + 16] == 0.0 && out[(size_t)(n - 3) * 17 + 16] == 0.0 &&
           out[(size_t)(n - 4) * 17 + 16] == 0.0, "degenerate Gaussians culled");
  }
  expect(orc_project(7, p.data(), n, stride, deg, cams.data(), Ws[0], Hs[0], znear, nullptr, nullptr) == -1,
         "bad precision rejected");

  // tile list: count, then fill, in every tile size
  for (int ts : {8, 16, 32}) {
    int64_t count = 0;
    orc_tile_list(p.data(), n, stride, deg, nv, cams.data(), wh.data(), ts, ts, znear, 0, nullptr, nullptr, &count);
    std::vector<uint32_t> t((size_t)count + 1), g((size_t)count + 1);
    int64_t count2 = 0;
    orc_tile_list(p.data(), n, stride, deg, nv, cams.data(), wh.data(), ts, ts, znear, count, t.data(), g.data(),
                  &count2);
    expect(count2 == count, "tile list count");
  }

  // renders: every mode, with and without the prefilter, whole and windowed
  const int W = Ws[0], H = Hs[0];
  const size_t HW = (size_t)W * H;
  const int32_t window[5] = {3, 2, W - 4, H - 1, 3};
  for (int mode = 0; mode < 3; ++mode)
    for (int pre = 0; pre < 2; ++pre)
      for (int win = 0; win < 2; ++win) {
        std::vector<double> rgb(3 * HW), dep(HW), alp(HW), tf(HW), mg(HW);
        std::vector<int32_t> nc(HW);
        expect(orc_render(mode, pre, p.data(), n, stride, deg, cams.data(), W, H, znear, bg, rgb.data(), dep.data(),
                          alp.data(), tf.data(), nc.data(), mg.data(), win ? window : nullptr) == 0, "render");
        for (size_t k = 0; k < HW; ++k)
          if (!(alp[k] >= 0.0 && alp[k] <= 1.0) || !std::isfinite(rgb[k])) {
            expect(false, "render values finite and alpha in [0, 1]");
            break;
          }
      }
  expect(orc_render(5, 0, p.data(), n, stride, deg, cams.data(), W, H, znear, bg, nullptr, nullptr, nullptr, nullptr,
                    nullptr, nullptr, nullptr) == -1, "bad mode rejected");

  // backward: every mode, every optional output, whole views and windows
  size_t tot = 0;
  for (int v = 0; v < nv; ++v) tot += (size_t)Ws[v] * Hs[v];
  std::vector<float> grgb(3 * tot), gdep(tot), galp(tot);
  {
    size_t off = 0;
    for (int v = 0; v < nv; ++v) {
      const size_t hw = (size_t)Ws[v] * Hs[v];
      for (size_t k = 0; k < 3 * hw; ++k) grgb[3 * off + k] = (float)r.range(-1.0, 1.0);
      for (size_t k = 0; k < hw; ++k) {
        gdep[off + k] = (float)r.range(-0.1, 0.1);
        galp[off + k] = (float)r.range(-1.0, 1.0);
      }
      off += hw;
    }
  }
  std::vector<int32_t> wins;
  for (int v = 0; v < nv; ++v) {
    const int32_t w[5] = {1, 1, Ws[v] - 2, Hs[v] - 1, 2};
    wins.insert(wins.end(), w, w + 5);
  }
  for (int pinned = 0; pinned < 3; ++pinned)
    for (int extra = 0; extra < 2; ++extra) {
      std::vector<double> grad((size_t)P * n, -1.0), g2((size_t)nv * n * 10), gcam((size_t)nv * 12),
          gabs((size_t)P * n);
      expect(orc_backward(pinned, p.data(), n, stride, deg, nv, cams.data(), wh.data(), znear, bg, grgb.data(),
                          gdep.data(), galp.data(), grad.data(), extra ? g2.data() : nullptr,
                          extra ? wins.data() : nullptr, extra ? gcam.data() : nullptr,
                          extra ? gabs.data() : nullptr) == 0, "backward");
      for (int q = 0; q < P; ++q)
        for (int i = n - 5; i < n - 1; ++i)
          if (i != n - 5 && grad[(size_t)q * n + i] != 0.0) expect(false, "culled Gaussians get zero gradient");
      // up to rounding: an element whose exact gradient is zero (a rotation
      // of an isotropic Gaussian) can carry a residue of order 1e-16
      double amax = 0.0;
      for (double a : gabs) amax = std::fmax(amax, a);
      if (extra)
        for (size_t k = 0; k < grad.size(); ++k)
          if (!(std::fabs(grad[k]) <= gabs[k] * (1.0 + 1e-12) + 1e-12 * amax)) {
            expect(false, "summand magnitudes bound the gradient");
            break;
          }
    }
}

}  // namespace

int main() {
  Rng r{0x9e3779b97f4a7c15ull};
  orc_num_threads(2);
  // exponential and activations over a range with overflow and underflow
  {
    const int64_t m = 4096;
    std::vector<float> x(m), y(m), s(m), o(m);
    std::vector<double> tie(m);
    for (int64_t k = 0; k < m; ++k) x[k] = (float)(-120.0 + 240.0 * (double)k / (double)(m - 1));
    x[0] = std::numeric_limits<float>::quiet_NaN();
    orc_exp32(x.data(), y.data(), tie.data(), m);
    orc_exp32(x.data(), y.data(), nullptr, m);
    orc_activations(x.data(), x.data(), s.data(), o.data(), m);
    expect(std::isinf(y[m - 1]) && y[1] == 0.0f, "exp overflow and underflow");
  }
  for (int deg = 0; deg <= 3; ++deg) {
    const int K = (deg + 1) * (deg + 1);
    std::vector<double> dirs(3 * 50), out(50 * K), grad(50 * K * 3);
    for (int k = 0; k < 50; ++k) {
      double a = r.range(-1, 1), b = r.range(-1, 1), c = r.range(-1, 1);
      const double nn = std::sqrt(a * a + b * b + c * c) + 1e-12;
      dirs[3 * k] = a / nn;
      dirs[3 * k + 1] = b / nn;
      dirs[3 * k + 2] = c / nn;
    }
    orc_sh_basis(deg, dirs.data(), 50, out.data(), grad.data());
    orc_sh_basis(deg, dirs.data(), 50, out.data(), nullptr);
  }
  run_case(r, 0, 40, 40, 1);
  run_case(r, 3, 40, 45, 2);
  run_case(r, 1, 6, 9, 1);
  std::printf("%s\n", failures ? "FAILED" : "clean");
  return failures ? 1 : 0;
}
