// Front-to-back alpha compositing of the sorted tile lists, its backward,
// the L1 mapping loss and Adam.
//
// One workgroup per screen tile, one thread per pixel (wave64 = 4 rows of a
// 16-wide tile). The tile's instance list is staged through LDS in batches;
// every lane reads the same LDS record, so the reads are broadcasts. A pixel
// stops when compositing the next Gaussian would take its transmittance below
// 1e-4 (that Gaussian is not composited); alpha is clamped to 0.99 and
// alphas below 1/255 are skipped. The workgroup leaves the tile as soon as
// every pixel has stopped.
//
// The backward walks each pixel's list in reverse from the last composited
// Gaussian, recovering T_k = T_{k+1} / (1 - alpha_k) from the stored final
// transmittance instead of storing per-Gaussian blend state, and keeps the
// suffix sum S_k of later contributions. Per-pair screen-space gradients are
// summed as ten moments per Gaussian over each 16-lane row with DPP, over the
// workgroup in LDS, and only then added with one global atomic per (tile
// batch, Gaussian, component).
//
// Compiled with -ffp-contract=off. The exponent of a pair is formed with the
// float roundings of its plain definition, -(A dx^2 + C dy^2)/2 - B dx dy
// summed as ((A dx) dx + (C dy) dy) and (B dx) dy, so it is the same float as
// a plain float evaluation of the formula; the forward and backward recompute
// it bit-identically. For thin Gaussians the terms cancel and any other
// association of the sum would differ from it by much more than an ulp.

#include "gsr_internal.h"

namespace gsr {
namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr uint32_t kWaitLimit = 1u << 22;   // bounded wait of a fused backward unit

// Blend-ready record of one Gaussian in LDS: q0 = (u, v, -A/2, -B),
// q1 = (-C/2, opacity, z, 0), q2 = (r, g, b, 0). Halving and negating are
// exact, so ((-A/2 dx) dx + (-C/2 dy) dy) + (-B dx) dy rounds exactly like
// -((A dx) dx + (C dy) dy)/2 - (B dx) dy.
__device__ __forceinline__ void stage_record(const float4& w0, const float4& w1, const float4& w2, float4& q0,
                                             float4& q1, float4& q2) {
  q0 = make_float4(w0.x, w0.y, -0.5f * w1.x, -w1.y);
  q1 = make_float4(-0.5f * w1.z, w0.w, w0.z, 0.0f);
  q2 = make_float4(w2.x, w2.y, w2.z, 0.0f);
}

// Alpha of one pair. Returns false when the pair is skipped (exponent
// positive or alpha below 1/255). G = exp(power), clamped = alpha hit 0.99.
__device__ __forceinline__ bool pair_alpha(const float4& q0, const float4& q1, float xs, float ys, float& dx,
                                           float& dy, float& G, float& alpha, bool& clamped) {
  dx = q0.x - xs;
  dy = q0.y - ys;
  const float power = ((q0.z * dx) * dx + (q1.x * dy) * dy) + (q0.w * dx) * dy;
  G = __builtin_amdgcn_exp2f(power * kLog2e);
  const float araw = q1.y * G;
  clamped = araw > kAlphaMax;
  alpha = clamped ? kAlphaMax : araw;
  return (power <= 0.0f) && (alpha >= kAlphaMin);
}

__device__ __forceinline__ int find_view(const ViewDesc* views, int num_views, int tile) {
  int v = 0;
  while (v + 1 < num_views && tile >= views[v + 1].tile_offset) ++v;
  return v;
}

// Pixels per thread: a thread owns PPT pixels of one tile column, TH/PPT rows
// apart, so every LDS record it reads serves PPT pairs and the backward's
// wave reduction covers 64 * PPT pixels. The Gaussian loop is unrolled by
// two: the alphas of consecutive Gaussians are independent, only the
// transmittance update is sequential, which gives each wave independent work
// to overlap with LDS and transcendental latency.
template <int TW, int TH, int PPT>
struct TileShape {
  static constexpr int NT = TW * TH / PPT;       // threads per workgroup
  static constexpr int ROWS = TH / PPT;          // row stride between a thread's pixels
  static_assert(NT % 64 == 0, "workgroup must be whole wavefronts");
};

// Front-to-back update of one pixel with one Gaussian whose alpha is known.
// Branchy on purpose: most pairs are skipped (alpha below 1/255), and a wave
// whose lanes all skip jumps over the update.
// CK: the sums of the current backward chunk (dC) are kept as well.
template <bool CK>
__device__ __forceinline__ void composite_one(bool ok, float alpha, const float4& q1, const float4& q2, float& T,
                                              float& C0, float& C1, float& C2, float& D, float* dC, bool& done,
                                              uint32_t& last, uint32_t pos) {
  if (done || !ok) return;
  const float Tn = T * (1.0f - alpha);
  if (Tn < kTransMin) {
    done = true;
    return;
  }
  const float w = alpha * T;
  C0 = fmaf(w, q2.x, C0);
  C1 = fmaf(w, q2.y, C1);
  C2 = fmaf(w, q2.z, C2);
  D = fmaf(w, q1.z, D);
  if (CK) {
    dC[0] = fmaf(w, q2.x, dC[0]);
    dC[1] = fmaf(w, q2.y, dC[1]);
    dC[2] = fmaf(w, q2.z, dC[2]);
    dC[3] = fmaf(w, q1.z, dC[3]);
  }
  T = Tn;
  last = pos;
}

// Stores of the per-pixel state the backward reads. In the fused launch the
// backward of a tile runs in the same grid as its forward, on any XCD: the
// state is then written with device-coherent stores.
template <bool X>
__device__ __forceinline__ void st_f32(float* p, float v) {
  if (X) __hip_atomic_store(reinterpret_cast<uint32_t*>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}
template <bool X>
__device__ __forceinline__ void st_u32(uint32_t* p, uint32_t v) {
  if (X) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}
template <bool X>
__device__ __forceinline__ float ld_f32(const float* p) {
  if (X) return __uint_as_float(__hip_atomic_load(reinterpret_cast<const uint32_t*>(p), __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT));
  return *p;
}
template <bool X>
__device__ __forceinline__ uint32_t ld_u32(const uint32_t* p) {
  if (X) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return *p;
}

// Chunked backward state of one pixel: slot s holds (T before chunk s,
// colour and depth composited within chunk s).
template <bool X>
__device__ __forceinline__ void write_ckpt_T(const BlendArgs& a, uint32_t slot, int64_t pix, float T) {
  st_f32<X>(a.ckpt + (int64_t)slot * kCkptFields * a.ckpt_stride + pix, T);
}
template <bool X>
__device__ __forceinline__ void write_ckpt_sums(const BlendArgs& a, uint32_t slot, int64_t pix, const float* dC) {
  const int64_t st = a.ckpt_stride;
  float* c = a.ckpt + (int64_t)slot * kCkptFields * st + pix;
#pragma unroll
  for (int f = 0; f < 4; ++f) st_f32<X>(c + (f + 1) * st, dC[f]);
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, m, 64));
  return x;
}

// At list position `pos` = s * chunk_len (s >= 1): every pixel still
// compositing records T into slot s and the sums of chunk s - 1 into slot
// s - 1, and starts chunk s. A stopped pixel's last composited position lies
// before pos, so the backward never reads these slots for it.
template <int PPT, bool X>
__device__ __forceinline__ void chunk_boundary(const BlendArgs& a, uint32_t& pos, uint32_t end, const bool* done,
                                               const int64_t* pix, const float* T, float (*dC)[4], uint32_t* mych) {
  const uint32_t s = pos / (uint32_t)a.chunk_len;
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    if (done[i]) continue;
    write_ckpt_T<X>(a, s, pix[i], T[i]);
    write_ckpt_sums<X>(a, s - 1, pix[i], dC[i]);
    dC[i][0] = dC[i][1] = dC[i][2] = dC[i][3] = 0.0f;
    mych[i] = s;
  }
  pos += (uint32_t)a.chunk_len;
  if (pos >= end) pos = 0xFFFFFFFFu;
}

// LDS of the forward: one batch of blend-ready records per thread.
template <int NT>
struct FwdShared {
  float4 q0[NT], q1[NT], q2[NT];
  uint32_t tl;
  float loss[NT / 64];
};

// Forward of one tile. CK: record the chunked backward's per-pixel state
// (a.chunk_len > 0). X: the backward runs in the same launch (the state is
// written device-coherently and the tile is marked done at the end).
// Returns the tile's largest last position (every thread).
template <int TW, int TH, int PPT, bool CK, bool X>
__device__ __forceinline__ uint32_t forward_tile(const BlendArgs& a, FwdShared<TW * TH / PPT>& sh, int tile) {
  using Shape = TileShape<TW, TH, PPT>;
  constexpr int NT = Shape::NT;
  constexpr int ROWS = Shape::ROWS;
  constexpr int BATCH = NT;
  float4* s_q0 = sh.q0;
  float4* s_q1 = sh.q1;
  float4* s_q2 = sh.q2;
  uint32_t& s_tl = sh.tl;
  float* s_loss = sh.loss;
  const int view = find_view(a.views, a.num_views, tile);
  const ViewDesc& V = a.views[view];
  const int lt = tile - V.tile_offset;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int tid = threadIdx.x;
  const int px = tx * TW + (tid % TW);
  int py[PPT];
  bool inside[PPT], done[PPT];
  float ys[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT];
  float dC[PPT][4];
  uint32_t last[PPT], mych[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    py[i] = ty * TH + (tid / TW) + i * ROWS;
    inside[i] = px < V.width && py[i] < V.height;
    done[i] = !inside[i];
    ys[i] = (float)py[i] + 0.5f;
    T[i] = 1.0f;
    C0[i] = C1[i] = C2[i] = D[i] = 0.0f;
    dC[i][0] = dC[i][1] = dC[i][2] = dC[i][3] = 0.0f;
    last[i] = 0;
    mych[i] = 0;
  }
  const float xs = (float)px + 0.5f;
  const uint2 rg = a.ranges[tile];
  int64_t pix[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) pix[i] = V.pix_offset + (int64_t)py[i] * V.width + px;
  // next list position whose state the chunked backward starts from
  const uint32_t ck_end = CK ? (uint32_t)a.chunk_len * (uint32_t)a.max_chunks : 0u;
  uint32_t nextck = CK && a.max_chunks > 1 ? (uint32_t)a.chunk_len : 0xFFFFFFFFu;
  if (tid == 0) s_tl = 0;
  __syncthreads();
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += BATCH) {
    bool all_done = true;
#pragma unroll
    for (int i = 0; i < PPT; ++i) all_done = all_done && done[i];
    if (__syncthreads_count(all_done) == NT) break;
    const uint32_t j = b0 + tid;
    if (j < rg.y) {
      const Splat* sp = a.splats + a.inst_vals[j];
      stage_record(sp->w0, sp->w1, sp->w2, s_q0[tid], s_q1[tid], s_q2[tid]);
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)BATCH, rg.y - b0);
    const uint32_t pos0 = b0 - rg.x + 1;
    int k = 0;
    for (; k + 1 < cnt; k += 2) {
      // the wave leaves the batch when all its pixels have stopped; the exit
      // is wave-uniform so that the loop state stays in scalar registers
      bool busy = false;
#pragma unroll
      for (int i = 0; i < PPT; ++i) busy = busy || !done[i];
      if (__ballot(busy) == 0ull) break;
      if (CK && b0 - rg.x + k == nextck) {
        chunk_boundary<PPT, X>(a, nextck, ck_end, done, pix, T, dC, mych);
      }
      const float4 qa0 = s_q0[k], qa1 = s_q1[k], qb0 = s_q0[k + 1], qb1 = s_q1[k + 1];
      float al_a[PPT], al_b[PPT];
      bool ok_a[PPT], ok_b[PPT];
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        float dx, dy, G;
        bool cl;
        ok_a[i] = pair_alpha(qa0, qa1, xs, ys[i], dx, dy, G, al_a[i], cl);
        ok_b[i] = pair_alpha(qb0, qb1, xs, ys[i], dx, dy, G, al_b[i], cl);
        // both alphas are formed before the first per-lane branch, so that
        // the two exponentials' latencies overlap (without this the compiler
        // sinks the second one past the first Gaussian's update)
        __asm__ volatile("" ::"v"(al_a[i]), "v"(al_b[i]));
      }
      const float4 qa2 = s_q2[k], qb2 = s_q2[k + 1];
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        composite_one<CK>(ok_a[i], al_a[i], qa1, qa2, T[i], C0[i], C1[i], C2[i], D[i], dC[i], done[i], last[i],
                          pos0 + k);
        composite_one<CK>(ok_b[i], al_b[i], qb1, qb2, T[i], C0[i], C1[i], C2[i], D[i], dC[i], done[i], last[i],
                          pos0 + k + 1);
      }
    }
    if (k < cnt) {
      if (CK && b0 - rg.x + k == nextck) {
        chunk_boundary<PPT, X>(a, nextck, ck_end, done, pix, T, dC, mych);
      }
      const float4 q0 = s_q0[k], q1 = s_q1[k], q2 = s_q2[k];
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        float dx, dy, G, al;
        bool cl;
        const bool ok = pair_alpha(q0, q1, xs, ys[i], dx, dy, G, al, cl);
        composite_one<CK>(ok, al, q1, q2, T[i], C0[i], C1[i], C2[i], D[i], dC[i], done[i], last[i], pos0 + k);
      }
    }
  }
  const ViewImages im = a.images[view];
  const int64_t HW = (int64_t)V.width * V.height;
  uint32_t tl = 0;
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    if (!inside[i]) continue;
    const int64_t p = (int64_t)py[i] * V.width + px;
    im.rgb[p] = fmaf(T[i], a.bg[0], C0[i]);
    im.rgb[HW + p] = fmaf(T[i], a.bg[1], C1[i]);
    im.rgb[2 * HW + p] = fmaf(T[i], a.bg[2], C2[i]);
    im.depth[p] = D[i];
    im.alpha[p] = 1.0f - T[i];
    st_f32<X>(a.tfinal + pix[i], T[i]);
    st_u32<X>(a.last + pix[i], last[i]);
    tl = max(tl, last[i]);
    // the sums of the chunk the pixel ended in; read only when an earlier
    // chunk's walk starts past its own end, i.e. last > chunk_len
    if (CK && last[i] > (uint32_t)a.chunk_len) write_ckpt_sums<X>(a, mych[i], pix[i], dC[i]);
  }
  tl = wave_max_u32(tl);
  if ((tid & 63) == 0) atomicMax(&s_tl, tl);
  if (a.loss_target) {
    // the L1 mapping loss of the composited pixels, with the same float
    // operations as loss_l1_kernel, so the image gradients are identical
    const ViewImages tg = a.loss_target[view], gr = a.loss_grad[view];
    const float inv3 = 1.0f / (3.0f * (float)HW), inv1 = a.depth_weight / (float)HW;
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      if (!inside[i]) continue;
      const int64_t p = (int64_t)py[i] * V.width + px;
      const float out[3] = {fmaf(T[i], a.bg[0], C0[i]), fmaf(T[i], a.bg[1], C1[i]), fmaf(T[i], a.bg[2], C2[i])};
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float d = out[ch] - tg.rgb[ch * HW + p];
        st_f32<X>(gr.rgb + ch * HW + p, d > 0.0f ? inv3 : (d < 0.0f ? -inv3 : 0.0f));
        acc += fabsf(d) * inv3;
      }
      const float dd = D[i] - tg.depth[p];
      st_f32<X>(gr.depth + p, dd > 0.0f ? inv1 : (dd < 0.0f ? -inv1 : 0.0f));
      acc += fabsf(dd) * inv1;
      if (gr.alpha) st_f32<X>(gr.alpha + p, 0.0f);
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) s_loss[tid >> 6] = acc;
  }
  // fused: every wave's stores complete before the barrier, so that the
  // release below covers the whole workgroup's writes
  if (X) __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (tid == 0) {
    st_u32<X>(a.tile_last + tile, s_tl);
    if (a.loss_target && a.loss) {
      float sum = 0.0f;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) sum += s_loss[w];
      unsafeAtomicAdd(a.loss, sum);
    }
    if (X) __hip_atomic_store(a.tile_done + tile, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  return s_tl;
}

template <int TW, int TH, int PPT, bool CK>
__global__ void __launch_bounds__(TW * TH / PPT) blend_forward_kernel(BlendArgs a) {
  __shared__ FwdShared<TW * TH / PPT> sh;
  forward_tile<TW, TH, PPT, CK, false>(a, sh, a.order ? (int)a.order[blockIdx.x] : (int)blockIdx.x);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float x) {
  const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, false);
  return x + __int_as_float(y);
}

// Sum over the 64 lanes of a wavefront with DPP moves only (no LDS traffic):
// pairs and quads by quad permutes, the 16-lane rows by two rotations, then
// row 0 + row 1 and row 2 + row 3 by a broadcast of lane 15 of the row above,
// and rows 0-1 into rows 2-3 by a broadcast of lane 31. The total ends in
// lane 63; other lanes hold partial sums.
__device__ __forceinline__ float wave_sum_lane63(float x) {
  x = dpp_add<0xB1, 0xF>(x);    // quad_perm [1,0,3,2]
  x = dpp_add<0x4E, 0xF>(x);    // quad_perm [2,3,0,1]
  x = dpp_add<0x124, 0xF>(x);   // row_ror:4
  x = dpp_add<0x128, 0xF>(x);   // row_ror:8
  x = dpp_add<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
  x = dpp_add<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
  return x;
}

// Per-(wave, Gaussian) sums the backward reduces. The conic and mean
// gradients are linear in the moments of dL/dpower over the pixels, so the
// per-pair work accumulates the moments and the lane that publishes the
// wave sum turns them into (u, v, A, B, C) gradients.
enum { M_R = 0, M_G, M_B, M_Z, M_O, M_X, M_XX, M_Y, M_XY, M_YY, M_N };

// Reverse step of one pixel over one Gaussian, without branches: recover
// T_k, form the pair's moments, update the suffix sum. A pair that was not
// composited (ok false) leaves T and S alone and contributes zero moments;
// a clamped alpha passes no gradient to opacity or the exponent. FIRST: the
// moments are assigned (the thread's first pixel) rather than accumulated.
// ROWY: every 16-lane row of the wave is one image row (one pixel per
// thread, tiles 16 or 32 wide), so dy is the same across the row; and
// dL/dpower = opacity x dL/dopacity-term (alpha = o G unclamped): the lane
// keeps the dx and dx^2 moments of dL/dopacity's term (in M_X, M_XX); the
// workgroup's sums apply the rows' dy and the opacity.
template <bool FIRST, bool ROWY>
__device__ __forceinline__ void reverse_one(bool ok, float alpha, float G, bool clamped, float dx, float dy,
                                            const float4& q1, const float4& q2, float gc0, float gc1, float gc2,
                                            float gd, float tb, float& T, float& S, float* m) {
  const float r1m = __builtin_amdgcn_rcpf(1.0f - alpha);
  const float Tk = T * r1m;                              // T_k, transmittance before k
  const float x = fmaf(gc0, q2.x, fmaf(gc1, q2.y, fmaf(gc2, q2.z, gd * q1.z)));
  const float galpha = fmaf(Tk, x - S, tb * r1m);
  const float Sn = fmaf(alpha, x, (1.0f - alpha) * S);
  const float w = ok ? alpha * Tk : 0.0f;
  const bool live = ok && !clamped;
  const float go = live ? galpha * G : 0.0f;
  const float gpow = live ? galpha * alpha : 0.0f;     // dL/dpower
  T = ok ? Tk : T;
  S = ok ? Sn : S;
  if (ROWY) {
    const float gx = go * dx;
    m[M_R] = w * gc0;
    m[M_G] = w * gc1;
    m[M_B] = w * gc2;
    m[M_Z] = w * gd;
    m[M_O] = go;
    m[M_X] = gx;
    m[M_XX] = gx * dx;
    return;
  }
  const float gx = gpow * dx, gy = gpow * dy;
  if (FIRST) {
    m[M_R] = w * gc0;
    m[M_G] = w * gc1;
    m[M_B] = w * gc2;
    m[M_Z] = w * gd;
    m[M_O] = go;
    m[M_X] = gx;
    m[M_Y] = gy;
    m[M_XX] = gx * dx;
    m[M_XY] = gx * dy;
    m[M_YY] = gy * dy;
  } else {
    m[M_R] = fmaf(w, gc0, m[M_R]);
    m[M_G] = fmaf(w, gc1, m[M_G]);
    m[M_B] = fmaf(w, gc2, m[M_B]);
    m[M_Z] = fmaf(w, gd, m[M_Z]);
    m[M_O] += go;
    m[M_X] += gx;
    m[M_Y] += gy;
    m[M_XX] = fmaf(gx, dx, m[M_XX]);
    m[M_XY] = fmaf(gx, dy, m[M_XY]);
    m[M_YY] = fmaf(gy, dy, m[M_YY]);
  }
}

// Sum over each 16-lane row of a wavefront with fused DPP adds (quad
// permutes, then row rotations by 4 and 8): every lane ends with its row's
// total. Step-major over the M_N moments so that the independent chains fill
// the DPP read-after-write wait states.
template <int N>
__device__ __forceinline__ void row_sums(float* m) {
#pragma unroll
  for (int c = 0; c < N; ++c) m[c] = dpp_add<0xB1, 0xF>(m[c]);   // quad_perm [1,0,3,2]
#pragma unroll
  for (int c = 0; c < N; ++c) m[c] = dpp_add<0x4E, 0xF>(m[c]);   // quad_perm [2,3,0,1]
#pragma unroll
  for (int c = 0; c < N; ++c) m[c] = dpp_add<0x124, 0xF>(m[c]);  // row_ror:4
#pragma unroll
  for (int c = 0; c < N; ++c) m[c] = dpp_add<0x128, 0xF>(m[c]);  // row_ror:8
}

// The row form of the backward (ROWY in reverse_one): every 16-lane row of
// a wavefront is one image row. Its rows then store seven moments (the
// M_Y, M_XY and M_YY of the row follow from them and the row's dy).
template <int TW, int PPT>
constexpr bool kRowForm = PPT == 1 && TW % 16 == 0;
template <int TW, int PPT>
constexpr int kStoredMoments = kRowForm<TW, PPT> ? M_N - 3 : M_N;

// Row-reduce one Gaussian's MS stored moments and store the four row
// partials of this wave (lanes 15, 31, 47, 63 each hold one row's sum).
template <int NW, int BATCH, int MS>
__device__ __forceinline__ void publish(float* m, bool any, int lane, int wave, int k,
                                        float (*s_red)[4][MS][BATCH]) {
  // the wave's slots start each batch at zero: nothing to write when no lane
  // composited the Gaussian
  if (!any) return;
  static_assert(M_Y == M_N - 3 && M_XY == M_N - 2 && M_YY == M_N - 1, "the dy moments come last");
  const int row = lane >> 4;
  row_sums<MS>(m);
  if ((lane & 15) == 15) {
#pragma unroll
    for (int c = 0; c < MS; ++c) s_red[wave][row][c][k] = m[c];
  }
}

// LDS of the backward: one batch of records, their ids, the row partials of
// the MS stored moments, NW * 4 * MS * BATCH floats, and the batch's sums.
template <int NW, int BATCH, int MS>
struct BwdShared {
  float4 q0[BATCH], q1[BATCH], q2[BATCH];
  uint32_t id[BATCH];
  float red[NW][4][MS][BATCH];   // moments per (wave, 16-lane row)
  float tot[M_N][BATCH];         // per Gaussian of the batch, over the workgroup
  uint32_t fail;
};
template <int TW, int TH, int PPT, int BATCH>
using BwdSharedFor = BwdShared<TW * TH / PPT / 64, BATCH, kStoredMoments<TW, PPT>>;

// Backward of one work unit: a tile's whole list, or with chunking chunk
// `chunk` of it. BATCH: Gaussians staged per round (the batch depth). X: the
// tile's forward runs in the same launch and the state is read
// device-coherently; with wait the unit first waits until the tile is marked
// done and reads the tile's longest walk from memory, else the caller is the
// tile's own forward workgroup and passes it (tile_last).
template <int TW, int TH, int PPT, int BATCH, bool X>
__device__ __forceinline__ void backward_unit(const BlendArgs& a, BwdSharedFor<TW, TH, PPT, BATCH>& sh,
                                              int tile, int chunk, bool wait, uint32_t tile_last) {
  using Shape = TileShape<TW, TH, PPT>;
  constexpr int NT = Shape::NT;
  constexpr int ROWS = Shape::ROWS;
  constexpr int NW = NT / 64;
  constexpr bool ROWY = kRowForm<TW, PPT>;
  constexpr int MS = kStoredMoments<TW, PPT>;
  static_assert(BATCH <= NT, "one staged Gaussian per thread");
  float4* s_q0 = sh.q0;
  float4* s_q1 = sh.q1;
  float4* s_q2 = sh.q2;
  uint32_t* s_id = sh.id;
  float (*s_red)[4][MS][BATCH] = sh.red;
  float (*s_tot)[BATCH] = sh.tot;
  uint32_t lo = 0, hi = 0xFFFFFFFFu;
  if (a.chunk_len > 0) {
    lo = (uint32_t)chunk * (uint32_t)a.chunk_len;
    if (chunk < a.max_chunks - 1) hi = lo + (uint32_t)a.chunk_len;
  }
  if (X && wait) {
    // Wait for the tile's forward. Workgroups are dispatched in index order
    // and every forward precedes every backward unit, so the forward this
    // unit waits for is resident or done, and forwards wait for nothing. The
    // wait is bounded all the same: on expiry the error word is set and the
    // unit adds nothing.
    if (threadIdx.x == 0) {
      uint32_t spins = 0, fail = 0;
      while (__hip_atomic_load(a.tile_done + tile, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
        if (++spins > kWaitLimit) {
          fail = 1;
          atomicOr(a.err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      sh.fail = fail;
    }
    __syncthreads();
    if (sh.fail) return;
  }
  const uint2 rg = a.ranges[tile];
  const uint32_t maxlast = min(wait || !X ? ld_u32<X>(a.tile_last + tile) : tile_last, rg.y - rg.x);
  if (lo >= maxlast) return;   // nothing composited in this unit's positions
  const uint32_t top = min(hi, maxlast);
  const int view = find_view(a.views, a.num_views, tile);
  const ViewDesc& V = a.views[view];
  const int lt = tile - V.tile_offset;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int px = tx * TW + (tid % TW);
  const float xs = (float)px + 0.5f;
  const int64_t HW = (int64_t)V.width * V.height;
  // image gradients: those of the fused loss when the forward formed them
  const ViewImages gimg = X ? a.loss_grad[view] : a.images[view];
  float ys[PPT], T[PPT], S[PPT], gc0[PPT], gc1[PPT], gc2[PPT], gd[PPT], tb[PPT];
  uint32_t mylast[PPT];
  uint32_t tmax = 0;
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int py = ty * TH + (tid / TW) + i * ROWS;
    ys[i] = (float)py + 0.5f;
    T[i] = 1.0f;
    S[i] = 0.0f;
    gc0[i] = gc1[i] = gc2[i] = gd[i] = 0.0f;
    float ga = 0.0f;
    mylast[i] = 0;
    if (px < V.width && py < V.height) {
      const int64_t p = (int64_t)py * V.width + px;
      T[i] = ld_f32<X>(a.tfinal + V.pix_offset + p);
      mylast[i] = ld_u32<X>(a.last + V.pix_offset + p);
      if (gimg.rgb) {
        gc0[i] = ld_f32<X>(gimg.rgb + p);
        gc1[i] = ld_f32<X>(gimg.rgb + HW + p);
        gc2[i] = ld_f32<X>(gimg.rgb + 2 * HW + p);
      }
      if (gimg.depth) gd[i] = ld_f32<X>(gimg.depth + p);
      if (gimg.alpha) ga = ld_f32<X>(gimg.alpha + p);
    }
    // T_final (dL/dalpha_out - dL/drgb . bg): the background term of dL/dalpha_k
    tb[i] = T[i] * (ga - (gc0[i] * a.bg[0] + gc1[i] * a.bg[1] + gc2[i] * a.bg[2]));
    if (mylast[i] > hi) {
      // composited Gaussians lie past this chunk: start from the state the
      // forward recorded at the chunk's end. The suffix the walk carries is
      // normalised by the transmittance, S = sum_{j >= hi} x_j w_j / T_hi with
      // x_j = dL/drgb . rgb_j + dL/ddepth z_j; the sum is taken over the
      // per-chunk sums of the later chunks up to the one holding the pixel's
      // last composited Gaussian.
      const int64_t st = a.ckpt_stride;
      const int64_t pix = V.pix_offset + (int64_t)(ty * TH + (tid / TW) + i * ROWS) * V.width + px;
      const uint32_t clast = min((mylast[i] - 1) / (uint32_t)a.chunk_len, (uint32_t)a.max_chunks - 1);
      float rest = 0.0f;
      for (uint32_t c = chunk + 1; c <= clast; ++c) {
        const float* ck = a.ckpt + (int64_t)c * kCkptFields * st + pix;
        rest += fmaf(gc0[i], ld_f32<X>(ck + st),
                     fmaf(gc1[i], ld_f32<X>(ck + 2 * st), fmaf(gc2[i], ld_f32<X>(ck + 3 * st), gd[i] * ld_f32<X>(ck + 4 * st))));
      }
      const float Th = ld_f32<X>(a.ckpt + (int64_t)(chunk + 1) * kCkptFields * st + pix);
      T[i] = Th;
      S[i] = rest / Th;
    }
    tmax = max(tmax, mylast[i]);
  }
  // list positions at or past the wave's largest last position are skipped
  const uint32_t wlast = __builtin_amdgcn_readfirstlane(wave_max_u32(tmax));
  // the unit walks positions [lo, top) from the back
  const int64_t base = (int64_t)rg.x + lo;
  for (int64_t bend = (int64_t)rg.x + top; bend > base; bend -= BATCH) {
    const int64_t b0 = bend - BATCH > base ? bend - BATCH : base;
    const int cnt = (int)(bend - b0);
    __syncthreads();
    if (tid < cnt) {
      const uint32_t sid = a.inst_vals[b0 + tid];
      s_id[tid] = sid;
      const Splat* sp = a.splats + sid;
      stage_record(sp->w0, sp->w1, sp->w2, s_q0[tid], s_q1[tid], s_q2[tid]);
    }
    {
      float* mine = &s_red[wave][0][0][0];
      for (int e = lane; e < 4 * MS * BATCH; e += 64) mine[e] = 0.0f;
    }
    __syncthreads();
    const uint32_t lbase = (uint32_t)(b0 - rg.x);
    int k = cnt - 1;
    for (; k >= 1; k -= 2) {
      // Gaussians k (nearer the back, processed first) and k - 1
      const bool la = lbase + k < wlast;
      const bool lb = lbase + k - 1 < wlast;
      if (!la && !lb) continue;
      const float4 qa0 = s_q0[k], qa1 = s_q1[k], qa2 = s_q2[k];
      const float4 qb0 = s_q0[k - 1], qb1 = s_q1[k - 1], qb2 = s_q2[k - 1];
      float ma[M_N], mb[M_N];
      bool ca = false, cb = false;
      bool okA[PPT], okB[PPT], clA[PPT], clB[PPT];
      float alA[PPT], alB[PPT], GA[PPT], GB[PPT], dxA[PPT], dyA[PPT], dxB[PPT], dyB[PPT];
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        float dxa, dya, Ga, ala, dxb, dyb, Gb, alb;
        bool cla, clb;
        // both alphas unconditionally (positions past the wave's walk are
        // masked below), so that the two exponentials' latencies overlap
        const bool pa = pair_alpha(qa0, qa1, xs, ys[i], dxa, dya, Ga, ala, cla);
        const bool pb = pair_alpha(qb0, qb1, xs, ys[i], dxb, dyb, Gb, alb, clb);
        const bool oka = la && pa && (lbase + k < mylast[i]);
        const bool okb = lb && pb && (lbase + k - 1 < mylast[i]);
        ca = ca || oka;
        cb = cb || okb;
        okA[i] = oka; okB[i] = okb;
        alA[i] = ala; alB[i] = alb;
        GA[i] = Ga; GB[i] = Gb;
        clA[i] = cla; clB[i] = clb;
        dxA[i] = dxa; dyA[i] = dya; dxB[i] = dxb; dyB[i] = dyb;
      }
      // a Gaussian no lane of the wave composited changes nothing: skip it
      // with a wave-uniform branch
      const bool anya = __ballot(ca) != 0ull, anyb = __ballot(cb) != 0ull;
      if (anya) {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
          if (i == 0)
            reverse_one<true, ROWY>(okA[i], alA[i], GA[i], clA[i], dxA[i], dyA[i], qa1, qa2, gc0[i], gc1[i], gc2[i], gd[i],
                              tb[i], T[i], S[i], ma);
          else
            reverse_one<false, ROWY>(okA[i], alA[i], GA[i], clA[i], dxA[i], dyA[i], qa1, qa2, gc0[i], gc1[i], gc2[i],
                               gd[i], tb[i], T[i], S[i], ma);
        }
      }
      if (anyb) {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
          if (i == 0)
            reverse_one<true, ROWY>(okB[i], alB[i], GB[i], clB[i], dxB[i], dyB[i], qb1, qb2, gc0[i], gc1[i], gc2[i], gd[i],
                              tb[i], T[i], S[i], mb);
          else
            reverse_one<false, ROWY>(okB[i], alB[i], GB[i], clB[i], dxB[i], dyB[i], qb1, qb2, gc0[i], gc1[i], gc2[i],
                               gd[i], tb[i], T[i], S[i], mb);
        }
      }
      publish<NW, BATCH, MS>(ma, anya, lane, wave, k, s_red);
      publish<NW, BATCH, MS>(mb, anyb, lane, wave, k - 1, s_red);
    }
    if (k == 0 && lbase < wlast) {
      const float4 q0 = s_q0[0], q1 = s_q1[0], q2 = s_q2[0];
      float m[M_N];
      bool cc = false;
      bool okc[PPT], clc[PPT];
      float alc[PPT], Gc[PPT], dxc[PPT], dyc[PPT];
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        okc[i] = pair_alpha(q0, q1, xs, ys[i], dxc[i], dyc[i], Gc[i], alc[i], clc[i]) && (lbase < mylast[i]);
        cc = cc || okc[i];
      }
      const bool anyc = __ballot(cc) != 0ull;
      if (anyc) {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
          if (i == 0)
            reverse_one<true, ROWY>(okc[i], alc[i], Gc[i], clc[i], dxc[i], dyc[i], q1, q2, gc0[i], gc1[i], gc2[i], gd[i],
                              tb[i], T[i], S[i], m);
          else
            reverse_one<false, ROWY>(okc[i], alc[i], Gc[i], clc[i], dxc[i], dyc[i], q1, q2, gc0[i], gc1[i], gc2[i], gd[i],
                               tb[i], T[i], S[i], m);
        }
      }
      publish<NW, BATCH, MS>(m, anyc, lane, wave, 0, s_red);
    }
    __syncthreads();
    // sum the row partials of every wave, then turn the moments into
    // screen-space gradients and add them with one atomic per (Gaussian,
    // component). In the row form M_Y, M_XY and M_YY are the rows' sums of
    // dL/dopacity's term (O) and of its dx moment weighted by the row's dy
    // (dy^2 for M_YY; dy formed as every lane of the row formed it), and the
    // spatial moments take the opacity.
    for (int e = tid; e < cnt * M_N; e += NT) {
      const int c = e / cnt, kk = e - c * cnt;
      float sum = 0.0f;
      if (c < MS) {
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
          for (int r = 0; r < 4; ++r) sum += s_red[w][r][c][kk];
      } else if (ROWY) {
        const float v = s_q0[kk].y;
        const int src = c == M_XY ? M_X : M_O;
#pragma unroll 1
        for (int w = 0; w < NW; ++w)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float dy = v - ((float)(ty * TH + (w * 64 + r * 16) / TW) + 0.5f);
            const float t = s_red[w][r][src < MS ? src : 0][kk];
            sum += c == M_YY ? dy * (dy * t) : dy * t;
          }
      }
      s_tot[c][kk] = sum;
    }
    __syncthreads();
    for (int kk = tid; kk < cnt; kk += NT) {
      float mm[M_N];
#pragma unroll
      for (int c = 0; c < M_N; ++c) mm[c] = s_tot[c][kk];
      const float4 q0 = s_q0[kk], q1 = s_q1[kk];
      if (ROWY) {
        const float o = q1.y;
        mm[M_X] *= o;
        mm[M_XX] *= o;
        mm[M_Y] *= o;
        mm[M_XY] *= o;
        mm[M_YY] *= o;
      }
      float g[G2_N];
      // d power / d u = -(A dx + B dy) = 2 (-A/2) dx + (-B) dy, likewise for v
      g[G2_U] = 2.0f * q0.z * mm[M_X] + q0.w * mm[M_Y];
      g[G2_V] = q0.w * mm[M_X] + 2.0f * q1.x * mm[M_Y];
      g[G2_A] = -0.5f * mm[M_XX];
      g[G2_B] = -mm[M_XY];
      g[G2_C] = -0.5f * mm[M_YY];
      g[G2_O] = mm[M_O];
      g[G2_R] = mm[M_R];
      g[G2_G] = mm[M_G];
      g[G2_BL] = mm[M_B];
      g[G2_Z] = mm[M_Z];
      float* dst = a.g2 + (int64_t)s_id[kk] * G2_N;
#pragma unroll
      for (int c = 0; c < G2_N; ++c)
        if (g[c] != 0.0f) unsafeAtomicAdd(dst + c, g[c]);
    }
  }
}

// Work units alone: the chunk that takes the rest of the list (the longest
// possible) of every tile first, then chunks 0, 1, ... of every tile.
template <int TW, int TH, int PPT, int BATCH>
__global__ void __launch_bounds__(TW * TH / PPT) __attribute__((amdgpu_waves_per_eu(4)))
blend_backward_kernel(BlendArgs a) {
  __shared__ BwdSharedFor<TW, TH, PPT, BATCH> sh;
  int unit = (int)blockIdx.x, chunk = 0;
  if (a.chunk_len > 0) {
    const int cu = unit / a.num_tiles;
    unit -= cu * a.num_tiles;
    chunk = cu == 0 ? a.max_chunks - 1 : cu - 1;
  }
  backward_unit<TW, TH, PPT, BATCH, false>(a, sh, a.order ? (int)a.order[unit] : unit, chunk, false, 0u);
}

// Forward and backward of every tile in one launch: workgroups below
// num_tiles composite a tile, the rest take the backward's work units, each
// waiting for its tile's forward. The backward's units then fill the
// forward's tail (tiles whose lists are short finish early) and the
// forward's tiles no longer wait for the slowest one before any backward
// starts. The two phases share one LDS allocation.
template <int TW, int TH, int PPT, int BATCH, bool CK>
__global__ void __launch_bounds__(TW * TH / PPT) __attribute__((amdgpu_waves_per_eu(4)))
blend_fused_kernel(BlendArgs a) {
  using F = FwdShared<TW * TH / PPT>;
  using B = BwdSharedFor<TW, TH, PPT, BATCH>;
  __shared__ __align__(16) unsigned char smem[sizeof(F) > sizeof(B) ? sizeof(F) : sizeof(B)];
  const int b = (int)blockIdx.x;
  int tile, chunk;
  uint32_t tl = 0;
  if (b < a.num_tiles) {
    // the tile's forward, then the first chunk of its backward (the whole
    // list when unchunked) without waiting: each thread reads back only its
    // own pixels' state, and the tile's longest walk comes from LDS
    tile = a.order ? (int)a.order[b] : b;
    chunk = 0;
    tl = forward_tile<TW, TH, PPT, CK, true>(a, *reinterpret_cast<F*>(smem), tile);
    __syncthreads();   // every thread has read the forward's LDS before the backward reuses it
  } else {
    // chunks 1, 2, ... of every tile, in chunk order, each waiting for its
    // tile's forward
    const int unit = b - a.num_tiles;
    const int cu = unit / a.num_tiles, t = unit - cu * a.num_tiles;
    tile = a.order ? (int)a.order[t] : t;
    chunk = cu + 1;
  }
  // one copy of the backward for both kinds of workgroup
  backward_unit<TW, TH, PPT, BATCH, true>(a, *reinterpret_cast<B*>(smem), tile, chunk, b >= a.num_tiles, tl);
}

// The fused launch as a persistent grid over a work queue, for more units
// than the device holds at once (the plain grid above needs every workgroup
// resident, or a waiting backward unit could hold the slot its tile's forward
// needs). As many workgroups as fit take units from a counter in the plain
// grid's order: every tile's forward with its first chunk, then chunk 1 of
// every tile, then chunk 2, ... A later chunk is thus taken only after its
// tile's forward was taken by a running workgroup, which never waits, so
// every wait ends whatever the tile count.
template <int TW, int TH, int PPT, int BATCH, bool CK>
__global__ void __launch_bounds__(TW * TH / PPT) __attribute__((amdgpu_waves_per_eu(4)))
blend_fused_queue_kernel(BlendArgs a, uint32_t units) {
  using F = FwdShared<TW * TH / PPT>;
  using B = BwdSharedFor<TW, TH, PPT, BATCH>;
  __shared__ __align__(16) unsigned char smem[sizeof(F) > sizeof(B) ? sizeof(F) : sizeof(B)];
  __shared__ uint32_t s_unit;
  while (true) {
    if (threadIdx.x == 0) s_unit = atomicAdd(a.queue, 1u);
    __syncthreads();
    const uint32_t u = s_unit;
    if (u >= units) break;
    if (u < (uint32_t)a.num_tiles) {
      const int tile = a.order ? (int)a.order[u] : (int)u;
      const uint32_t tl = forward_tile<TW, TH, PPT, CK, true>(a, *reinterpret_cast<F*>(smem), tile);
      __syncthreads();
      backward_unit<TW, TH, PPT, BATCH, true>(a, *reinterpret_cast<B*>(smem), tile, 0, false, tl);
    } else {
      const int unit = (int)(u - (uint32_t)a.num_tiles);
      const int cu = unit / a.num_tiles, t = unit - cu * a.num_tiles;
      backward_unit<TW, TH, PPT, BATCH, true>(a, *reinterpret_cast<B*>(smem), a.order ? (int)a.order[t] : t,
                                              cu + 1, true, 0u);
    }
    __syncthreads();   // the LDS and s_unit are free for the next unit
  }
}

// ---------------------------------------------------------------------------
// Splat-parallel backward (a selectable schedule). One wavefront per tile.
// The tile's list is walked back to front in batches of 64 positions; lane j
// owns position hi - 1 - j of the batch [lo, hi) and accumulates that
// Gaussian's gradient over the tile's pixels in registers. The pixels stream
// through the lanes as a software pipeline: at step t lane j takes pixel
// t - j, so the pixel meets the batch's Gaussians back to front, and its
// reverse-walk state (transmittance, suffix) moves one lane up per step by a
// DPP wave shift. Lane 0 takes a pixel's state from LDS, lane 63 leaves it
// there for the next batch. The pixels are ordered by their walk length
// (longest first), so a batch streams only the pixels whose walks reach it.
// No wave reduction: one set of atomics per (tile, Gaussian).
// ---------------------------------------------------------------------------
template <int NPIX>
struct SplatShared {
  float4 pix[NPIX];      // per ranked pixel: (x, y sample point, background term of dL/dalpha, last as bits)
  float4 grad[NPIX];     // per ranked pixel: dL/d(r, g, b, depth)
  float2 state[NPIX];    // per ranked pixel: (T, S) entering the current batch
  uint32_t last[NPIX];   // per pixel of the tile, in tile order
};

__device__ __forceinline__ float lane_shift_up(float x) {
  // lane i receives lane i - 1's value (wave_shr:1); lane 0 receives 0
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xF, 0xF, false));
}

template <int TW, int TH>
__global__ void __launch_bounds__(64) blend_backward_splat_kernel(BlendArgs a) {
  constexpr int NPIX = TW * TH;
  __shared__ SplatShared<NPIX> sh;
  const int lane = threadIdx.x;
  const int tile = a.order ? (int)a.order[blockIdx.x] : (int)blockIdx.x;
  const uint2 rg = a.ranges[tile];
  const uint32_t top = min(a.tile_last[tile], rg.y - rg.x);
  if (top == 0) return;
  const int view = find_view(a.views, a.num_views, tile);
  const ViewDesc& V = a.views[view];
  const int lt = tile - V.tile_offset;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const ViewImages gimg = a.images[view];
  const int64_t HW = (int64_t)V.width * V.height;
  for (int q = lane; q < NPIX; q += 64) {
    const int px = tx * TW + q % TW, py = ty * TH + q / TW;
    sh.last[q] = (px < V.width && py < V.height) ? a.last[V.pix_offset + (int64_t)py * V.width + px] : 0u;
  }
  __syncthreads();
  // rank of every pixel by walk length, longest first (ties by tile order)
  for (int q = lane; q < NPIX; q += 64) {
    const uint32_t lq = sh.last[q];
    int r = 0;
    for (int o = 0; o < NPIX; ++o) {
      const uint32_t lo = sh.last[o];
      r += (lo > lq || (lo == lq && o < q)) ? 1 : 0;
    }
    const int px = tx * TW + q % TW, py = ty * TH + q / TW;
    float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, gd = 0.0f, ga = 0.0f;
    if (lq > 0) {
      const int64_t p = (int64_t)py * V.width + px;
      T = a.tfinal[V.pix_offset + p];
      if (gimg.rgb) {
        g0 = gimg.rgb[p];
        g1 = gimg.rgb[HW + p];
        g2 = gimg.rgb[2 * HW + p];
      }
      if (gimg.depth) gd = gimg.depth[p];
      if (gimg.alpha) ga = gimg.alpha[p];
    }
    const float tb = T * (ga - (g0 * a.bg[0] + g1 * a.bg[1] + g2 * a.bg[2]));
    sh.pix[r] = make_float4((float)px + 0.5f, (float)py + 0.5f, tb, __uint_as_float(lq));
    sh.grad[r] = make_float4(g0, g1, g2, gd);
    sh.state[r] = make_float2(T, 0.0f);
  }
  __syncthreads();
  for (int hi = (int)top; hi > 0; hi -= 64) {
    const int lo = hi > 64 ? hi - 64 : 0;
    // pixels whose walk reaches this batch (last > lo): a prefix of the ranking
    int n = 0;
    for (int r0 = 0; r0 < NPIX; r0 += 64)
      n += __popcll(__ballot(__float_as_uint(sh.pix[r0 + lane].w) > (uint32_t)lo));
    const int pos = hi - 1 - lane;
    const bool have = pos >= lo;
    float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0, q2 = q0;
    uint32_t sid = 0;
    if (have) {
      sid = a.inst_vals[rg.x + pos];
      const Splat* sp = a.splats + sid;
      stage_record(sp->w0, sp->w1, sp->w2, q0, q1, q2);
    }
    float m[M_N];
#pragma unroll
    for (int c = 0; c < M_N; ++c) m[c] = 0.0f;
    float Tin = 0.0f, Sin = 0.0f;
    for (int t = 0; t < n + 63; ++t) {
      const int r = t - lane;
      const bool valid = r >= 0 && r < n;
      const int rr = valid ? r : 0;
      const float4 pa = sh.pix[rr];
      const float4 pg = sh.grad[rr];
      float T = Tin, S = Sin;
      if (lane == 0) {
        const float2 st = sh.state[rr];
        T = st.x;
        S = st.y;
      }
      float dx, dy, G, alpha;
      bool clamped;
      const bool ok = pair_alpha(q0, q1, pa.x, pa.y, dx, dy, G, alpha, clamped) && valid && have &&
                      (uint32_t)pos < __float_as_uint(pa.w);
      reverse_one<false, false>(ok, alpha, G, clamped, dx, dy, q1, q2, pg.x, pg.y, pg.z, pg.w, pa.z, T, S, m);
      if (lane == 63 && valid) sh.state[r] = make_float2(T, S);
      Tin = lane_shift_up(T);
      Sin = lane_shift_up(S);
    }
    if (have) {
      float g[G2_N];
      g[G2_U] = 2.0f * q0.z * m[M_X] + q0.w * m[M_Y];
      g[G2_V] = q0.w * m[M_X] + 2.0f * q1.x * m[M_Y];
      g[G2_A] = -0.5f * m[M_XX];
      g[G2_B] = -m[M_XY];
      g[G2_C] = -0.5f * m[M_YY];
      g[G2_O] = m[M_O];
      g[G2_R] = m[M_R];
      g[G2_G] = m[M_G];
      g[G2_BL] = m[M_B];
      g[G2_Z] = m[M_Z];
      float* dst = a.g2 + (int64_t)sid * G2_N;
#pragma unroll
      for (int c = 0; c < G2_N; ++c)
        if (g[c] != 0.0f) unsafeAtomicAdd(dst + c, g[c]);
    }
    __syncthreads();   // lane 63's states reach LDS before the next batch reads them
  }
}

template <int TW, int TH>
void splat_launch(const BlendArgs& a, hipStream_t st) {
  blend_backward_splat_kernel<TW, TH><<<a.num_tiles, 64, 0, st>>>(a);
}

template <int TW, int TH>
void fwd_launch(const BlendArgs& a, int ppt, hipStream_t st) {
  constexpr int P2 = TW * TH >= 128 ? 2 : 1;
  const bool ck = a.chunk_len > 0;
  if (ppt == 2 && P2 == 2) {
    if (ck) blend_forward_kernel<TW, TH, P2, true><<<a.num_tiles, TW * TH / P2, 0, st>>>(a);
    else blend_forward_kernel<TW, TH, P2, false><<<a.num_tiles, TW * TH / P2, 0, st>>>(a);
  } else {
    if (ck) blend_forward_kernel<TW, TH, 1, true><<<a.num_tiles, TW * TH, 0, st>>>(a);
    else blend_forward_kernel<TW, TH, 1, false><<<a.num_tiles, TW * TH, 0, st>>>(a);
  }
}
template <int TW, int TH, int PPT>
void bwd_launch_depth(const BlendArgs& a, int depth, hipStream_t st) {
  constexpr int NT = TW * TH / PPT;
  constexpr int D64 = NT >= 64 ? 64 : NT;
  if (depth == 0) depth = NT >= 256 ? 32 : 64;
  const int64_t units = (int64_t)a.num_tiles * (a.chunk_len > 0 ? a.max_chunks : 1);
  const dim3 grid((unsigned)units);
  if (depth == 16) blend_backward_kernel<TW, TH, PPT, 16><<<grid, NT, 0, st>>>(a);
  else if (depth == 32) blend_backward_kernel<TW, TH, PPT, 32><<<grid, NT, 0, st>>>(a);
  else blend_backward_kernel<TW, TH, PPT, D64><<<grid, NT, 0, st>>>(a);
}

template <int TW, int TH, int PPT>
void fused_launch_ppt(const BlendArgs& a, hipStream_t st) {
  constexpr int NT = TW * TH / PPT;
  constexpr int D = NT >= 256 ? 32 : (NT >= 64 ? 64 : NT);
  // a workgroup per tile (forward and the first chunk), one per later chunk
  const int64_t units = (int64_t)a.num_tiles * (a.chunk_len > 0 ? a.max_chunks - 1 : 0);
  const int64_t total = a.num_tiles + units;
  if (a.queue) {
    const int64_t g = total < (int64_t)a.queue_grid ? total : (int64_t)a.queue_grid;
    const dim3 grid((unsigned)(g > 1 ? g : 1));
    if (a.chunk_len > 0) blend_fused_queue_kernel<TW, TH, PPT, D, true><<<grid, NT, 0, st>>>(a, (uint32_t)total);
    else blend_fused_queue_kernel<TW, TH, PPT, D, false><<<grid, NT, 0, st>>>(a, (uint32_t)total);
    return;
  }
  const dim3 grid((unsigned)total);
  if (a.chunk_len > 0) blend_fused_kernel<TW, TH, PPT, D, true><<<grid, NT, 0, st>>>(a);
  else blend_fused_kernel<TW, TH, PPT, D, false><<<grid, NT, 0, st>>>(a);
}

template <int TW, int TH, int PPT>
int64_t fused_resident_ppt() {
  constexpr int NT = TW * TH / PPT;
  constexpr int D = NT >= 256 ? 32 : (NT >= 64 ? 64 : NT);
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, blend_fused_kernel<TW, TH, PPT, D, true>, NT, 0) !=
      hipSuccess)
    return 0;
  return (int64_t)cus * per_cu;
}

template <int TW, int TH>
int64_t fused_resident(int ppt) {
  if (ppt == 2 && TW * TH >= 128) return fused_resident_ppt<TW, TH, (TW * TH >= 128 ? 2 : 1)>();
  return fused_resident_ppt<TW, TH, 1>();
}

template <int TW, int TH>
void fused_launch(const BlendArgs& a, int ppt, hipStream_t st) {
  if (ppt == 2 && TW * TH >= 128) fused_launch_ppt<TW, TH, (TW * TH >= 128 ? 2 : 1)>(a, st);
  else fused_launch_ppt<TW, TH, 1>(a, st);
}

template <int TW, int TH>
void bwd_launch(const BlendArgs& a, int ppt, int depth, hipStream_t st) {
  if (ppt == 2 && TW * TH >= 128) bwd_launch_depth<TW, TH, (TW * TH >= 128 ? 2 : 1)>(a, depth, st);
  else bwd_launch_depth<TW, TH, 1>(a, depth, st);
}

__global__ void __launch_bounds__(256) loss_l1_kernel(const ViewDesc* __restrict__ views,
                                                      const ViewImages* __restrict__ rendered,
                                                      const ViewImages* __restrict__ target,
                                                      const ViewImages* __restrict__ grad, float depth_weight,
                                                      float* __restrict__ loss) {
  __shared__ float wsum[4];
  const int view = blockIdx.y;
  const ViewDesc& V = views[view];
  const int64_t HW = (int64_t)V.width * V.height;
  const float inv3 = 1.0f / (3.0f * (float)HW), inv1 = depth_weight / (float)HW;
  const ViewImages r = rendered[view], t = target[view], g = grad[view];
  float acc = 0.0f;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < HW; p += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float d = r.rgb[ch * HW + p] - t.rgb[ch * HW + p];
      g.rgb[ch * HW + p] = d > 0.0f ? inv3 : (d < 0.0f ? -inv3 : 0.0f);
      acc += fabsf(d) * inv3;
    }
    const float dd = r.depth[p] - t.depth[p];
    g.depth[p] = dd > 0.0f ? inv1 : (dd < 0.0f ? -inv1 : 0.0f);
    acc += fabsf(dd) * inv1;
    if (g.alpha) g.alpha[p] = 0.0f;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) unsafeAtomicAdd(loss, wsum[0] + wsum[1] + wsum[2] + wsum[3]);
}

__device__ __forceinline__ void adam_one(float gi, float& mi, float& vi, float& pi, float b1, float b2, float eps,
                                         float bc1, float bc2, float lr) {
  mi = b1 * mi + (1.0f - b1) * gi;
  vi = b2 * vi + (1.0f - b2) * gi * gi;
  pi -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Adam over the parameter planes: workgroup column y = plane (its learning
// rate in a scalar register), a grid-stride walk along the plane; with VEC
// (every plane 16-byte aligned) four scalars per load and store, the last
// num mod 4 scalars one by one.
template <bool VEC>
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t num,
                                                   int64_t stride, const float* __restrict__ lr, float b1, float b2,
                                                   float eps, float bc1, float bc2,
                                                   const uint32_t* __restrict__ step_dev,
                                                   const uint32_t* __restrict__ skip) {
  if (skip && (skip[0] | skip[1])) return;
  if (step_dev) {
    // in double, as the host does: 1 - b^step cancels badly in float
    __shared__ float s_bc[2];
    if (threadIdx.x == 0) {
      const int step = *step_dev;
      s_bc[0] = (float)(1.0 - pow((double)b1, (double)step));
      s_bc[1] = (float)(1.0 - pow((double)b2, (double)step));
    }
    __syncthreads();
    bc1 = s_bc[0];
    bc2 = s_bc[1];
  }
  const int64_t off = (int64_t)blockIdx.y * stride;
  const float lrp = lr[blockIdx.y];
  p += off;
  g += off;
  m += off;
  v += off;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (VEC) {
    const int64_t n4 = num >> 2;
    for (; i < n4; i += step) {
      const float4 gi = reinterpret_cast<const float4*>(g)[i];
      float4 mi = reinterpret_cast<const float4*>(m)[i];
      float4 vi = reinterpret_cast<const float4*>(v)[i];
      float4 pi = reinterpret_cast<const float4*>(p)[i];
      adam_one(gi.x, mi.x, vi.x, pi.x, b1, b2, eps, bc1, bc2, lrp);
      adam_one(gi.y, mi.y, vi.y, pi.y, b1, b2, eps, bc1, bc2, lrp);
      adam_one(gi.z, mi.z, vi.z, pi.z, b1, b2, eps, bc1, bc2, lrp);
      adam_one(gi.w, mi.w, vi.w, pi.w, b1, b2, eps, bc1, bc2, lrp);
      reinterpret_cast<float4*>(m)[i] = mi;
      reinterpret_cast<float4*>(v)[i] = vi;
      reinterpret_cast<float4*>(p)[i] = pi;
    }
    i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  }
  for (; i < num; i += step) {
    float mi = m[i], vi = v[i], pi = p[i];
    adam_one(g[i], mi, vi, pi, b1, b2, eps, bc1, bc2, lrp);
    m[i] = mi;
    v[i] = vi;
    p[i] = pi;
  }
}

int grid_cap(int64_t n, int block) {
  int64_t gsz = (n + block - 1) / block;
  if (gsz < 1) gsz = 1;
  if (gsz > 16384) gsz = 16384;
  return (int)gsz;
}

}  // namespace

bool blend_supported(int tile_w, int tile_h) {
  return (tile_w == 16 && tile_h == 16) || (tile_w == 16 && tile_h == 8) || (tile_w == 8 && tile_h == 8) ||
         (tile_w == 32 && tile_h == 8);
}

void launch_blend_forward(const BlendArgs& a, int tile_w, int tile_h, int ppt, hipStream_t st) {
  if (a.num_tiles == 0) return;
  if (tile_w == 16 && tile_h == 16) fwd_launch<16, 16>(a, ppt, st);
  else if (tile_w == 16 && tile_h == 8) fwd_launch<16, 8>(a, ppt, st);
  else if (tile_w == 8 && tile_h == 8) fwd_launch<8, 8>(a, ppt, st);
  else if (tile_w == 32 && tile_h == 8) fwd_launch<32, 8>(a, ppt, st);
}

void launch_blend_fused(const BlendArgs& a, int tile_w, int tile_h, int ppt, hipStream_t st) {
  if (a.num_tiles == 0) return;
  if (tile_w == 16 && tile_h == 16) fused_launch<16, 16>(a, ppt, st);
  else if (tile_w == 16 && tile_h == 8) fused_launch<16, 8>(a, ppt, st);
  else if (tile_w == 8 && tile_h == 8) fused_launch<8, 8>(a, ppt, st);
  else if (tile_w == 32 && tile_h == 8) fused_launch<32, 8>(a, ppt, st);
}

int64_t blend_fused_resident(int tile_w, int tile_h, int ppt) {
  int64_t r = 0;
  if (tile_w == 16 && tile_h == 16) r = fused_resident<16, 16>(ppt);
  else if (tile_w == 16 && tile_h == 8) r = fused_resident<16, 8>(ppt);
  else if (tile_w == 8 && tile_h == 8) r = fused_resident<8, 8>(ppt);
  else if (tile_w == 32 && tile_h == 8) r = fused_resident<32, 8>(ppt);
  (void)hipGetLastError();
  return r;
}

bool batch_depth_supported(int depth) { return depth == 0 || depth == 16 || depth == 32 || depth == 64; }

bool chunking_supported(int chunk_len, int max_chunks) {
  if (chunk_len == 0) return true;
  return chunk_len > 0 && chunk_len % 16 == 0 && chunk_len <= (1 << 20) && max_chunks >= 1 && max_chunks <= 64;
}

void launch_blend_backward(const BlendArgs& a, int tile_w, int tile_h, int ppt, int depth, hipStream_t st) {
  if (a.num_tiles == 0) return;
  if (tile_w == 16 && tile_h == 16) bwd_launch<16, 16>(a, ppt, depth, st);
  else if (tile_w == 16 && tile_h == 8) bwd_launch<16, 8>(a, ppt, depth, st);
  else if (tile_w == 8 && tile_h == 8) bwd_launch<8, 8>(a, ppt, depth, st);
  else if (tile_w == 32 && tile_h == 8) bwd_launch<32, 8>(a, ppt, depth, st);
}

void launch_blend_backward_splat(const BlendArgs& a, int tile_w, int tile_h, hipStream_t st) {
  if (a.num_tiles == 0) return;
  if (tile_w == 16 && tile_h == 16) splat_launch<16, 16>(a, st);
  else if (tile_w == 16 && tile_h == 8) splat_launch<16, 8>(a, st);
  else if (tile_w == 8 && tile_h == 8) splat_launch<8, 8>(a, st);
  else if (tile_w == 32 && tile_h == 8) splat_launch<32, 8>(a, st);
}

void launch_loss_l1(const ViewDesc* views, const ViewImages* rendered, const ViewImages* target,
                    const ViewImages* grad, int num_views, int max_pixels, float depth_weight, float* loss,
                    bool clear_loss, hipStream_t st) {
  if (loss && clear_loss) launch_fill_f32(loss, 0.0f, 1, st);
  dim3 grid(grid_cap(max_pixels, 256) < 1024 ? grid_cap(max_pixels, 256) : 1024, num_views);
  loss_l1_kernel<<<grid, 256, 0, st>>>(views, rendered, target, grad, depth_weight, loss);
}

void launch_adam(float* p, const float* g, float* m, float* v, int64_t num, int64_t stride, int planes,
                 const float* lr_dev, float b1, float b2, float eps, float bc1, float bc2, const uint32_t* step_dev,
                 const uint32_t* skip, hipStream_t st) {
  if (num == 0 || planes == 0) return;
  const bool vec = stride % 4 == 0 && (((uintptr_t)p | (uintptr_t)g | (uintptr_t)m | (uintptr_t)v) & 15u) == 0;
  const int64_t per = vec ? (num + 3) / 4 : num;
  const dim3 grid((unsigned)std::min<int64_t>(std::max<int64_t>((per + 255) / 256, 1), 1024), (unsigned)planes);
  if (vec)
    adam_kernel<true><<<grid, 256, 0, st>>>(p, g, m, v, num, stride, lr_dev, b1, b2, eps, bc1, bc2, step_dev, skip);
  else
    adam_kernel<false><<<grid, 256, 0, st>>>(p, g, m, v, num, stride, lr_dev, b1, b2, eps, bc1, bc2, step_dev, skip);
}

}  // namespace gsr
