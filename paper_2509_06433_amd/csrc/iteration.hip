// The mapping iteration as one HIP graph: render, loss, backward and Adam of
// the continuous map optimisation (paper Sec. II-B, mapping thread), replayed
// per call without host synchronisation.
//
// A graph fixes every launch's grid, so the instance storage has a fixed
// capacity and every kernel after the instance-offset scan reads the count
// from device memory, clamped to the capacity. An iteration whose count
// exceeds the capacity (or whose sort look-back wait expired) still runs
// with bounded, in-range work; its Adam node sees the flag and leaves the
// parameters alone, and the closing node counts it as skipped. The host sees
// the counters through a copy into pinned memory at the end of each replay,
// without waiting for it, and captures a larger graph on the next call.

#include <algorithm>
#include <cstring>
#include <vector>

#include "context.h"

namespace gsr {

namespace {

// Counts an iteration without Gaussians (otherwise the projection backward
// does, in its first workgroup, which saves a node per replay).
__global__ void iteration_end_kernel(IterCounters c) {
  if (threadIdx.x == 0) count_iteration(c);
}

}  // namespace

struct GraphState {
  Buffers B;
  RenderPlan P;
  // what the capture depends on
  float* params = nullptr;
  float* grad = nullptr;
  float* loss = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  int64_t num = -1, stride = -1;
  int deg = -1;
  std::vector<int32_t> sizes;          // width, height per view
  float depth_weight = 0.f, beta1 = 0.f, beta2 = 0.f, eps = 0.f;
  bool adam = false;
  uint32_t profile_mask = 0;
  int64_t capacity = 0;
  bool captured = false;
  // host copies of the descriptors last uploaded
  std::vector<ViewDesc> views;
  std::vector<ViewImages> outs, targets;
  std::vector<float> lr;
  DevBuf tdesc, gimg, lrbuf, stats;
  uint32_t* host_stats = nullptr;      // pinned, written by the node that counts each replay
  uint32_t* host_stats_dev = nullptr;  // its device address
  // One captured graph, instantiated kRing times. With timed stages each
  // instance's event-record nodes are given their own events, so a replay
  // never touches an instance that may still run: instance k is reused only
  // after its previous replay has finished, and its stage times are
  // harvested then.
  static constexpr int kRing = 4;
  struct Instance {
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool launched = false;
    std::vector<TimedPair> events;   // stage, start, end
  };
  hipGraph_t graph = nullptr;
  Instance inst[kRing];
  int next = 0;
  std::vector<TimedPair> timed;      // the placeholder events captured in the graph
  std::vector<std::pair<hipGraphNode_t, hipGraphNode_t>> timed_nodes;
  hipStream_t cap = nullptr;
  hipEvent_t done = nullptr;
  int64_t captures = 0;
  uint32_t seen_skipped = 0;
  bool grow = false;
};

namespace {

// Adds the stage times of instance k's finished replay to the context.
int harvest(gsr_ctx* ctx, GraphState::Instance& I) {
  if (!I.launched) return GSR_OK;
  HIP_TRY(ctx, hipEventSynchronize(I.done));
  for (const TimedPair& t : I.events) {
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, t.a, t.b));
    ctx->acc_ms[t.stage] += ms;
    ctx->acc_n[t.stage] += 1;
  }
  I.launched = false;
  return GSR_OK;
}

void drop_graph(gsr_ctx* ctx, GraphState* G) {
  for (GraphState::Instance& I : G->inst) {
    if (I.launched) (void)harvest(ctx, I);
    if (I.exec) (void)hipGraphExecDestroy(I.exec);
    I.exec = nullptr;
    for (const TimedPair& t : I.events) {
      ctx->ev_pool.push_back(t.a);
      ctx->ev_pool.push_back(t.b);
    }
    I.events.clear();
  }
  if (G->graph) (void)hipGraphDestroy(G->graph);
  G->graph = nullptr;
  for (const TimedPair& t : G->timed) {
    ctx->ev_pool.push_back(t.a);
    ctx->ev_pool.push_back(t.b);
  }
  G->timed.clear();
  G->timed_nodes.clear();
  G->next = 0;
  G->captured = false;
}

int init_state(gsr_ctx* ctx, GraphState* G) {
  HIP_TRY(ctx, hipStreamCreateWithFlags(&G->cap, hipStreamNonBlocking));
  HIP_TRY(ctx, hipEventCreateWithFlags(&G->done, hipEventDisableTiming));
  for (GraphState::Instance& I : G->inst) HIP_TRY(ctx, hipEventCreateWithFlags(&I.done, hipEventDisableTiming));
  HIP_TRY(ctx, hipHostMalloc((void**)&G->host_stats, sizeof(uint32_t) * kStatWords, hipHostMallocDefault));
  std::memset(G->host_stats, 0, sizeof(uint32_t) * kStatWords);
  HIP_TRY(ctx, hipHostGetDevicePointer((void**)&G->host_stats_dev, G->host_stats, 0));
  RET_IF(ensure(ctx, G->stats, sizeof(uint32_t) * kStatWords));
  HIP_TRY(ctx, hipMemset(G->stats.p, 0, sizeof(uint32_t) * kStatWords));
  HIP_TRY(ctx, hipDeviceSynchronize());
  return GSR_OK;
}

// Instance count of the current parameters, from the front half of a render
// into the graph's own buffers.
int measure_instances(gsr_ctx* ctx, GraphState* G, const float* params, const gsr_image* out, int64_t* count,
                      hipStream_t st) {
  RenderPlan& P = G->P;
  P.capacity = std::max<int64_t>(P.capacity, 0);
  RET_IF(size_render(ctx, G->B, P, out, st));
  ClearList L{};
  front_clears(ctx, G->B, P, L);
  launch_clear(L, st);
  const uint32_t mask = ctx->profile_mask;
  ctx->profile_mask = 0;
  const int r = launch_front(ctx, G->B, P, params, st);
  ctx->profile_mask = mask;
  RET_IF(r);
  uint32_t t[2];
  HIP_TRY(ctx, hipMemcpyAsync(ctx->host_total, G->B.total.p, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  std::memcpy(t, ctx->host_total, sizeof(t));
  if (t[1] != 0) return GSR_ERR_DEVICE;
  *count = (int64_t)t[0];
  return GSR_OK;
}

int upload_descriptors(gsr_ctx* ctx, GraphState* G, int nv, const std::vector<ViewImages>& outs,
                       const std::vector<ViewImages>& targets, const float* lr, int planes, bool adam, bool force,
                       hipStream_t st) {
  if (force || std::memcmp(G->views.data(), G->P.views.data(), sizeof(ViewDesc) * nv) != 0) {
    RET_IF(upload(ctx, G->B.views.p, G->P.views.data(), sizeof(ViewDesc) * nv, st));
    G->views = G->P.views;
  }
  if (force || std::memcmp(G->outs.data(), outs.data(), sizeof(ViewImages) * nv) != 0) {
    RET_IF(upload(ctx, G->B.images.p, outs.data(), sizeof(ViewImages) * nv, st));
    G->outs = outs;
  }
  if (force || std::memcmp(G->targets.data(), targets.data(), sizeof(ViewImages) * nv) != 0) {
    RET_IF(upload(ctx, G->tdesc.p, targets.data(), sizeof(ViewImages) * nv, st));
    G->targets = targets;
  }
  if (adam && (force || std::memcmp(G->lr.data(), lr, sizeof(float) * planes) != 0)) {
    RET_IF(upload(ctx, G->lrbuf.p, lr, sizeof(float) * planes, st));
    G->lr.assign(lr, lr + planes);
  }
  return GSR_OK;
}

// Records the whole iteration on the capture stream.
int record_iteration(gsr_ctx* ctx, GraphState* G, float* params, float* grad, float* loss, const gsr_adam* adam,
                     float depth_weight, int planes, hipStream_t st) {
  Buffers& B = G->B;
  RenderPlan& P = G->P;
  uint32_t* totals = as<uint32_t>(B.total);
  // one clear for everything the iteration accumulates into
  ClearList L{};
  front_clears(ctx, B, P, L);
  back_clears(B, P, L);
  // (the gradient is overwritten by the projection backward, so it is not
  // cleared)
  // (g2 is not cleared: it is zero before the first replay and the
  // projection backward zeroes the rows it reads)
  if (loss) L.add(loss, 1);
  const bool fused = use_fused_blend(ctx, P);
  if (fused) L.add(as<uint32_t>(B.tile_done), P.ntiles + 1);
  {
    StageTimer tm(ctx, GSR_STAGE_ZERO, st);
    launch_clear(L, st);
  }
  CHECK_LAUNCH(ctx);
  RET_IF(launch_front(ctx, B, P, params, st));
  // the L1 loss and its image gradients are formed by the compositing itself
  const FusedLoss fl{as<ViewImages>(G->tdesc), depth_weight, loss};
  RET_IF(launch_back(ctx, B, P, st, &fl, fused));
  // the iteration is counted (and the counters reach the pinned host copy)
  // by the projection backward, after every kernel that can raise the error
  // or overflow flag and before Adam, which reads the step count
  const IterCounters ic{totals, as<uint32_t>(G->stats), G->host_stats_dev, adam ? 1 : 0};
  RET_IF(launch_bwd(ctx, B, P, params, grad, false, true, st, fused, &ic));
  if (P.num == 0) {
    iteration_end_kernel<<<1, 64, 0, st>>>(ic);
    CHECK_LAUNCH(ctx);
  }
  if (adam) {
    StageTimer tm(ctx, GSR_STAGE_ADAM, st);
    launch_adam(params, grad, adam->m, adam->v, P.num, P.stride, planes, as<float>(G->lrbuf), adam->beta1,
                adam->beta2, adam->eps, 1.0f, 1.0f, as<uint32_t>(G->stats) + kStatAdamSteps, totals + 1, st);
  }
  CHECK_LAUNCH(ctx);
  return GSR_OK;
}

int capture(gsr_ctx* ctx, GraphState* G, float* params, float* grad, float* loss, const gsr_adam* adam,
            float depth_weight, int planes) {
  drop_graph(ctx, G);
  // events are created before the capture: no event is created while it runs
  const int want = 4 * (__builtin_popcount(ctx->profile_mask) + 2);
  while ((int)ctx->ev_pool.size() < want) {
    hipEvent_t e = nullptr;
    HIP_TRY(ctx, hipEventCreate(&e));
    ctx->ev_pool.push_back(e);
  }
  std::vector<TimedPair> timed;
  // the screen-space gradient accumulators start at zero; each replay leaves
  // them zero again
  launch_fill_f32(as<float>(G->B.g2), 0.0f, G->P.total * G2_N, G->cap);
  CHECK_LAUNCH(ctx);
  HIP_TRY(ctx, hipStreamSynchronize(G->cap));
  HIP_TRY(ctx, hipStreamBeginCapture(G->cap, hipStreamCaptureModeThreadLocal));
  ctx->capture_timed = &timed;
  const int r = record_iteration(ctx, G, params, grad, loss, adam, depth_weight, planes, G->cap);
  ctx->capture_timed = nullptr;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(G->cap, &graph);
  G->timed = timed;
  if (r != GSR_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    drop_graph(ctx, G);
    (void)hipGetLastError();
    if (r != GSR_OK) return r;
    ctx->hip_err = (int)e;
    return GSR_ERR_HIP;
  }
  G->graph = graph;
  for (const TimedPair& t : G->timed) {
    if (!t.na || !t.nb) {
      ctx->hip_err = (int)hipErrorInvalidValue;
      return GSR_ERR_HIP;
    }
    G->timed_nodes.emplace_back(t.na, t.nb);
  }
  // instances, each with its own events (set while no replay can be running)
  const int ring = G->timed.empty() ? 1 : GraphState::kRing;
  for (int k = 0; k < ring; ++k) {
    GraphState::Instance& I = G->inst[k];
    HIP_TRY(ctx, hipGraphInstantiate(&I.exec, graph, nullptr, nullptr, 0));
    for (size_t j = 0; j < G->timed.size(); ++j) {
      hipEvent_t a = take_event(ctx), b = take_event(ctx);
      if (!a || !b) return GSR_ERR_HIP;
      I.events.push_back(TimedPair{G->timed[j].stage, a, b});
      HIP_TRY(ctx, hipGraphExecEventRecordNodeSetEvent(I.exec, G->timed_nodes[j].first, a));
      HIP_TRY(ctx, hipGraphExecEventRecordNodeSetEvent(I.exec, G->timed_nodes[j].second, b));
    }
  }
  G->captured = true;
  G->captures += 1;
  return GSR_OK;
}

// Launches the next instance on `st`, after harvesting its previous replay.
int replay(gsr_ctx* ctx, GraphState* G, hipStream_t st) {
  const int ring = G->timed.empty() ? 1 : GraphState::kRing;
  GraphState::Instance& I = G->inst[G->next];
  G->next = (G->next + 1) % ring;
  if (!G->timed.empty()) RET_IF(harvest(ctx, I));
  HIP_TRY(ctx, hipGraphLaunch(I.exec, st));
  HIP_TRY(ctx, hipEventRecord(I.done, st));
  I.launched = !G->timed.empty();
  return GSR_OK;
}

int iteration_impl(gsr_ctx* ctx, float* params, int64_t num, int64_t stride, int32_t deg, int32_t nv,
                   const gsr_camera* cams, const gsr_image* out, const gsr_image* targets, float depth_weight,
                   float* grad, float* loss, const gsr_adam* adam, hipStream_t st) {
  gsr_gaussians g{params, num, stride, deg};
  RET_IF(check_gaussians(&g));
  RET_IF(check_cams(cams, nv));
  if (!out || !targets || (num > 0 && !grad)) return GSR_ERR_INVALID;
  for (int v = 0; v < nv; ++v)
    if (!out[v].rgb || !out[v].depth || !out[v].alpha || !targets[v].rgb || !targets[v].depth)
      return GSR_ERR_INVALID;
  const int planes = num_planes(deg);
  if (adam) {
    if (!adam->lr_per_plane || adam->step < 0 || (num > 0 && (!adam->m || !adam->v))) return GSR_ERR_INVALID;
    if (!(adam->beta1 >= 0.f && adam->beta1 < 1.f && adam->beta2 >= 0.f && adam->beta2 < 1.f))
      return GSR_ERR_INVALID;
  }
  if (!ctx->graph) {
    ctx->graph = new (std::nothrow) GraphState();
    if (!ctx->graph) return GSR_ERR_OOM;
    const int r = init_state(ctx, ctx->graph);
    if (r != GSR_OK) {
      destroy_graph(ctx);
      return r;
    }
  }
  GraphState* G = ctx->graph;
  ctx->last_stream = st;
  ctx->q_bufs = nullptr;
  ctx->q_plan = nullptr;

  // a finished replay that had to skip asks for a larger capacity
  if (G->captured) {
    const hipError_t q = hipEventQuery(G->done);
    if (q == hipSuccess) {
      if (G->host_stats[kStatSkipped] != G->seen_skipped) {
        G->seen_skipped = G->host_stats[kStatSkipped];
        if ((int64_t)G->host_stats[kStatMaxInstances] > G->capacity) G->grow = true;
      }
    } else {
      (void)hipGetLastError();
    }
  }

  std::vector<int32_t> sizes(2 * nv);
  for (int v = 0; v < nv; ++v) {
    sizes[2 * v] = cams[v].width;
    sizes[2 * v + 1] = cams[v].height;
  }
  const bool same = G->captured && !G->grow && G->params == params && G->grad == grad && G->loss == loss &&
                    G->num == num && G->stride == stride && G->deg == deg && G->sizes == sizes &&
                    G->depth_weight == depth_weight && G->adam == (adam != nullptr) &&
                    G->profile_mask == ctx->profile_mask &&
                    (!adam || (G->m == adam->m && G->v == adam->v && G->beta1 == adam->beta1 &&
                               G->beta2 == adam->beta2 && G->eps == adam->eps));

  RenderPlan plan;
  RET_IF(plan_render(ctx, &g, nv, cams, &plan));
  std::vector<ViewImages> outs(nv), tgts(nv);
  for (int v = 0; v < nv; ++v) {
    outs[v] = ViewImages{out[v].rgb, out[v].depth, out[v].alpha};
    tgts[v] = ViewImages{targets[v].rgb, targets[v].depth, nullptr};
  }

  if (!same) {
    HIP_TRY(ctx, hipStreamSynchronize(st));
    HIP_TRY(ctx, hipDeviceSynchronize());
    drop_graph(ctx, G);
    const int64_t old_cap = G->capacity;
    const bool layout_same = G->num == num && G->deg == deg && G->sizes == sizes && G->P.nv == nv;
    plan.capacity = layout_same ? old_cap : 0;
    G->P = plan;
    int64_t count = 0;
    RET_IF(measure_instances(ctx, G, params, out, &count, st));
    int64_t need = count;
    if (layout_same) {
      need = std::max<int64_t>(count, (int64_t)G->host_stats[kStatMaxInstances]);
    } else {
      const uint32_t zero = 0;
      RET_IF(upload(ctx, as<uint32_t>(G->stats) + kStatMaxInstances, &zero, sizeof(zero), st));
      G->host_stats[kStatMaxInstances] = 0;
    }
    int64_t cap = need + need / 4 + 4096;
    if (layout_same && !G->grow && old_cap >= need) cap = old_cap;
    G->P.capacity = cap;
    G->capacity = cap;
    G->grow = false;
    RET_IF(size_render(ctx, G->B, G->P, out, st));
    RET_IF(ensure(ctx, G->tdesc, sizeof(ViewImages) * nv));
    int64_t gpix = 0;
    for (int v = 0; v < nv; ++v) gpix += 4 * (int64_t)cams[v].width * cams[v].height;
    RET_IF(ensure(ctx, G->gimg, sizeof(float) * (size_t)gpix));
    std::vector<ViewImages> gims(nv);
    float* gp = as<float>(G->gimg);
    for (int v = 0; v < nv; ++v) {
      const int64_t hw = (int64_t)cams[v].width * cams[v].height;
      gims[v] = ViewImages{gp, gp + 3 * hw, nullptr};
      gp += 4 * hw;
    }
    RET_IF(upload(ctx, G->B.images2.p, gims.data(), sizeof(ViewImages) * nv, st));
    RET_IF(ensure(ctx, G->lrbuf, sizeof(float) * planes));
    RET_IF(upload_descriptors(ctx, G, nv, outs, tgts, adam ? adam->lr_per_plane : nullptr, planes, adam != nullptr,
                              true, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    G->params = params;
    G->grad = grad;
    G->loss = loss;
    G->num = num;
    G->stride = stride;
    G->deg = deg;
    G->sizes = sizes;
    G->depth_weight = depth_weight;
    G->adam = adam != nullptr;
    G->m = adam ? adam->m : nullptr;
    G->v = adam ? adam->v : nullptr;
    G->beta1 = adam ? adam->beta1 : 0.f;
    G->beta2 = adam ? adam->beta2 : 0.f;
    G->eps = adam ? adam->eps : 0.f;
    G->profile_mask = ctx->profile_mask;
    RET_IF(capture(ctx, G, params, grad, loss, adam, depth_weight, planes));
  } else {
    G->P.views = plan.views;
    RET_IF(upload_descriptors(ctx, G, nv, outs, tgts, adam ? adam->lr_per_plane : nullptr, planes, adam != nullptr,
                              false, st));
  }
  if (adam && adam->step > 0) {
    const uint32_t s0 = (uint32_t)(adam->step - 1);
    RET_IF(upload(ctx, as<uint32_t>(G->stats) + kStatAdamSteps, &s0, sizeof(s0), st));
  }
  RET_IF(replay(ctx, G, st));
  HIP_TRY(ctx, hipEventRecord(G->done, st));
  ctx->q_bufs = &G->B;
  ctx->q_plan = &G->P;
  ctx->q_params = params;
  return GSR_OK;
}

}  // namespace

int harvest_graph(gsr_ctx* ctx) {
  GraphState* G = ctx->graph;
  if (!G) return GSR_OK;
  for (GraphState::Instance& I : G->inst) RET_IF(harvest(ctx, I));
  return GSR_OK;
}

void destroy_graph(gsr_ctx* ctx) {
  GraphState* G = ctx->graph;
  if (!G) return;
  if (ctx->q_bufs == &G->B) {
    ctx->q_bufs = nullptr;
    ctx->q_plan = nullptr;
  }
  drop_graph(ctx, G);
  free_buffers(G->B);
  DevBuf* bufs[] = {&G->tdesc, &G->gimg, &G->lrbuf, &G->stats};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (G->host_stats) (void)hipHostFree(G->host_stats);
  if (G->done) (void)hipEventDestroy(G->done);
  if (G->cap) (void)hipStreamDestroy(G->cap);
  for (GraphState::Instance& I : G->inst)
    if (I.done) (void)hipEventDestroy(I.done);
  delete G;
  ctx->graph = nullptr;
}

}  // namespace gsr

extern "C" {

int gsr_mapping_iteration(gsr_ctx* ctx, float* params, int64_t num, int64_t stride, int32_t sh_degree,
                          int32_t num_views, const gsr_camera* cams, const gsr_image* out,
                          const gsr_image* targets, float depth_weight, float* grad_params, float* loss,
                          const gsr_adam* adam, void* stream) {
  if (!ctx) return GSR_ERR_INVALID;
  try {
    return gsr::iteration_impl(ctx, params, num, stride, sh_degree, num_views, cams, out, targets, depth_weight,
                               grad_params, loss, adam, (hipStream_t)stream);
  } catch (const std::bad_alloc&) {
    return GSR_ERR_OOM;
  } catch (...) {
    return GSR_ERR_INVALID;
  }
}

int gsr_mapping_status(gsr_ctx* ctx, gsr_mapping_stats* out) {
  if (!ctx || !out) return GSR_ERR_INVALID;
  std::memset(out, 0, sizeof(*out));
  gsr::GraphState* G = ctx->graph;
  if (!G) return GSR_OK;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  HIP_TRY(ctx, hipEventSynchronize(G->done));
  uint32_t s[gsr::kStatWords];
  HIP_TRY(ctx, hipMemcpy(s, G->stats.p, sizeof(s), hipMemcpyDeviceToHost));
  out->iterations = s[gsr::kStatIterations];
  out->skipped = s[gsr::kStatSkipped];
  out->captures = G->captures;
  out->capacity = G->capacity;
  out->last_instances = s[gsr::kStatLastInstances];
  out->adam_steps = s[gsr::kStatAdamSteps];
  return s[gsr::kStatErrors] ? GSR_ERR_DEVICE : GSR_OK;
}

}  // extern "C"
