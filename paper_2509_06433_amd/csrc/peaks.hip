// Achievable-peak probes of the device: the denominators of the roofline
// fractions the benchmark reports, measured on the GPU it runs on rather
// than taken from the data sheet. None of this is on the rendering path.
//
//   copy  device-to-device copy with 16-byte loads and stores: HBM bytes
//         (read + write) per second
//   valu  independent FP32 fused multiply-add chains, one instruction per
//         lane per step (no packed FP32 math): VALU lane operations per second
//   exp   independent chains of the hardware 2^x: its lane rate
//   lds   conflict-free 16-byte LDS reads: LDS bytes per second
//
// Each probe runs its kernel once to warm up, then `reps` times between two
// HIP events on the given stream, and reports the average.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsr_peaks.h"

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                      int64_t n4) {
  // four 16-byte items per thread, loads issued before the stores
  const int64_t base = ((int64_t)blockIdx.x * kBlock) * 4 + threadIdx.x;
  float4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + (int64_t)k * kBlock;
    v[k] = i < n4 ? src[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + (int64_t)k * kBlock;
    if (i < n4) dst[i] = v[k];
  }
}

constexpr int kChains = 8;
constexpr int kSteps = 2048;

__global__ void __launch_bounds__(kBlock) valu_kernel(float x, float y, float* __restrict__ sink) {
  float a[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) a[c] = (float)(threadIdx.x + c);
  for (int s = 0; s < kSteps; ++s) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = __builtin_fmaf(a[c], x, y);
  }
  float t = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) t += a[c];
  if (t == 1.2345f) sink[threadIdx.x] = t;      // keeps the chains live; never true for the inputs used
}

__global__ void __launch_bounds__(kBlock) exp_kernel(float* __restrict__ sink) {
  float a[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) a[c] = -(float)(threadIdx.x & 7) * 0.125f - 0.01f * c;
  for (int s = 0; s < kSteps; ++s) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = -__builtin_amdgcn_exp2f(a[c]);   // stays in (-1, 0)
  }
  float t = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) t += a[c];
  if (t == 1.2345f) sink[threadIdx.x] = t;
}

constexpr int kLdsWords4 = 4096;      // 64 KiB of 16-byte words per workgroup
constexpr int kLdsRounds = 64;        // each round reads the whole buffer once (16 reads per thread)

__global__ void __launch_bounds__(kBlock) lds_kernel(uint32_t seed, float* __restrict__ sink) {
  __shared__ uint4 buf[kLdsWords4];
  for (int i = threadIdx.x; i < kLdsWords4; i += kBlock) buf[i] = make_uint4(i, seed, i ^ seed, 3u);
  __syncthreads();
  // consecutive lanes read consecutive 16-byte words (no bank conflict) at
  // fixed offsets; two three-input integer adds consume each 16-byte read, so
  // the VALU stays below the LDS's rate
  uint32_t a0 = 0u, a1 = 0u;
  for (int r = 0; r < kLdsRounds; ++r) {
#pragma unroll
    for (int j = 0; j < kLdsWords4 / kBlock; ++j) {
      const uint4 v = buf[threadIdx.x + j * kBlock];
      a0 = a0 + v.x + v.y;
      a1 = a1 + v.z + v.w;
    }
    __syncthreads();                       // a fence: every round reads the buffer again
  }
  if ((a0 ^ a1) == 0x9e3779b9u) sink[threadIdx.x] = (float)a0;
}

int device_cus(int* cus) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GSR_PEAKS_ERR_HIP;
  if (hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return GSR_PEAKS_ERR_HIP;
  return 0;
}

// Times `reps` launches of `launch` (after one warm-up) on `st`: ms per launch.
template <class F>
int time_launches(F launch, int reps, hipStream_t st, double* ms_per) {
  hipEvent_t a = nullptr, b = nullptr;
  int rc = 0;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = GSR_PEAKS_ERR_HIP;
  if (!rc) {
    launch();
    if (hipGetLastError() != hipSuccess || hipEventRecord(a, st) != hipSuccess) rc = GSR_PEAKS_ERR_HIP;
  }
  if (!rc) {
    for (int r = 0; r < reps; ++r) launch();
    float ms = 0.f;
    if (hipGetLastError() != hipSuccess || hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess)
      rc = GSR_PEAKS_ERR_HIP;
    *ms_per = (double)ms / reps;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return rc;
}

}  // namespace

extern "C" {

int gsr_peak_copy(int64_t bytes, int32_t reps, void* stream, double* bytes_per_s) {
  if (bytes < (1 << 20) || bytes > (int64_t(1) << 36) || reps < 1 || !bytes_per_s) return GSR_PEAKS_ERR_INVALID;
  const int64_t n4 = bytes / 16;
  hipStream_t st = (hipStream_t)stream;
  void *src = nullptr, *dst = nullptr;
  if (hipMalloc(&src, n4 * 16) != hipSuccess || hipMalloc(&dst, n4 * 16) != hipSuccess) {
    (void)hipGetLastError();
    if (src) (void)hipFree(src);
    return GSR_PEAKS_ERR_OOM;
  }
  int rc = hipMemsetAsync(src, 0, n4 * 16, st) == hipSuccess ? 0 : GSR_PEAKS_ERR_HIP;
  const int64_t blocks = (n4 + 4 * kBlock - 1) / (4 * kBlock);
  double ms = 0.0;
  if (!rc)
    rc = time_launches([&] { copy_kernel<<<(unsigned)blocks, kBlock, 0, st>>>((const float4*)src, (float4*)dst, n4); },
                       reps, st, &ms);
  if (!rc) *bytes_per_s = 2.0 * (double)(n4 * 16) / (ms * 1e-3);
  (void)hipFree(src);
  (void)hipFree(dst);
  return rc;
}

// Workgroups per CU for the compute probes: eight waves of 64 per SIMD.
static int64_t compute_blocks(int cus) { return (int64_t)cus * 8; }

int gsr_peak_valu(int32_t reps, void* stream, double* lane_ops_per_s) {
  if (reps < 1 || !lane_ops_per_s) return GSR_PEAKS_ERR_INVALID;
  int cus = 0;
  if (device_cus(&cus)) return GSR_PEAKS_ERR_HIP;
  hipStream_t st = (hipStream_t)stream;
  float* sink = nullptr;
  if (hipMalloc(&sink, kBlock * sizeof(float)) != hipSuccess) return GSR_PEAKS_ERR_OOM;
  const int64_t blocks = compute_blocks(cus);
  double ms = 0.0;
  const int rc = time_launches([&] { valu_kernel<<<(unsigned)blocks, kBlock, 0, st>>>(0.999f, 0.001f, sink); },
                               reps, st, &ms);
  if (!rc) *lane_ops_per_s = (double)blocks * kBlock * kSteps * kChains / (ms * 1e-3);
  (void)hipFree(sink);
  return rc;
}

int gsr_peak_exp(int32_t reps, void* stream, double* lane_ops_per_s) {
  if (reps < 1 || !lane_ops_per_s) return GSR_PEAKS_ERR_INVALID;
  int cus = 0;
  if (device_cus(&cus)) return GSR_PEAKS_ERR_HIP;
  hipStream_t st = (hipStream_t)stream;
  float* sink = nullptr;
  if (hipMalloc(&sink, kBlock * sizeof(float)) != hipSuccess) return GSR_PEAKS_ERR_OOM;
  const int64_t blocks = compute_blocks(cus);
  double ms = 0.0;
  const int rc = time_launches([&] { exp_kernel<<<(unsigned)blocks, kBlock, 0, st>>>(sink); }, reps, st, &ms);
  // each step is one 2^x and one negation per chain: the 2^x lane rate
  if (!rc) *lane_ops_per_s = (double)blocks * kBlock * kSteps * kChains / (ms * 1e-3);
  (void)hipFree(sink);
  return rc;
}

int gsr_peak_lds(int32_t reps, void* stream, double* bytes_per_s) {
  if (reps < 1 || !bytes_per_s) return GSR_PEAKS_ERR_INVALID;
  int cus = 0;
  if (device_cus(&cus)) return GSR_PEAKS_ERR_HIP;
  hipStream_t st = (hipStream_t)stream;
  float* sink = nullptr;
  if (hipMalloc(&sink, kBlock * sizeof(float)) != hipSuccess) return GSR_PEAKS_ERR_OOM;
  // 64 KiB of LDS per workgroup: two workgroups per CU
  const int64_t blocks = (int64_t)cus * 2 * 4;
  double ms = 0.0;
  const int rc = time_launches([&] { lds_kernel<<<(unsigned)blocks, kBlock, 0, st>>>(7u, sink); }, reps, st, &ms);
  if (!rc) *bytes_per_s = (double)blocks * kBlock * kLdsRounds * (kLdsWords4 / kBlock) * 16.0 / (ms * 1e-3);
  (void)hipFree(sink);
  return rc;
}

}  // extern "C"
