// Sharing the live map with another process on the same GPU (gsr_ipc_*).
//
// The paper's viewer is a separate process that reads the GS map straight
// from GPU memory through inter-process handles, so that rendering for the
// operator never copies the map and never stalls the mapping loop (Sec. III,
// Fig. "CUDA_IPC"). These calls are the HIP form of that: a device buffer is
// exported as a handle plus its offset inside its allocation, the other
// process opens it, and an inter-process event orders the viewer's reads
// after the mapper's writes.

#include <cstring>

#include "context.h"

namespace {

static_assert(sizeof(hipIpcMemHandle_t) <= sizeof(gsr_ipc_handle), "memory handle fits");
static_assert(sizeof(hipIpcEventHandle_t) <= sizeof(gsr_ipc_handle), "event handle fits");

// Exported allocations stay well below the size whose opening has been seen
// not to return on some drivers.
constexpr size_t kMaxExportBytes = size_t(1) << 30;

// HIP error code of the last failed call of this file on the calling thread
// (these calls take no context to record it in)
thread_local int g_last_hip_error = 0;

int hip_status(hipError_t e) {
  if (e == hipSuccess) return GSR_OK;
  g_last_hip_error = (int)e;
  (void)hipGetLastError();
  return GSR_ERR_HIP;
}

}  // namespace

namespace gsr {
int ipc_last_hip_error() { return g_last_hip_error; }
}  // namespace gsr

extern "C" {

int gsr_ipc_export_memory(const void* dev_ptr, gsr_ipc_handle* out, int64_t* offset, int64_t* alloc_bytes) {
  if (!dev_ptr || !out || !offset) return GSR_ERR_INVALID;
  void* base = nullptr;
  size_t size = 0;
  RET_IF(hip_status(hipMemGetAddressRange(&base, &size, const_cast<void*>(dev_ptr))));
  if (!base || size == 0) return GSR_ERR_INVALID;
  if (size > kMaxExportBytes) return GSR_ERR_UNSUPPORTED;
  hipIpcMemHandle_t h;
  RET_IF(hip_status(hipIpcGetMemHandle(&h, base)));
  std::memset(out, 0, sizeof(*out));
  std::memcpy(out->bytes, &h, sizeof(h));
  *offset = (int64_t)(static_cast<const char*>(dev_ptr) - static_cast<const char*>(base));
  if (alloc_bytes) *alloc_bytes = (int64_t)size;
  return GSR_OK;
}

int gsr_ipc_open_memory(const gsr_ipc_handle* h, int64_t offset, void** dev_ptr, void** base_out) {
  if (!h || !dev_ptr || !base_out || offset < 0) return GSR_ERR_INVALID;
  hipIpcMemHandle_t mh;
  std::memcpy(&mh, h->bytes, sizeof(mh));
  void* base = nullptr;
  RET_IF(hip_status(hipIpcOpenMemHandle(&base, mh, hipIpcMemLazyEnablePeerAccess)));
  *base_out = base;
  *dev_ptr = static_cast<char*>(base) + offset;
  return GSR_OK;
}

int gsr_ipc_close_memory(void* base) {
  if (!base) return GSR_ERR_INVALID;
  return hip_status(hipIpcCloseMemHandle(base));
}

int gsr_ipc_event_create(void** event, gsr_ipc_handle* out) {
  if (!event || !out) return GSR_ERR_INVALID;
  hipEvent_t e = nullptr;
  RET_IF(hip_status(hipEventCreateWithFlags(&e, hipEventInterprocess | hipEventDisableTiming)));
  hipIpcEventHandle_t h;
  const int r = hip_status(hipIpcGetEventHandle(&h, e));
  if (r != GSR_OK) {
    (void)hipEventDestroy(e);
    return r;
  }
  std::memset(out, 0, sizeof(*out));
  std::memcpy(out->bytes, &h, sizeof(h));
  *event = e;
  return GSR_OK;
}

int gsr_ipc_event_open(const gsr_ipc_handle* h, void** event) {
  if (!h || !event) return GSR_ERR_INVALID;
  hipIpcEventHandle_t eh;
  std::memcpy(&eh, h->bytes, sizeof(eh));
  hipEvent_t e = nullptr;
  RET_IF(hip_status(hipIpcOpenEventHandle(&e, eh)));
  *event = e;
  return GSR_OK;
}

int gsr_ipc_event_record(void* event, void* stream) {
  if (!event) return GSR_ERR_INVALID;
  return hip_status(hipEventRecord((hipEvent_t)event, (hipStream_t)stream));
}

int gsr_ipc_event_wait(void* event, void* stream) {
  if (!event) return GSR_ERR_INVALID;
  return hip_status(hipStreamWaitEvent((hipStream_t)stream, (hipEvent_t)event, 0));
}

int gsr_ipc_event_destroy(void* event) {
  if (!event) return GSR_ERR_INVALID;
  return hip_status(hipEventDestroy((hipEvent_t)event));
}

}  // extern "C"
