// Allocation-free forward: hdc_forward with the workspace taken from a
// file-scope device array instead of a caller-provided buffer, for callers
// that cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The array `scratch` lives in the library's code object: every GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  Host code may not use the array's name as a device address; the
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and that pointer is what the kernels receive.  Every call on
// one GPU shares that GPU's array, so calls that overlap on one GPU (several
// streams or threads at once) race; the kernels write every workspace element
// they read, so nothing needs clearing between calls.
#include <mutex>

#include "../../include/hdconv.h"
#include "hdc_kernels.hpp"

// reports an error through hdc_last_error (defined with the other entry points)
extern "C" __attribute__((visibility("hidden"))) hdc_status hdc_internal_fail(hdc_status st, const char* msg);

static constexpr size_t kScratchBytes = HDC_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// the current device's copy of `scratch` (looked up on the first call on that device)
hdc_status scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hdc_internal_fail(HDC_ERR_HIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return hdc_internal_fail(HDC_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return hdc_internal_fail(HDC_ERR_HIP, e != hipSuccess ? hipGetErrorString(e) : "scratch address is NULL");
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return HDC_OK;
}

}  // namespace

extern "C" {

hdc_status hdc_forward_noalloc(hdc_plan p, const void* f, const void* g, void* h, void* stream) {
  if (!p) return hdc_internal_fail(HDC_ERR_INVALID_ARG, "NULL plan");
  size_t need = 0;
  hdc_status st = hdc_plan_workspace_size(p, &need);
  if (st != HDC_OK) return st;
  if (need > kScratchBytes) {
    char msg[192];
    snprintf(msg, sizeof(msg),
             "the plan needs %zu bytes of workspace; the allocation-free forward holds %zu (use hdc_forward with a "
             "caller workspace)", need, kScratchBytes);
    return hdc_internal_fail(HDC_ERR_WORKSPACE, msg);
  }
  void* ws = nullptr;
  if (need) {
    st = scratch_ptr(&ws);
    if (st != HDC_OK) return st;
  }
  return hdc_forward(p, f, g, h, ws, need ? kScratchBytes : 0, stream);
}

}  // extern "C"
