// Scratch memory of the allocation-free exact counting call
// (mochy_count_exact_range_noalloc).
//
// A file-scope device array holds everything that call's kernels need beyond
// the graph, the context and the outputs (the work-item schedule, the
// light-pair lists of the correction).  Every device the library runs on
// holds its own copy from the first context created on it until the process
// ends.  In host code `scratch` names a host-side stand-in, never device
// memory: its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and only that address is
// handed to kernels.
#include <mutex>

#include "common.h"

namespace mochy_noalloc {
constexpr size_t kBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kBytes];
}  // namespace mochy_noalloc

const size_t kNoallocBytes = mochy_noalloc::kBytes;

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device
}  // namespace

mochy_status noalloc_setup(mochy_ctx* ctx) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (ctx->device < 0 || ctx->device >= kMaxDevices) {
    ctx->err = "device index beyond the allocation-free scratch table";
    return MOCHY_EINVAL;
  }
  if (!g_scratch[ctx->device]) {
    // mochy_ctx_create made ctx->device current before calling here
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(mochy_noalloc::scratch));
    if (e != hipSuccess || p == nullptr) {
      ctx->err = std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e);
      (void)hipGetLastError();
      return MOCHY_EDEVICE;
    }
    g_scratch[ctx->device] = p;
  }
  ctx->noalloc_scratch = g_scratch[ctx->device];
  return MOCHY_OK;
}
