// Static device workspace of cr_frobenius_batch_noalloc: a fixed array in the
// library's code object, so that the entry point never calls hipMalloc.  Each
// device that loads the library holds its own copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

namespace {

constexpr size_t kScratchBytes = 128ull << 20;  // CR_NOALLOC_WORKSPACE_BYTES
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_ws_mutex;
void *g_ws_ptr[kMaxDevices] = {};

}  // namespace

namespace crf {

// Device address of the current device's copy of `scratch` (looked up once per
// device with that device current; the host-side name is only a stand-in).
hipError_t static_workspace(void **ptr, size_t *bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_ws_mutex);
    if (!g_ws_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255) != 0) return hipErrorInvalidSymbol;
        g_ws_ptr[dev] = p;
    }
    *ptr = g_ws_ptr[dev];
    *bytes = kScratchBytes;
    return hipSuccess;
}

}  // namespace crf
