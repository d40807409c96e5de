// Device allocation through the caller's hook or hipMalloc.
#include "devmem.hpp"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

namespace crf {

namespace {
std::mutex g_hook_mutex;
cr_alloc_fn g_alloc = nullptr;
cr_free_fn g_free = nullptr;
void *g_ctx = nullptr;
}  // namespace

bool dev_alloc(DevBlock &b, size_t bytes) {
    b = DevBlock{};
    if (bytes == 0) bytes = 256;
    cr_alloc_fn a;
    cr_free_fn f;
    void *ctx;
    {
        std::lock_guard<std::mutex> lk(g_hook_mutex);
        a = g_alloc;
        f = g_free;
        ctx = g_ctx;
    }
    if (!a) {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return false;
        b.ptr = p;
        b.bytes = bytes;
        return true;
    }
    void *p = a(bytes, ctx);
    if (!p) return false;
    if (reinterpret_cast<uintptr_t>(p) % 256 != 0) {
        f(p, ctx);
        return false;
    }
    b.ptr = p;
    b.bytes = bytes;
    b.free_fn = f;
    b.ctx = ctx;
    return true;
}

void dev_free(DevBlock &b) {
    if (b.ptr) {
        if (b.free_fn) {
            // the hook may hand the block out again at once: no kernel or copy
            // of the library may still use it
            (void)hipDeviceSynchronize();
            b.free_fn(b.ptr, b.ctx);
        } else {
            (void)hipFree(b.ptr);
        }
    }
    b = DevBlock{};
}

cr_status set_allocator(cr_alloc_fn alloc, cr_free_fn free_fn, void *ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr)) return CR_EINVAL;
    std::lock_guard<std::mutex> lk(g_hook_mutex);
    g_alloc = alloc;
    g_free = free_fn;
    g_ctx = alloc ? ctx : nullptr;
    return CR_OK;
}

}  // namespace crf
