// Device memory of the library: through the caller's allocator hook when one
// is set (cr_set_allocator), else hipMalloc / hipFree.  Each block remembers
// the hook that allocated it and is returned through that hook.
#pragma once
#include <cstddef>

#include "../../include/crfrob.h"

namespace crf {

struct DevBlock {
    void *ptr = nullptr;
    size_t bytes = 0;
    cr_free_fn free_fn = nullptr;  // null: the block came from hipMalloc
    void *ctx = nullptr;
};

// Allocates `bytes` on the current device into b (b must be empty); false on
// failure or when a hook returns memory that is not 256-byte aligned.
bool dev_alloc(DevBlock &b, size_t bytes);
// Waits for the device before a hook's free (hipFree waits by itself), then
// returns the block; leaves b empty.
void dev_free(DevBlock &b);
// Installs the hooks (both null: back to hipMalloc); CR_EINVAL if only one is set.
cr_status set_allocator(cr_alloc_fn alloc, cr_free_fn free_fn, void *ctx);

}  // namespace crf
