// hook.cpp -- automatic logging of allocations.  CRAC interposes on the
// cudaMalloc family so that every allocation and free is logged without the
// application's help (Sec. 3.1, "Log-and-replay"; Sec. 3.2, "Issue of
// library-allocated memory").  Here an allocator that calls out to a pair of
// C functions -- PyTorch's pluggable allocator, or a caller's own wrapper
// around hipMalloc -- gets them from this file, and each allocation is
// registered in the installed context as it is made and unregistered as it
// is freed, so the context's live set is exactly the active allocations.
#include <hip/hip_runtime.h>

#include "ckpt_runtime.h"

using namespace ckpt;

namespace {
ckpt_ctx *g_ctx = nullptr;   // guarded by hook_mutex()
uint32_t g_flags = 0;
uint64_t g_allocs = 0, g_frees = 0, g_failures = 0;
}  // namespace

std::recursive_mutex &ckpt::hook_mutex()
{
    static std::recursive_mutex *m = new std::recursive_mutex();   // outlives static destruction
    return *m;
}

void ckpt::hook_forget(ckpt_ctx *ctx)
{
    if (!ctx->hooked.load())
        return;
    std::lock_guard<std::recursive_mutex> lk(hook_mutex());
    if (g_ctx == ctx)
        g_ctx = nullptr;
    ctx->hooked = false;
}

extern "C" int ckpt_hook_install(ckpt_ctx *ctx, uint32_t flags)
{
    if (flags & ~(uint32_t)CKPT_HOOK_ADDRESS_STABLE)
        return set_error(CKPT_E_INVAL, "unknown hook flags 0x%x", flags);
    std::lock_guard<std::recursive_mutex> lk(hook_mutex());
    if (g_ctx)
        g_ctx->hooked = false;
    g_ctx = ctx;
    g_flags = flags;
    g_allocs = g_frees = g_failures = 0;
    if (ctx)
        ctx->hooked = true;
    return CKPT_OK;
}

extern "C" void *ckpt_hook_malloc(size_t bytes, int device, void *stream)
{
    (void)stream;
    if (bytes == 0)
        return nullptr;
    std::lock_guard<std::recursive_mutex> lk(hook_mutex());
    void *p = nullptr;
    if (!g_ctx || device != g_ctx->cfg.device) {
        // nothing logs this device's allocations: plain memory, not registered
        DeviceGuard dg(device);
        return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
    }
    ckpt_id id = 0;
    if (g_flags & CKPT_HOOK_ADDRESS_STABLE) {
        if (ckpt_vmm_alloc(g_ctx, bytes, nullptr, &p, &id) != CKPT_OK) {
            g_failures++;
            return nullptr;
        }
    } else {
        DeviceGuard dg(device);
        if (hipMalloc(&p, bytes) != hipSuccess) {
            g_failures++;
            return nullptr;
        }
        if (ckpt_register(g_ctx, p, bytes, CKPT_DEVICE, &id) != CKPT_OK) {
            (void)hipFree(p);
            g_failures++;
            return nullptr;
        }
    }
    g_allocs++;
    return p;
}

extern "C" void ckpt_hook_free(void *ptr, size_t bytes, int device, void *stream)
{
    (void)bytes;
    (void)stream;
    if (!ptr)
        return;
    std::lock_guard<std::recursive_mutex> lk(hook_mutex());
    if (g_ctx && g_ctx->vmm_of.count((uint64_t)(uintptr_t)ptr)) {
        if (ckpt_vmm_free(g_ctx, ptr) == CKPT_OK)
            g_frees++;
        return;
    }
    if (g_ctx && device == g_ctx->cfg.device && drop_registration(g_ctx, (uint64_t)(uintptr_t)ptr) == CKPT_OK)
        g_frees++;
    DeviceGuard dg(device);
    (void)hipFree(ptr);   // waits for the device's queued work first
}

extern "C" int ckpt_hook_stats(uint64_t *allocs, uint64_t *frees, uint64_t *failures)
{
    if (!allocs || !frees || !failures)
        return set_error(CKPT_E_INVAL, "NULL argument");
    std::lock_guard<std::recursive_mutex> lk(hook_mutex());
    *allocs = g_allocs;
    *frees = g_frees;
    *failures = g_failures;
    return CKPT_OK;
}
