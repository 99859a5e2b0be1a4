// hook.cpp -- automatic logging of allocations.  CRAC interposes on the
// cudaMalloc family so that every allocation and free is logged without the
// application's help (Sec. 3.1, "Log-and-replay"; Sec. 3.2, "Issue of
// library-allocated memory").  Here an allocator that calls out to a pair of
// C functions -- PyTorch's pluggable allocator, or a caller's own wrapper
// around hipMalloc -- gets them from this file, and each allocation is
// registered in the installed context as it is made and unregistered as it
// is freed, so the context's live set is exactly the active allocations.
#include <hip/hip_runtime.h>

#include <map>
#include <unordered_map>
#include <utility>
#include <vector>

#include "ckpt_runtime.h"

using namespace ckpt;

namespace {
ckpt_ctx *g_ctx = nullptr;   // guarded by hook_mutex()
uint32_t g_flags = 0;
uint64_t g_allocs = 0, g_frees = 0, g_failures = 0;

// The block cache (CKPT_HOOK_CACHE).  A freed block stays mapped, its
// registration dropped, and waits in a bin keyed by the stream it was
// allocated for and its size class; the next allocation of that class on
// that stream takes it and is registered with its own size.  Work queued on
// the stream before the free stays ordered before any use of the new
// allocation, as in a stream-ordered caching allocator.
struct Block {
    uint64_t cap = 0;        // bytes of the block (its size class)
    uintptr_t stream = 0;    // the stream it was first allocated for
    bool vmm = false;        // address-stable mapping of the context
    bool live = false;       // registered and handed out
    bool keep = true;        // cached when freed (false: a block of its request's size, released)
};
std::unordered_map<uint64_t, Block> g_blocks;                            // every cache block
std::map<std::pair<uintptr_t, uint64_t>, std::vector<uint64_t>> g_bins;   // free ones
uint64_t g_cached_blocks = 0, g_cached_bytes = 0, g_hits = 0;
uint64_t g_gran = 0;   // mapping granularity of the installed context (address-stable cache)

// Classes of four per power of two (at most 25% over the request), at least
// 512 bytes, rounded up to `gran` when it is not 0.  0 when b is too large.
uint64_t size_class(uint64_t b, uint64_t gran)
{
    if (b > (uint64_t(1) << 62))
        return 0;
    uint64_t c = 512;
    if (b > 512) {
        const int e = 63 - __builtin_clzll(b - 1);   // 2^e < b <= 2^(e+1)
        const uint64_t step = uint64_t(1) << (e - 2);
        c = (b + step - 1) / step * step;
    }
    if (gran)
        c = (c + gran - 1) / gran * gran;
    return c;
}

// Releases every free block; the caller holds hook_mutex() and g_ctx is set.
uint64_t trim_locked()
{
    if (!g_cached_blocks)
        return 0;
    DeviceGuard dg(g_ctx->cfg.device);
    // free blocks may still be read or written by work queued before their free
    (void)hipDeviceSynchronize();
    uint64_t n = 0;
    for (auto &kv : g_bins)
        for (uint64_t p : kv.second) {
            auto it = g_blocks.find(p);
            if (it == g_blocks.end())
                continue;
            n += it->second.cap;
            if (it->second.vmm)
                vmm_block_unmap(g_ctx, p);
            else
                (void)hipFree((void *)(uintptr_t)p);
            g_blocks.erase(it);
        }
    g_bins.clear();
    g_cached_blocks = g_cached_bytes = 0;
    return n;
}

// Frees the cached blocks and forgets the live ones (freed later by the
// uncached path) when the installed context changes.
void cache_reset_locked()
{
    if (g_ctx)
        trim_locked();
    g_blocks.clear();
    g_bins.clear();
    g_cached_blocks = g_cached_bytes = g_hits = 0;
}

int new_block(uint64_t cap, bool vmm, uint64_t *p)
{
    if (vmm)
        return vmm_block_map(g_ctx, cap, p);
    DeviceGuard dg(g_ctx->cfg.device);
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, cap);
    if (e != hipSuccess)
        return set_error(CKPT_E_NOMEM, "hipMalloc of %llu bytes: %s", (unsigned long long)cap, hipGetErrorString(e));
    *p = (uint64_t)(uintptr_t)q;
    return CKPT_OK;
}

void *cache_malloc(size_t bytes, void *stream)
{
    const bool vmm = g_flags & CKPT_HOOK_ADDRESS_STABLE;
    const uint64_t cap = size_class(bytes, vmm ? g_gran : 0);
    if (!cap)
        return nullptr;
    const auto key = std::make_pair((uintptr_t)stream, cap);
    uint64_t p = 0;
    auto bin = g_bins.find(key);
    while (!p && bin != g_bins.end() && !bin->second.empty()) {
        const uint64_t q = bin->second.back();
        bin->second.pop_back();
        g_cached_blocks--;
        g_cached_bytes -= cap;
        // a mapping released behind the cache's back is not handed out again
        if (vmm && !g_ctx->vmm.count(q)) {
            g_blocks.erase(q);
            continue;
        }
        p = q;
        g_hits++;
    }
    if (!p) {
        Block b;
        b.cap = cap;
        b.stream = (uintptr_t)stream;
        b.vmm = vmm;
        int rc = new_block(cap, vmm, &p);
        if (rc != CKPT_OK && g_cached_blocks) {
            trim_locked();   // out of memory: give the cached blocks back and try once more
            rc = new_block(cap, vmm, &p);
        }
        if (rc != CKPT_OK) {
            // the class rounds up by as much as a quarter: a request that fits
            // only at its own size gets a block of that size, released when freed
            const uint64_t unit = vmm ? g_gran : uint64_t(2) << 20;
            const uint64_t exact = (bytes + unit - 1) / unit * unit;
            if (exact >= cap || new_block(exact, vmm, &p) != CKPT_OK)
                return nullptr;
            b.cap = exact;
            b.keep = false;
        }
        g_blocks[p] = b;
    }
    uint64_t id = 0;
    if (add_registration(g_ctx, p, bytes, CKPT_DEVICE, 0, &id) != CKPT_OK) {
        g_bins[key].push_back(p);
        g_cached_blocks++;
        g_cached_bytes += cap;
        return nullptr;
    }
    if (vmm)
        g_ctx->vmm_of[p] = p;
    g_blocks[p].live = true;
    return (void *)(uintptr_t)p;
}

// true when ptr was a live cache block (now back in its bin)
bool cache_free(uint64_t p)
{
    auto it = g_blocks.find(p);
    if (it == g_blocks.end() || !it->second.live)
        return false;
    Block &b = it->second;
    (void)drop_registration(g_ctx, p);
    if (b.vmm) {
        g_ctx->vmm_of.erase(p);
        if (!g_ctx->vmm.count(p)) {   // released elsewhere: nothing to keep
            g_blocks.erase(it);
            return true;
        }
    }
    if (!b.keep) {
        // not a class size: released at once (after the device's queued work)
        DeviceGuard dg(g_ctx->cfg.device);
        (void)hipDeviceSynchronize();
        if (b.vmm)
            vmm_block_unmap(g_ctx, p);
        else
            (void)hipFree((void *)(uintptr_t)p);
        g_blocks.erase(it);
        return true;
    }
    b.live = false;
    g_bins[std::make_pair(b.stream, b.cap)].push_back(p);
    g_cached_blocks++;
    g_cached_bytes += b.cap;
    return true;
}
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
    if (g_ctx == ctx) {
        cache_reset_locked();
        g_ctx = nullptr;
    }
    ctx->hooked = false;
}

void ckpt::hook_trim_for(ckpt_ctx *ctx)
{
    if (!ctx->hooked.load())
        return;
    std::lock_guard<std::recursive_mutex> lk(hook_mutex());
    if (g_ctx == ctx)
        trim_locked();
}

extern "C" int ckpt_hook_install(ckpt_ctx *ctx, uint32_t flags)
{
    if (flags & ~(uint32_t)(CKPT_HOOK_ADDRESS_STABLE | CKPT_HOOK_CACHE))
        return set_error(CKPT_E_INVAL, "unknown hook flags 0x%x", flags);
    std::lock_guard<std::recursive_mutex> lk(hook_mutex());
    uint64_t gran = 0;
    if (ctx && (flags & CKPT_HOOK_CACHE) && (flags & CKPT_HOOK_ADDRESS_STABLE)) {
        size_t g = 0;
        CKPT_TRY(ckpt_vmm_granularity(ctx, &g));
        gran = g;
    }
    cache_reset_locked();
    if (g_ctx)
        g_ctx->hooked = false;
    g_ctx = ctx;
    g_flags = flags;
    g_gran = gran;
    g_allocs = g_frees = g_failures = 0;
    if (ctx)
        ctx->hooked = true;
    return CKPT_OK;
}

extern "C" void *ckpt_hook_malloc(size_t bytes, int device, void *stream)
{
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
    if (g_flags & CKPT_HOOK_CACHE) {
        p = cache_malloc(bytes, stream);
        if (!p) {
            g_failures++;
            return nullptr;
        }
    } else if (g_flags & CKPT_HOOK_ADDRESS_STABLE) {
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
    const uint64_t a = (uint64_t)(uintptr_t)ptr;
    if (g_ctx && cache_free(a)) {
        g_frees++;
        return;
    }
    if (g_ctx && g_ctx->vmm_of.count(a)) {
        if (ckpt_vmm_free(g_ctx, ptr) == CKPT_OK)
            g_frees++;
        return;
    }
    if (g_ctx && device == g_ctx->cfg.device && drop_registration(g_ctx, a) == CKPT_OK)
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

extern "C" int ckpt_hook_cache_stats(uint64_t *blocks, uint64_t *bytes, uint64_t *hits)
{
    if (!blocks || !bytes || !hits)
        return set_error(CKPT_E_INVAL, "NULL argument");
    std::lock_guard<std::recursive_mutex> lk(hook_mutex());
    *blocks = g_cached_blocks;
    *bytes = g_cached_bytes;
    *hits = g_hits;
    return CKPT_OK;
}

extern "C" int ckpt_hook_trim(uint64_t *released)
{
    std::lock_guard<std::recursive_mutex> lk(hook_mutex());
    const uint64_t n = g_ctx ? trim_locked() : 0;
    if (released)
        *released = n;
    return CKPT_OK;
}
