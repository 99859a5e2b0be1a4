// vmm.cpp -- address-stable device memory and restore at the original
// addresses (Sec. 3.1 and Sec. 3.2, "restoring the CUDA library-allocated
// regions"): HIP virtual memory management reserves a virtual range at a
// requested address and maps physical device memory into it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "ckpt_runtime.h"

using namespace ckpt;

namespace {

hipMemAllocationProp device_prop(int device)
{
    hipMemAllocationProp prop;
    memset(&prop, 0, sizeof(prop));
    prop.type = hipMemAllocationTypePinned;
    prop.location.type = hipMemLocationTypeDevice;
    prop.location.id = device;
    return prop;
}

int granularity(int device, uint64_t *out)
{
    hipMemAllocationProp prop = device_prop(device);
    size_t g = 0;
    HIP_TRY(hipMemGetAllocationGranularity(&g, &prop, hipMemAllocationGranularityMinimum));
    if (g == 0 || (g & (g - 1)) != 0)
        return set_error(CKPT_E_HIP, "allocation granularity %zu is not a power of two", g);
    *out = g;
    return CKPT_OK;
}

// Windows: the first address-stable allocation without a requested address
// picks a region of kWindowUsable + kWindowGuard bytes (by reserving it and
// releasing it again at once), and allocations are then placed from its
// bottom up, each with its own reservation at the chosen address.  The runtime
// hands out its own addresses top-down, and in another process its first
// allocations may land somewhat lower or higher than in this one; the bottom
// of the region sits far below all of them, so the same addresses are free
// again in a fresh process.  The runtime may still place memory of its own in
// the region later: such a spot is marked taken and the next one is tried.
constexpr uint64_t kWindowUsable = uint64_t(1) << 40;   // 1 TiB
constexpr uint64_t kWindowGuard = uint64_t(1) << 38;    // 256 GiB
constexpr int kPlaceTries = 8;

// Take [a, a + n) out of a window's free list when it lies in one free range.
bool window_take(VmmWindow &w, uint64_t a, uint64_t n)
{
    auto it = w.free.upper_bound(a);
    if (it == w.free.begin())
        return false;
    --it;
    const uint64_t s = it->first, e = s + it->second;
    if (a < s || a + n > e)
        return false;
    w.free.erase(it);
    if (s < a)
        w.free.emplace(s, a - s);
    if (a + n < e)
        w.free.emplace(a + n, e - (a + n));
    return true;
}

void window_give(VmmWindow &w, uint64_t a, uint64_t n)
{
    auto it = w.free.emplace(a, n).first;
    auto nx = std::next(it);
    if (nx != w.free.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        w.free.erase(nx);
    }
    if (it != w.free.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            w.free.erase(it);
        }
    }
}

VmmWindow *window_of(ckpt_ctx *ctx, uint64_t a, uint64_t n)
{
    for (VmmWindow &w : ctx->windows)
        if (a < w.base + w.usable && w.base < a + n)
            return &w;
    return nullptr;
}

// hipMemAddressReserve exactly at `want`: CKPT_E_ADDR when the runtime would
// put the range elsewhere.
int reserve_exact(uint64_t want, uint64_t bytes)
{
    void *p = nullptr;
    hipError_t e = hipMemAddressReserve(&p, bytes, 0, (void *)(uintptr_t)want, 0);
    if (e != hipSuccess)
        return set_error(CKPT_E_ADDR, "cannot reserve [0x%llx, +%llu): %s", (unsigned long long)want,
                         (unsigned long long)bytes, hipGetErrorString(e));
    if ((uint64_t)(uintptr_t)p != want) {
        (void)hipMemAddressFree(p, bytes);
        return set_error(CKPT_E_ADDR, "[0x%llx, +%llu) is not free (the runtime offered %p)",
                         (unsigned long long)want, (unsigned long long)bytes, p);
    }
    return CKPT_OK;
}

// A reservation of `bytes`: at `want`, or (want 0) at the lowest free spot of
// a window.  *in_window: the addresses are also booked in a window.
int reserve_va(ckpt_ctx *ctx, uint64_t want, uint64_t bytes, uint64_t *base, bool *in_window)
{
    if (want) {
        VmmWindow *w = window_of(ctx, want, bytes);
        if (w && !window_take(*w, want, bytes))
            return set_error(CKPT_E_ADDR, "[0x%llx, +%llu) is taken", (unsigned long long)want,
                             (unsigned long long)bytes);
        const int rc = reserve_exact(want, bytes);
        if (rc != CKPT_OK) {
            if (w)
                window_give(*w, want, bytes);
            return rc;
        }
        *base = want;
        *in_window = w != nullptr;
        return CKPT_OK;
    }
    if (ctx->windows.empty()) {
        VmmWindow w;
        w.usable = kWindowUsable;
        void *p = nullptr;
        HIP_TRY(hipMemAddressReserve(&p, kWindowUsable + kWindowGuard, 0, nullptr, 0));
        (void)hipMemAddressFree(p, kWindowUsable + kWindowGuard);
        w.base = (uint64_t)(uintptr_t)p;
        w.free.emplace(w.base, w.usable);
        ctx->windows.push_back(w);
    }
    VmmWindow &w = ctx->windows.front();
    for (int t = 0; t < kPlaceTries; t++) {
        uint64_t a = 0;
        for (const auto &f : w.free)
            if (f.second >= bytes) {
                a = f.first;
                break;
            }
        if (!a)
            break;
        window_take(w, a, bytes);
        if (reserve_exact(a, bytes) == CKPT_OK) {
            *base = a;
            *in_window = true;
            return CKPT_OK;
        }
        // the runtime holds memory there now: leave the spot booked as taken
    }
    // the window is full or crowded: anywhere the runtime chooses
    void *p = nullptr;
    HIP_TRY(hipMemAddressReserve(&p, bytes, 0, nullptr, 0));
    *base = (uint64_t)(uintptr_t)p;
    *in_window = false;
    return CKPT_OK;
}

void release_va(ckpt_ctx *ctx, uint64_t base, uint64_t bytes, bool in_window)
{
    (void)hipMemAddressFree((void *)(uintptr_t)base, bytes);
    if (in_window)
        if (VmmWindow *w = window_of(ctx, base, bytes))
            window_give(*w, base, bytes);
}

// Virtual addresses for [want, want + bytes) (anywhere when want is 0), fresh
// device memory mapped there, readable and writable from the device.  Nothing
// is left behind on failure.
int map_range(ckpt_ctx *ctx, uint64_t want, uint64_t bytes, uint64_t *base)
{
    const int dev = ctx->cfg.device;
    uint64_t va = 0;
    bool in_window = false;
    CKPT_TRY(reserve_va(ctx, want, bytes, &va, &in_window));
    void *p = (void *)(uintptr_t)va;
    hipMemAllocationProp prop = device_prop(dev);
    hipMemGenericAllocationHandle_t h{};
    hipError_t e = hipMemCreate(&h, bytes, &prop, 0);
    if (e != hipSuccess) {
        release_va(ctx, va, bytes, in_window);
        return set_error(CKPT_E_NOMEM, "hipMemCreate of %llu bytes: %s", (unsigned long long)bytes,
                         hipGetErrorString(e));
    }
    e = hipMemMap(p, bytes, 0, h, 0);
    if (e == hipSuccess) {
        hipMemAccessDesc acc;
        memset(&acc, 0, sizeof(acc));
        acc.location.type = hipMemLocationTypeDevice;
        acc.location.id = dev;
        acc.flags = hipMemAccessFlagsProtReadWrite;
        e = hipMemSetAccess(p, bytes, &acc, 1);
        if (e != hipSuccess)
            (void)hipMemUnmap(p, bytes);
    }
    if (e != hipSuccess) {
        (void)hipMemRelease(h);
        release_va(ctx, va, bytes, in_window);
        return hip_fail(e, "hipMemMap / hipMemSetAccess", __LINE__);
    }
    VmmRange r;
    r.bytes = bytes;
    r.h = h;
    r.in_window = in_window;
    ctx->vmm.emplace(va, r);
    *base = va;
    return CKPT_OK;
}

void unmap_range(ckpt_ctx *ctx, std::map<uint64_t, VmmRange>::iterator it)
{
    void *p = (void *)(uintptr_t)it->first;
    (void)hipMemUnmap(p, it->second.bytes);
    (void)hipMemRelease(it->second.h);
    release_va(ctx, it->first, it->second.bytes, it->second.in_window);
    ctx->vmm.erase(it);
}

// Drop a registration inside a context range; release the range with its last.
void vmm_drop(ckpt_ctx *ctx, uint64_t start)
{
    auto of = ctx->vmm_of.find(start);
    if (of == ctx->vmm_of.end())
        return;
    const uint64_t base = of->second;
    ctx->vmm_of.erase(of);
    (void)drop_registration(ctx, start);
    auto it = ctx->vmm.find(base);
    if (it != ctx->vmm.end() && --it->second.refs == 0)
        unmap_range(ctx, it);
}

// The live registration that overlaps [a, a + n), if any (n 0: starts at a).
const RangeEnd *overlapping(const ckpt_ctx *ctx, uint64_t a, uint64_t n, uint64_t *start)
{
    auto it = ctx->ranges.lower_bound(a);
    if (it != ctx->ranges.end() && (it->first == a || it->first < a + n)) {
        *start = it->first;
        return &it->second;
    }
    if (it != ctx->ranges.begin()) {
        auto pv = std::prev(it);
        if (a < pv->second.end || (n == 0 && pv->second.end > a)) {
            *start = pv->first;
            return &pv->second;
        }
    }
    return nullptr;
}

}  // namespace

void ckpt::vmm_release_all(ckpt_ctx *ctx)
{
    if (ctx->vmm.empty() && ctx->windows.empty())
        return;
    (void)hipDeviceSynchronize();
    while (!ctx->vmm.empty())
        unmap_range(ctx, ctx->vmm.begin());
    ctx->vmm_of.clear();
    ctx->windows.clear();
}

extern "C" int ckpt_vmm_granularity(ckpt_ctx *ctx, size_t *out)
{
    if (!ctx || !out)
        return set_error(CKPT_E_INVAL, "ctx or out is NULL");
    DeviceGuard dg(ctx->cfg.device);
    uint64_t g = 0;
    CKPT_TRY(granularity(ctx->cfg.device, &g));
    *out = g;
    return CKPT_OK;
}

extern "C" int ckpt_vmm_alloc(ckpt_ctx *ctx, size_t bytes, void *addr, void **out, ckpt_id *id)
{
    if (!ctx || !out || !id)
        return set_error(CKPT_E_INVAL, "ctx, out or id is NULL");
    if (bytes == 0)
        return set_error(CKPT_E_INVAL, "ckpt_vmm_alloc of 0 bytes");
    HookGuard hg(ctx);
    DeviceGuard dg(ctx->cfg.device);
    uint64_t g = 0;
    CKPT_TRY(granularity(ctx->cfg.device, &g));
    const uint64_t want = (uint64_t)(uintptr_t)addr;
    if (want % g != 0)
        return set_error(CKPT_E_INVAL, "address %p is not a multiple of the granularity %llu", addr,
                         (unsigned long long)g);
    const uint64_t span = (bytes + g - 1) / g * g;
    if (span < bytes)
        return set_error(CKPT_E_INVAL, "size %zu overflows", bytes);
    uint64_t s0 = 0;
    if (want && overlapping(ctx, want, span, &s0))
        return set_error(CKPT_E_ADDR, "[%p, +%llu) overlaps a live registration", addr, (unsigned long long)span);
    uint64_t base = 0;
    CKPT_TRY(map_range(ctx, want, span, &base));
    uint64_t rid = 0;
    const int rc = add_registration(ctx, base, bytes, CKPT_DEVICE, 0, &rid);
    if (rc != CKPT_OK) {
        unmap_range(ctx, ctx->vmm.find(base));
        return rc;
    }
    ctx->vmm[base].refs = 1;
    ctx->vmm_of[base] = base;
    *out = (void *)(uintptr_t)base;
    *id = rid;
    return CKPT_OK;
}

int ckpt::vmm_block_map(ckpt_ctx *ctx, uint64_t bytes, uint64_t *base)
{
    DeviceGuard dg(ctx->cfg.device);
    uint64_t g = 0;
    CKPT_TRY(granularity(ctx->cfg.device, &g));
    if (bytes == 0 || bytes % g != 0)
        return set_error(CKPT_E_INVAL, "block of %llu bytes is not a granularity multiple",
                         (unsigned long long)bytes);
    CKPT_TRY(map_range(ctx, 0, bytes, base));
    ctx->vmm[*base].refs = 1;   // the block's owner holds it, registered or not
    return CKPT_OK;
}

void ckpt::vmm_block_unmap(ckpt_ctx *ctx, uint64_t base)
{
    ctx->vmm_of.erase(base);
    auto it = ctx->vmm.find(base);
    if (it == ctx->vmm.end())
        return;
    DeviceGuard dg(ctx->cfg.device);
    unmap_range(ctx, it);
}

extern "C" int ckpt_vmm_free(ckpt_ctx *ctx, void *ptr)
{
    if (!ctx)
        return set_error(CKPT_E_INVAL, "ctx is NULL");
    HookGuard hg(ctx);
    const uint64_t start = (uint64_t)(uintptr_t)ptr;
    if (!ctx->vmm_of.count(start))
        return set_error(CKPT_E_NOTFOUND, "%p is not memory of the context", ptr);
    DeviceGuard dg(ctx->cfg.device);
    // the range may still be in use by work the caller queued on the device
    HIP_TRY(hipDeviceSynchronize());
    vmm_drop(ctx, start);
    return CKPT_OK;
}

namespace {

// What one call created, so that a failure can take it back.
struct Made {
    std::vector<uint64_t> regs;     // registration starts
    std::vector<uint64_t> ranges;   // mapped range bases
};

void undo_made(ckpt_ctx *ctx, const Made &made)
{
    for (uint64_t st : made.regs) {
        ctx->vmm_of.erase(st);
        (void)drop_registration(ctx, st);
    }
    for (uint64_t b : made.ranges) {
        auto it = ctx->vmm.find(b);
        if (it != ctx->vmm.end())
            unmap_range(ctx, it);
    }
}

// Steps 1-3 of a restore at the recorded addresses: every allocation of the
// table either matches a live registration exactly, or is re-created at its
// address (granule-aligned ranges mapped once) and registered there.
int recreate(ckpt_ctx *ctx, const std::vector<ckpt_alloc_rec> &allocs, const std::vector<uint64_t> &addrs,
             Made *made)
{
    const uint64_t n = allocs.size();
    if (addrs.size() != n)
        return set_error(CKPT_E_INVAL, "image has no address section");
    uint64_t g = 0;
    CKPT_TRY(granularity(ctx->cfg.device, &g));
    // blocks the hook keeps for reuse hold address ranges without being
    // registered: give them back so that the recorded addresses are free
    hook_trim_for(ctx);

    // 1. classify: refill a matching live registration, or re-create
    std::vector<char> create(n, 0);
    for (uint64_t k = 0; k < n; k++) {
        const ckpt_alloc_rec &r = allocs[k];
        const uint64_t a = addrs[k];
        if (a == 0 && r.size != 0)
            return set_error(CKPT_E_INVAL, "allocation %llu has no recorded address", (unsigned long long)k);
        if (a % 16 != 0)
            return set_error(CKPT_E_INVAL, "allocation %llu: address 0x%llx is not 16-byte aligned",
                             (unsigned long long)k, (unsigned long long)a);
        uint64_t s0 = 0;
        const RangeEnd *hit = overlapping(ctx, a, r.size, &s0);
        if (hit) {
            const auto row = std::lower_bound(ctx->live.begin(), ctx->live.end(), hit->id,
                                              [](const Reg &x, uint64_t v) { return x.id < v; });
            if (s0 == a && hit->end == a + r.size && row != ctx->live.end() && row->kind == r.kind)
                continue;
            return set_error(CKPT_E_ADDR, "allocation %llu at [0x%llx, +%llu) overlaps registration [0x%llx, 0x%llx)",
                             (unsigned long long)k, (unsigned long long)a, (unsigned long long)r.size,
                             (unsigned long long)s0, (unsigned long long)hit->end);
        }
        if (r.kind != CKPT_DEVICE)
            return set_error(CKPT_E_INVAL, "allocation %llu is managed memory and cannot be re-created at 0x%llx",
                             (unsigned long long)k, (unsigned long long)a);
        create[k] = 1;
    }
    // two allocations of the image may not overlap each other
    {
        std::vector<std::pair<uint64_t, uint64_t>> iv;
        for (uint64_t k = 0; k < n; k++)
            if (allocs[k].size)
                iv.emplace_back(addrs[k], addrs[k] + allocs[k].size);
        std::sort(iv.begin(), iv.end());
        for (size_t i = 1; i < iv.size(); i++)
            if (iv[i].first < iv[i - 1].second)
                return set_error(CKPT_E_INVAL, "allocations of the image overlap at 0x%llx",
                                 (unsigned long long)iv[i].first);
    }

    // 2. granule-aligned ranges covering the allocations to re-create; ranges
    //    that touch share a mapping
    struct Span {
        uint64_t lo, hi;
    };
    std::vector<Span> spans;
    {
        std::vector<Span> raw;
        for (uint64_t k = 0; k < n; k++)
            if (create[k] && allocs[k].size) {
                const uint64_t a = addrs[k], e = a + allocs[k].size;
                raw.push_back({a / g * g, (e + g - 1) / g * g});
            }
        std::sort(raw.begin(), raw.end(), [](const Span &x, const Span &y) { return x.lo < y.lo; });
        for (const Span &s : raw) {
            if (!spans.empty() && s.lo <= spans.back().hi)
                spans.back().hi = std::max(spans.back().hi, s.hi);
            else
                spans.push_back(s);
        }
        for (const Span &s : spans) {
            uint64_t s0 = 0;
            if (overlapping(ctx, s.lo, s.hi - s.lo, &s0))
                return set_error(CKPT_E_ADDR, "range [0x%llx, 0x%llx) holds a live registration at 0x%llx",
                                 (unsigned long long)s.lo, (unsigned long long)s.hi, (unsigned long long)s0);
        }
    }

    // 3. map and register; undo everything on failure
    auto fail = [&](int rc) {
        undo_made(ctx, *made);
        return rc;
    };
    for (const Span &s : spans) {
        uint64_t base = 0;
        const int rc = map_range(ctx, s.lo, s.hi - s.lo, &base);
        if (rc != CKPT_OK)
            return fail(rc);
        made->ranges.push_back(base);
    }
    for (uint64_t k = 0; k < n; k++) {
        if (!create[k])
            continue;
        const ckpt_alloc_rec &r = allocs[k];
        const uint64_t a = addrs[k];
        uint64_t rid = 0;
        int rc = add_registration(ctx, a, r.size, CKPT_DEVICE, r.id, &rid);
        if (rc != CKPT_OK)
            return fail(rc);
        made->regs.push_back(a);
        if (r.size) {
            // the span that holds it: the last with lo <= a
            auto sp = std::upper_bound(spans.begin(), spans.end(), a,
                                       [](uint64_t v, const Span &x) { return v < x.lo; });
            const uint64_t base = std::prev(sp)->lo;
            ctx->vmm_of[a] = base;
            ctx->vmm[base].refs++;
        }
    }

    return CKPT_OK;
}

}  // namespace

extern "C" int ckpt_restore_at(ckpt_ctx *ctx, void *stream, const ckpt_image *img, const ckpt_image *delta,
                               void **addrs_out, ckpt_verify_report *rep)
{
    if (!ctx || !img)
        return set_error(CKPT_E_INVAL, "ctx or image is NULL");
    if (delta && delta->mode == CKPT_INCREMENTAL && delta->base_serial == img->serial) {
        // the allocation table changed between the two: restore the merged image
        std::unique_ptr<ckpt_image> merged;
        CKPT_TRY(fold_delta(img, delta, &merged));
        if (merged)
            return ckpt_restore_at(ctx, stream, merged.get(), nullptr, addrs_out, rep);
    }
    HookGuard hg(ctx);
    DeviceGuard dg(ctx->cfg.device);
    Made made;
    CKPT_TRY(recreate(ctx, img->allocs, img->addrs, &made));

    // 4. refill and verify at those addresses
    const uint64_t n = img->allocs.size();
    std::vector<void *> dst(n);
    for (uint64_t k = 0; k < n; k++)
        dst[k] = (void *)(uintptr_t)img->addrs[k];
    const int rc = restore_impl(ctx, stream, img, delta, n ? dst.data() : nullptr, nullptr, n, rep,
                                !made.ranges.empty());
    if (rc != CKPT_OK && rc != CKPT_E_CORRUPT) {
        (void)hipDeviceSynchronize();
        undo_made(ctx, made);
        return rc;
    }
    if (addrs_out)
        for (uint64_t k = 0; k < n; k++)
            addrs_out[k] = dst[k];
    return rc;
}

extern "C" int ckpt_restore_file_at(ckpt_ctx *ctx, void *stream, const char *path, void **addrs_out,
                                    ckpt_verify_report *rep, ckpt_image **img_out)
{
    if (!ctx || !path)
        return set_error(CKPT_E_INVAL, "ctx or path is NULL");
    // the file's tables into ordinary host memory before any device work
    ImageFile f;
    CKPT_TRY(open_image_file(path, &f));
    const ImageHead &h = f.h;
    if (h.mode != CKPT_FULL)
        return set_error(CKPT_E_INVAL, "restore needs a full image");
    HookGuard hg(ctx);
    DeviceGuard dg(ctx->cfg.device);
    // the address ranges first: nothing of this call has used device memory yet
    Made made;
    CKPT_TRY(recreate(ctx, h.allocs, h.addrs, &made));
    ckpt_image *img = nullptr;
    int rc = load_image_file(ctx, &f, &img);
    if (rc == CKPT_OK) {
        // every allocation is now a live registration at its address: refilled in place
        rc = ckpt_restore_at(ctx, stream, img, nullptr, addrs_out, rep);
    }
    if (rc != CKPT_OK && rc != CKPT_E_CORRUPT) {
        (void)hipDeviceSynchronize();
        undo_made(ctx, made);
        ckpt_image_free(img);
        return rc;
    }
    if (img_out)
        *img_out = img;
    else
        ckpt_image_free(img);
    return rc;
}
