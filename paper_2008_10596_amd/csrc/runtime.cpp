// runtime.cpp -- host runtime of libckpt behind the C ABI in include/ckpt.h.
//
// Registration table (the log of live allocations), device staging, pinned
// host buffers, the checkpoint path (pack on the caller's stream, drain on a
// side stream), restore with verification, image (de)serialization and the
// batched form.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ckpt.h"
#include "ckpt_runtime.h"

using namespace ckpt;

// ------------------------------------------------------------------ errors

static thread_local int t_last_hip = 0;
static thread_local char t_last_msg[512];

int ckpt::set_error(int status, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_last_msg, sizeof(t_last_msg), fmt, ap);
    va_end(ap);
    return status;
}

int ckpt::hip_fail(hipError_t e, const char *what, int line)
{
    t_last_hip = (int)e;
    set_error(0, "%s failed: %s (runtime.cpp:%d)", what, hipGetErrorString(e), line);
    return e == hipErrorOutOfMemory ? CKPT_E_NOMEM : CKPT_E_HIP;
}

extern "C" int ckpt_last_hip_error(void) { return t_last_hip; }
extern "C" const char *ckpt_last_error(void) { return t_last_msg; }

extern "C" const char *ckpt_strerror(int status)
{
    switch (status) {
    case CKPT_OK: return "ok";
    case CKPT_E_INVAL: return "invalid argument";
    case CKPT_E_NOTFOUND: return "not found";
    case CKPT_E_NOMEM: return "out of memory";
    case CKPT_E_HIP: return "HIP runtime error";
    case CKPT_E_MISMATCH: return "image, base or destination mismatch";
    case CKPT_E_CORRUPT: return "checksum mismatch";
    case CKPT_E_AGAIN: return "not finished";
    case CKPT_E_BUDGET: return "staging budget exceeded";
    case CKPT_E_ADDR: return "address range not free";
    case CKPT_E_IO: return "file I/O error";
    default: return "unknown status";
    }
}

// ---------------------------------------------------------- device buffers

int DevBuf::ensure(size_t bytes)
{
    if (bytes <= cap)
        return CKPT_OK;
    release();
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        return hip_fail(e, "hipMalloc", __LINE__);
    }
    cap = want;
    return CKPT_OK;
}

void DevBuf::release()
{
    if (p)
        (void)hipFree(p);
    p = nullptr;
    cap = 0;
}

// ----------------------------------------------------- pinned host memory
//
// hipHostMalloc of gigabytes is slow (it pins every page), so freed pinned
// buffers are kept for reuse, up to a cap, and handed out best-fit.

namespace {
class PinnedPool {
public:
    void *get(size_t bytes, size_t *cap_out)
    {
        if (bytes == 0)
            bytes = 1;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.lower_bound(bytes);
            if (it != free_.end() && it->first <= bytes + bytes / 4 + (4u << 20)) {
                void *p = it->second;
                *cap_out = it->first;
                cached_ -= it->first;
                live_ += it->first;
                free_.erase(it);
                return p;
            }
        }
        const size_t rounded = (bytes + (2u << 20) - 1) & ~size_t((2u << 20) - 1);
        void *p = nullptr;
        if (hipHostMalloc(&p, rounded, hipHostMallocDefault) != hipSuccess) {
            trim(0);   // give cached buffers back and retry once
            if (hipHostMalloc(&p, rounded, hipHostMallocDefault) != hipSuccess)
                return nullptr;
        }
        *cap_out = rounded;
        std::lock_guard<std::mutex> lk(mu_);
        live_ += rounded;
        return p;
    }
    void put(void *p, size_t cap)
    {
        if (!p)
            return;
        std::lock_guard<std::mutex> lk(mu_);
        free_.emplace(cap, p);
        cached_ += cap;
        live_ -= cap;
        trim_locked(kMaxCached);
    }
    uint64_t live()
    {
        std::lock_guard<std::mutex> lk(mu_);
        return live_;
    }
    uint64_t cached()
    {
        std::lock_guard<std::mutex> lk(mu_);
        return cached_;
    }
    void trim(size_t keep)
    {
        std::lock_guard<std::mutex> lk(mu_);
        trim_locked(keep);
    }

private:
    void trim_locked(size_t keep)
    {
        while (cached_ > keep && !free_.empty()) {
            auto it = std::prev(free_.end());   // largest first
            (void)hipHostFree(it->second);
            cached_ -= it->first;
            free_.erase(it);
        }
    }
    // freed buffers kept for reuse; pinning gigabytes again costs far more
    // than keeping them, but they are host memory nobody else can use
    static constexpr size_t kMaxCached = size_t(32) << 30;
    std::mutex mu_;
    std::multimap<size_t, void *> free_;
    size_t cached_ = 0;
    size_t live_ = 0;   // handed out and not yet returned
};

PinnedPool &pinned_pool()
{
    static PinnedPool *pool = new PinnedPool();   // never destroyed: buffers may outlive statics
    return *pool;
}

std::atomic<uint64_t> g_serial{0};

uint64_t next_serial()
{
    static const uint64_t base = [] {
        const uint64_t t = (uint64_t)std::chrono::steady_clock::now().time_since_epoch().count();
        return (t * 0x9E3779B97F4A7C15ull) & 0xFFFFFFFF00000000ull;
    }();
    return base | (++g_serial & 0xFFFFFFFFull);
}


uint64_t ru16(uint64_t x) { return (x + 15) & ~uint64_t(15); }
}  // namespace

uint64_t ckpt::pinned_live_bytes() { return pinned_pool().live(); }

extern "C" int ckpt_host_memory(uint64_t *live, uint64_t *cached)
{
    if (live)
        *live = pinned_pool().live();
    if (cached)
        *cached = pinned_pool().cached();
    return CKPT_OK;
}

// Digest of an image's CRC section: FNV-1a over little-endian 64-bit words
// (the last word zero-padded).  Computed when asked for, not per checkpoint.
uint64_t ckpt::crc_digest(const void *p, size_t n)
{
    const uint8_t *b = (const uint8_t *)p;
    uint64_t h = 0xcbf29ce484222325ull;
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t w;
        memcpy(&w, b + i, 8);
        h = (h ^ w) * 0x100000001b3ull;
    }
    if (i < n) {
        uint64_t w = 0;
        memcpy(&w, b + i, n - i);
        h = (h ^ w) * 0x100000001b3ull;
    }
    return h;
}

int PinnedBuf::ensure(size_t bytes)
{
    if (bytes <= cap && p)
        return CKPT_OK;
    release();
    p = pinned_pool().get(bytes, &cap);
    if (!p) {
        cap = 0;
        return set_error(CKPT_E_NOMEM, "pinned host allocation of %zu bytes failed", bytes);
    }
    return CKPT_OK;
}

void PinnedBuf::release()
{
    if (p)
        pinned_pool().put(p, cap);
    p = nullptr;
    cap = 0;
}

// -------------------------------------------------------------- the image

int ckpt::alloc_meta(ckpt_image *img, uint64_t N)
{
    auto blk = std::make_shared<PinnedBuf>();
    CKPT_TRY(blk->ensure(std::max<uint64_t>(5 * N, 8)));
    img->meta = blk;
    img->crc = (uint32_t *)blk->p;
    img->flags = (uint8_t *)blk->p + 4 * N;
    return CKPT_OK;
}

void ckpt::image_wait(const ckpt_image *img)
{
    if (img && img->meta_ready)
        img->meta_ready->wait();
}

// New work on s that reuses the context's device arrays waits for the last
// asynchronous metadata copy out of them.
int ckpt::order_after_meta(ckpt_ctx *ctx, hipStream_t s)
{
    if (ctx->meta_pending) {
        HIP_TRY(hipStreamWaitEvent(s, ctx->meta_ev, 0));
        ctx->meta_pending = false;
    }
    return CKPT_OK;
}

ckpt_image::~ckpt_image()
{
    ckpt::image_wait(this);   // pinned buffers go back to the pool only when no copy targets them
    if (dense_owned && dense) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(device);
        (void)hipFree(dense);
        (void)hipSetDevice(prev);
    }
}

// ------------------------------------------------------------- device guard

DeviceGuard::DeviceGuard(int dev)
{
    (void)hipGetDevice(&prev_);
    ok_ = hipSetDevice(dev) == hipSuccess;
}
DeviceGuard::~DeviceGuard() { (void)hipSetDevice(prev_); }

// ------------------------------------------------------------------ context

extern "C" int ckpt_init(const ckpt_config *cfg_in, ckpt_ctx **out)
{
    if (!out)
        return set_error(CKPT_E_INVAL, "out is NULL");
    ckpt_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    if (cfg_in)
        cfg = *cfg_in;
    if (cfg.chunk_bytes == 0)
        cfg.chunk_bytes = 4096;
    if (cfg.chunk_bytes % 16 != 0 || cfg.chunk_bytes > (1u << 30))
        return set_error(CKPT_E_INVAL, "chunk_bytes %u: not a multiple of 16 in [16, 2^30]", cfg.chunk_bytes);
    // one 16-byte piece per lane per round and per-lane replicated tables are
    // the only forms (the others measured slower and were removed); the
    // fields stay for the structure's layout
    if (cfg.lane_pieces == 0)
        cfg.lane_pieces = 1;
    if (cfg.lane_pieces != 1)
        return set_error(CKPT_E_INVAL, "lane_pieces %u: only 1 (one 16-byte piece per lane per round)",
                         cfg.lane_pieces);
    if (cfg.table_mode == 0)
        cfg.table_mode = 2;
    if (cfg.table_mode != 2)
        return set_error(CKPT_E_INVAL, "table_mode %u: only 2 (replicated)", cfg.table_mode);
    if (cfg.block_threads == 0)
        cfg.block_threads = 1024;
    if (cfg.block_threads != 64 && cfg.block_threads != 128 && cfg.block_threads != 256 &&
        cfg.block_threads != 512 && cfg.block_threads != 1024)
        return set_error(CKPT_E_INVAL, "block_threads %u", cfg.block_threads);
    if (cfg.waves_per_chunk == 0)
        cfg.waves_per_chunk = 1;
    const uint32_t w = cfg.waves_per_chunk;
    if ((w & (w - 1)) != 0 || w > 16 || w > cfg.block_threads / 64)
        return set_error(CKPT_E_INVAL, "waves_per_chunk %u with block_threads %u", w, cfg.block_threads);
    if ((cfg.flags & CKPT_RESERVE_STAGING) && cfg.staging_budget == 0)
        return set_error(CKPT_E_INVAL, "CKPT_RESERVE_STAGING needs a staging_budget");
    // 0: non-temporal (streaming: every byte is touched once), except for a
    // pack whose dense image mostly starts off 128-byte lines (pack_hint)
    const bool hint_auto = cfg.load_hint == 0;
    if (cfg.load_hint == 0)
        cfg.load_hint = 2;
    if (cfg.load_hint > 2)
        return set_error(CKPT_E_INVAL, "load_hint %u", cfg.load_hint);
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDeviceCount", __LINE__);
    if (cfg.device < 0 || cfg.device >= ndev)
        return set_error(CKPT_E_INVAL, "device %d of %d", cfg.device, ndev);

    DeviceGuard g(cfg.device);
    auto *ctx = new ckpt_ctx();
    ctx->cfg = cfg;
    ctx->hint_auto = hint_auto;
    int rc = ctx_setup(ctx);
    if (rc != CKPT_OK) {
        ckpt_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return CKPT_OK;
}

// CRC operator tables on the device, shared by every context with the same
// device and rounds per wave, and kept until
// the process ends: a batch of hundreds of contexts uploads one set, and a
// context's later calls find its tables in place.
const uint32_t *ckpt::shared_tables(const ckpt_config &cfg, int *rc)
{
    static std::mutex mu;
    static std::map<std::pair<int, uint32_t>, void *> cache;
    const uint32_t r_full = (cfg.chunk_bytes + kRoundBytes - 1) / kRoundBytes;
    const uint32_t rw = (r_full + cfg.waves_per_chunk - 1) / cfg.waves_per_chunk;
    const auto key = std::make_pair(cfg.device, rw);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
        *rc = CKPT_OK;
        return (const uint32_t *)it->second;
    }
    // the set of the one-wave forms, then the quad form's
    std::vector<uint32_t> tabs(2 * kRepWords);
    build_tables_replicated(tabs.data(), rw);
    build_tables_replicated(tabs.data() + kRepWords, rw, kQuadSkipBytes);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, tabs.size() * 4);
    if (e == hipSuccess) {
        e = hipMemcpy(p, tabs.data(), tabs.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(p);
            p = nullptr;
        }
    }
    if (e != hipSuccess) {
        *rc = hip_fail(e, "tables", __LINE__);
        return nullptr;
    }
    cache.emplace(key, p);
    *rc = CKPT_OK;
    return (const uint32_t *)p;
}

int ckpt::ctx_setup(ckpt_ctx *ctx)
{
    const ckpt_config &cfg = ctx->cfg;
    HIP_TRY(hipDeviceGetAttribute(&ctx->cu_count, hipDeviceAttributeMultiprocessorCount, cfg.device));
    int managed = 0;
    if (hipDeviceGetAttribute(&managed, hipDeviceAttributeConcurrentManagedAccess, cfg.device) == hipSuccess)
        ctx->managed_prefetch = managed != 0;
    // the 124 KiB of tables in LDS fit one workgroup per CU (of 160 KiB)
    const int per_cu = cfg.wgs_per_cu ? (int)cfg.wgs_per_cu : 1;
    ctx->grid_chunks = ctx->cu_count * per_cu;
    ctx->grid_small = ctx->cu_count * 4;
    // CRC-32C of C zero bytes (the register from its init through C zero
    // bytes, then the final complement): the CRC of every full-length ZERO chunk
    ctx->zero_crc = host_shift(0xFFFFFFFFu, cfg.chunk_bytes) ^ 0xFFFFFFFFu;
    int rc = CKPT_OK;
    ctx->tables = shared_tables(cfg, &rc);
    if (rc != CKPT_OK)
        return rc;
    if (cfg.flags & CKPT_RESERVE_STAGING) {
        // the whole staging budget as one block, now: the dense image at its
        // start, a drain's or restore's segment slots after it
        CKPT_TRY(ctx->d_dense.ensure(cfg.staging_budget));
        ctx->reserved = true;
    }
    // this device's address of the allocation-free path's device array
    return noalloc_setup(cfg.device);
}

// Streams and events are made on first use, so that contexts that only hold
// registrations (members of a batch) stay cheap.
int ckpt::ctx_ready(ckpt_ctx *ctx)
{
    if (ctx->ready)
        return CKPT_OK;
    const ckpt_config &cfg = ctx->cfg;
    HIP_TRY(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&ctx->gat, hipStreamNonBlocking));
    for (auto &ev : ctx->ev)
        HIP_TRY(hipEventCreate(&ev));
    HIP_TRY(hipEventCreateWithFlags(&ctx->meta_ev, hipEventDisableTiming));
    CKPT_TRY(ctx->d_plan.ensure(sizeof(DevPlan)));
    CKPT_TRY(ctx->h_plan.ensure(sizeof(DevPlan)));
    ctx->ready = true;
    return CKPT_OK;
}

uint64_t ckpt::segment_bytes(const ckpt_config &cfg)
{
    if (cfg.segment_mib == 0xFFFFFFFFu)
        return 0;
    return (uint64_t)(cfg.segment_mib ? cfg.segment_mib : 256) << 20;
}

int ckpt::seg_events(ckpt_ctx *ctx, size_t n)
{
    while (ctx->seg_ev.size() < n) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreate(&e));
        ctx->seg_ev.push_back(e);
    }
    return CKPT_OK;
}

int ckpt::serial_staging(ckpt_ctx *ctx, uint64_t used, uint64_t bytes, uint8_t **out)
{
    if (ctx->reserved) {
        const uint64_t off = (used + 255) & ~uint64_t(255);
        if (off > ctx->d_dense.cap || bytes > ctx->d_dense.cap - off)
            return set_error(CKPT_E_BUDGET, "staging of %llu B past %llu B exceeds the reserved %llu B",
                             (unsigned long long)bytes, (unsigned long long)off,
                             (unsigned long long)ctx->d_dense.cap);
        *out = (uint8_t *)ctx->d_dense.p + off;
        return CKPT_OK;
    }
    CKPT_TRY(ctx->d_compact.ensure(std::max<uint64_t>(bytes, 16)));
    *out = (uint8_t *)ctx->d_compact.p;
    return CKPT_OK;
}

extern "C" void ckpt_destroy(ckpt_ctx *ctx)
{
    if (!ctx)
        return;
    hook_forget(ctx);
    {
        DeviceGuard g(ctx->cfg.device);
        if (ctx->g_exec)
            (void)hipGraphExecDestroy(ctx->g_exec);
        for (hipStream_t st : {ctx->side, ctx->cap, ctx->gat})
            if (st) {
                (void)hipStreamSynchronize(st);
                (void)hipStreamDestroy(st);
            }
        for (auto &ev : ctx->ev)
            if (ev)
                (void)hipEventDestroy(ev);
        for (hipEvent_t ev : ctx->seg_ev)
            (void)hipEventDestroy(ev);
        if (ctx->meta_ev)
            (void)hipEventDestroy(ctx->meta_ev);
        for (DevBuf *b : ctx->all_dev())
            b->release();
        ctx->h_up.release();
        ctx->h_plan.release();
        ctx->h_base_cb.release();
        vmm_release_all(ctx);
    }
    delete ctx;
}

// ------------------------------------------------------------ registration

int ckpt::add_registration(ckpt_ctx *ctx, uint64_t start, uint64_t bytes, uint32_t kind, uint64_t want_id,
                           uint64_t *id)
{
    if (start % 16 != 0)
        return set_error(CKPT_E_INVAL, "pointer 0x%llx is not 16-byte aligned", (unsigned long long)start);
    if (start == 0 && bytes != 0)
        return set_error(CKPT_E_INVAL, "NULL pointer with %llu bytes", (unsigned long long)bytes);
    if (start + bytes < start)
        return set_error(CKPT_E_INVAL, "range wraps the address space");
    // Overlap: a live range [s, e) with s < start + bytes and start < e, or the
    // same start (starts identify registrations).
    auto it = ctx->ranges.lower_bound(start);
    if (it != ctx->ranges.end() && (it->first == start || it->first < start + bytes))
        return set_error(CKPT_E_INVAL, "[0x%llx, +%llu) overlaps a live registration", (unsigned long long)start,
                         (unsigned long long)bytes);
    if (it != ctx->ranges.begin()) {
        auto pv = std::prev(it);
        if (start < pv->second.end)
            return set_error(CKPT_E_INVAL, "[0x%llx, +%llu) overlaps a live registration",
                             (unsigned long long)start, (unsigned long long)bytes);
    }
    Reg r;
    r.id = want_id >= ctx->next_id ? want_id : ctx->next_id;
    ctx->next_id = r.id + 1;
    r.kind = kind;
    r.ptr = start;
    r.size = bytes;
    ctx->live.push_back(r);   // the largest id so far: live stays in id order
    ctx->ranges.emplace(start, RangeEnd{start + bytes, r.id});
    *id = r.id;
    return CKPT_OK;
}

int ckpt::drop_registration(ckpt_ctx *ctx, uint64_t start)
{
    auto it = ctx->ranges.find(start);
    if (it == ctx->ranges.end())
        return set_error(CKPT_E_NOTFOUND, "0x%llx is not a live registration", (unsigned long long)start);
    const uint64_t id = it->second.id;
    ctx->ranges.erase(it);
    // live is in id order; ids are unique, so a binary search finds the row
    auto row = std::lower_bound(ctx->live.begin(), ctx->live.end(), id,
                                [](const Reg &a, uint64_t v) { return a.id < v; });
    if (row != ctx->live.end() && row->id == id)
        ctx->live.erase(row);
    return CKPT_OK;
}

extern "C" int ckpt_register(ckpt_ctx *ctx, void *ptr, size_t bytes, int kind, ckpt_id *out)
{
    if (!ctx || !out)
        return set_error(CKPT_E_INVAL, "ctx or out is NULL");
    HookGuard hg(ctx);
    if (kind != CKPT_DEVICE && kind != CKPT_MANAGED)
        return set_error(CKPT_E_INVAL, "unknown kind %d", kind);
    return add_registration(ctx, (uint64_t)(uintptr_t)ptr, bytes, (uint32_t)kind, 0, out);
}

extern "C" int ckpt_unregister(ckpt_ctx *ctx, void *ptr)
{
    if (!ctx)
        return set_error(CKPT_E_INVAL, "ctx is NULL");
    HookGuard hg(ctx);
    if (ctx->vmm_of.count((uint64_t)(uintptr_t)ptr))
        return set_error(CKPT_E_INVAL, "%p is memory of the context; release it with ckpt_vmm_free", ptr);
    return drop_registration(ctx, (uint64_t)(uintptr_t)ptr);
}

extern "C" int ckpt_live_count(const ckpt_ctx *ctx, size_t *out)
{
    if (!ctx || !out)
        return set_error(CKPT_E_INVAL, "ctx or out is NULL");
    HookGuard hg(ctx);
    *out = ctx->live.size();
    return CKPT_OK;
}

// -------------------------------------------------------------- timing

namespace {
float ev_ms(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess)
        return 0.f;
    return ms;
}
}  // namespace

extern "C" int ckpt_last_timing(const ckpt_ctx *ctx, ckpt_timing *out)
{
    if (!ctx || !out)
        return set_error(CKPT_E_INVAL, "ctx or out is NULL");
    *out = ctx->timing;
    return CKPT_OK;
}

// ---------------------------------------------------------- shared helpers

// Uploads the allocation table (addresses, sizes) and a fresh plan header to
// the device on stream s, then runs the size scan and the chunk map.
int ckpt::upload_table(ckpt_ctx *ctx, hipStream_t s, const std::vector<Row> &rows, bool dst_side,
                       uint64_t N_host, uint64_t n_items)
{
    const uint64_t n = rows.size();
    CKPT_TRY(ctx->d_addr.ensure(std::max<uint64_t>(n, 1) * 8));
    CKPT_TRY(ctx->d_size.ensure(std::max<uint64_t>(n, 1) * 8));
    CKPT_TRY(ctx->d_off.ensure((n + 1) * 8));
    CKPT_TRY(ctx->d_cb.ensure((n + 1) * 8));
    CKPT_TRY(ctx->d_map.ensure(std::max<uint64_t>(N_host, 1) * 4));
    const size_t up_bytes = sizeof(DevPlan) + 16 * n;
    CKPT_TRY(ctx->h_up.ensure(up_bytes));
    auto *plan = (DevPlan *)ctx->h_up.p;
    memset(plan, 0, sizeof(DevPlan));
    plan->n_allocs = n;
    plan->n_items = n_items;
    auto *addr = (uint64_t *)((uint8_t *)ctx->h_up.p + sizeof(DevPlan));
    auto *size = addr + n;
    for (uint64_t k = 0; k < n; k++) {
        addr[k] = rows[k].ptr;
        size[k] = rows[k].size;
    }
    (void)dst_side;
    // The scan reads the table from the pinned buffer and copies it to the
    // device itself (no copies on the runtime's copy path, which the previous
    // call's copies to the host may still be using).
    HIP_TRY(launch_upload_scan(s, ctx->h_up.p, (DevPlan *)ctx->d_plan.p, (uint64_t *)ctx->d_addr.p,
                               (uint64_t *)ctx->d_size.p, ctx->cfg.chunk_bytes, (uint64_t *)ctx->d_off.p,
                               (uint64_t *)ctx->d_cb.p));
    if (N_host)
        HIP_TRY(launch_chunk_map(s, (const DevPlan *)ctx->d_plan.p, (const uint64_t *)ctx->d_cb.p,
                                 (uint32_t *)ctx->d_map.p, ctx->grid_small));
    // every call synchronizes before it returns, so the kernel has read h_up
    // before the host next rewrites it
    return CKPT_OK;
}

int ckpt::read_plan(ckpt_ctx *ctx, hipStream_t s, DevPlan *out)
{
    HIP_TRY(hipMemcpyAsync(ctx->h_plan.p, ctx->d_plan.p, sizeof(DevPlan), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    memcpy(out, ctx->h_plan.p, sizeof(DevPlan));
    return CKPT_OK;
}

int ckpt::run_select(ckpt_ctx *ctx, hipStream_t s, int mode, const uint8_t *flags, const uint64_t *ids,
                     uint64_t max_items, uint64_t *soff, uint64_t *ids_out, uint64_t ids_cap)
{
    const uint64_t tiles = (max_items + kSelTile - 1) / kSelTile;
    CKPT_TRY(ctx->d_tile_b.ensure(std::max<uint64_t>(tiles, 1) * 8));
    CKPT_TRY(ctx->d_tile_c.ensure(std::max<uint64_t>(tiles, 1) * 8));
    SelArgs a;
    memset(&a, 0, sizeof(a));
    a.plan = (DevPlan *)ctx->d_plan.p;
    a.mode = mode;
    a.C = ctx->cfg.chunk_bytes;
    a.size = (const uint64_t *)ctx->d_size.p;
    a.cb = (const uint64_t *)ctx->d_cb.p;
    a.map = (const uint32_t *)ctx->d_map.p;
    a.flags = flags;
    a.ids = ids;
    a.tile_bytes = (uint64_t *)ctx->d_tile_b.p;
    a.tile_count = (uint64_t *)ctx->d_tile_c.p;
    a.soff = soff;
    a.ids_out = ids_out;
    a.ids_cap = ids_cap;
    HIP_TRY(launch_select(s, a, max_items));
    return CKPT_OK;
}

ChunkArgs ckpt::chunk_args(ckpt_ctx *ctx)
{
    ChunkArgs a;
    memset(&a, 0, sizeof(a));
    a.plan = (const DevPlan *)ctx->d_plan.p;
    a.plan_rw = (DevPlan *)ctx->d_plan.p;
    a.tables = ctx->tables;
    a.tables_quad = a.tables + kRepWords;
    a.C = ctx->cfg.chunk_bytes;
    a.waves_per_chunk = ctx->cfg.waves_per_chunk;
    a.nontemporal = ctx->cfg.load_hint == 2;
    a.zero_crc = ctx->zero_crc;
    a.size = (const uint64_t *)ctx->d_size.p;
    a.off = (const uint64_t *)ctx->d_off.p;
    a.cb = (const uint64_t *)ctx->d_cb.p;
    a.map = (const uint32_t *)ctx->d_map.p;
    return a;
}

namespace {

struct Layout {
    std::vector<uint64_t> off, cb;   // n + 1 each
    uint64_t data_bytes = 0, N = 0;
};

Layout host_layout(const std::vector<Row> &rows, uint32_t C)
{
    Layout L;
    L.off.resize(rows.size() + 1);
    L.cb.resize(rows.size() + 1);
    uint64_t o = 0, g = 0;
    for (size_t k = 0; k < rows.size(); k++) {
        L.off[k] = o;
        L.cb[k] = g;
        o += ru16(rows[k].size);
        g += (rows[k].size + C - 1) / C;
    }
    L.off[rows.size()] = o;
    L.cb[rows.size()] = g;
    L.data_bytes = o;
    L.N = g;
    return L;
}

bool same_table(const ckpt_image *a, const std::vector<Row> &rows, uint32_t C)
{
    if (a->C != C || a->allocs.size() != rows.size())
        return false;
    for (size_t k = 0; k < rows.size(); k++)
        if (a->allocs[k].id != rows[k].id || a->allocs[k].kind != rows[k].kind || a->allocs[k].size != rows[k].size)
            return false;
    return true;
}

bool same_table(const ckpt_image *a, const ckpt_image *b)
{
    if (a->C != b->C || a->allocs.size() != b->allocs.size())
        return false;
    for (size_t k = 0; k < a->allocs.size(); k++)
        if (a->allocs[k].id != b->allocs[k].id || a->allocs[k].kind != b->allocs[k].kind ||
            a->allocs[k].size != b->allocs[k].size)
            return false;
    return true;
}

}  // namespace

// ------------------------------------------------------------ graph prologue
//
// The device part of a full checkpoint without a base -- table upload from
// pinned memory, size scan, chunk map, pack, and, when the checkpoint drains,
// the select and a gather that stores every output's non-ZERO chunks straight
// into that output's pinned host buffer -- captured once in a hipGraph and
// replayed.  Every kernel reads its counts from the device plan, so one graph
// serves any table that fits the capacities it was captured with; the host
// only rewrites the pinned upload buffer (descriptors, and for the drain each
// output's host address, first chunk, and each row's output).  A changed
// buffer address (a buffer grown by another call) forces a new capture.

namespace {
uint64_t grow(uint64_t x, uint64_t floor) { return std::max<uint64_t>(floor, x + x / 4); }
}  // namespace

int ckpt::graph_prologue(ckpt_ctx *ctx, hipStream_t s, const std::vector<Row> &rows, uint64_t N,
                         uint64_t data_bytes, const GraphDrain *drain, bool nontemporal)
{
    const uint64_t n = rows.size();
    const size_t nout = drain ? drain->nout : 0;
    auto buffers = [&]() {
        std::vector<void *> v = {ctx->d_plan.p, ctx->d_addr.p, ctx->d_size.p, ctx->d_off.p, ctx->d_cb.p,
                                 ctx->d_map.p,  ctx->d_crc.p,  ctx->d_flags.p, ctx->d_dense.p, ctx->h_up.p};
        if (drain)
            for (void *p : {ctx->d_soff.p, ctx->d_tile_b.p, ctx->d_tile_c.p, ctx->d_drain.p})
                v.push_back(p);
        return v;
    };
    const bool fits = ctx->g_exec && n <= ctx->g_n && N <= ctx->g_N && data_bytes <= ctx->g_D &&
                      (drain != nullptr) == ctx->g_drain && nout <= ctx->g_outs && buffers() == ctx->g_ptrs &&
                      nontemporal == ctx->g_nt;
    if (!fits) {
        if (ctx->g_exec) {
            (void)hipGraphExecDestroy(ctx->g_exec);
            ctx->g_exec = nullptr;
        }
        const uint64_t nc = grow(n, 64), Nc = grow(N, 1024), oc = drain ? grow(nout, 8) : 0;
        // a reserved dense block is kept (a larger image is refused by the budget)
        const uint64_t Dc = ctx->reserved ? std::max<uint64_t>(data_bytes, ctx->d_dense.cap) : grow(data_bytes, 1 << 20);
        // the drain tables: out_addr[oc], out_chunk0[oc], row_out[nc] (u32)
        const uint64_t drain_bytes = drain ? 16 * oc + 4 * nc : 0;
        const uint64_t tiles = (Nc + kSelTile - 1) / kSelTile;
        CKPT_TRY(ctx->d_addr.ensure(nc * 8));
        CKPT_TRY(ctx->d_size.ensure(nc * 8));
        CKPT_TRY(ctx->d_off.ensure((nc + 1) * 8));
        CKPT_TRY(ctx->d_cb.ensure((nc + 1) * 8));
        CKPT_TRY(ctx->d_map.ensure(Nc * 4));
        CKPT_TRY(ctx->d_crc.ensure(Nc * 4));
        CKPT_TRY(ctx->d_flags.ensure(Nc));
        CKPT_TRY(ctx->d_dense.ensure(Dc));
        if (drain) {
            CKPT_TRY(ctx->d_soff.ensure(Nc * 8));
            CKPT_TRY(ctx->d_tile_b.ensure(tiles * 8));
            CKPT_TRY(ctx->d_tile_c.ensure(tiles * 8));
            CKPT_TRY(ctx->d_drain.ensure(drain_bytes));
        }
        CKPT_TRY(ctx->h_up.ensure(sizeof(DevPlan) + 16 * nc + drain_bytes));
        uint8_t *up = (uint8_t *)ctx->h_up.p;
        hipStream_t c = ctx->cap;
        HIP_TRY(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
        hipGraph_t graph = nullptr;
        auto capture = [&]() -> int {
            HIP_TRY(hipMemcpyAsync(ctx->d_plan.p, up, sizeof(DevPlan), hipMemcpyHostToDevice, c));
            HIP_TRY(hipMemcpyAsync(ctx->d_addr.p, up + sizeof(DevPlan), 8 * nc, hipMemcpyHostToDevice, c));
            HIP_TRY(hipMemcpyAsync(ctx->d_size.p, up + sizeof(DevPlan) + 8 * nc, 8 * nc, hipMemcpyHostToDevice, c));
            if (drain)
                HIP_TRY(hipMemcpyAsync(ctx->d_drain.p, up + sizeof(DevPlan) + 16 * nc, drain_bytes,
                                       hipMemcpyHostToDevice, c));
            HIP_TRY(launch_layout_scan(c, (DevPlan *)ctx->d_plan.p, (const uint64_t *)ctx->d_size.p,
                                       ctx->cfg.chunk_bytes, (uint64_t *)ctx->d_off.p, (uint64_t *)ctx->d_cb.p));
            HIP_TRY(launch_chunk_map(c, (const DevPlan *)ctx->d_plan.p, (const uint64_t *)ctx->d_cb.p,
                                     (uint32_t *)ctx->d_map.p, ctx->grid_small));
            ChunkArgs a = chunk_args(ctx);
            a.nontemporal = nontemporal ? 1 : 0;
            a.src = (const uint64_t *)ctx->d_addr.p;
            a.dense = (uint8_t *)ctx->d_dense.p;
            a.crc = (uint32_t *)ctx->d_crc.p;
            a.flags = (uint8_t *)ctx->d_flags.p;
            HIP_TRY(launch_chunks(c, kModePack, a, ctx->grid_chunks, ctx->cfg.block_threads));
            if (drain) {
                // the drain: serialized offsets of the non-ZERO chunks, then each
                // chunk straight into its output's pinned host buffer
                SelArgs sa;
                memset(&sa, 0, sizeof(sa));
                sa.plan = (DevPlan *)ctx->d_plan.p;
                sa.mode = kSelNonZero;
                sa.C = ctx->cfg.chunk_bytes;
                sa.size = (const uint64_t *)ctx->d_size.p;
                sa.cb = (const uint64_t *)ctx->d_cb.p;
                sa.map = (const uint32_t *)ctx->d_map.p;
                sa.flags = (const uint8_t *)ctx->d_flags.p;
                sa.tile_bytes = (uint64_t *)ctx->d_tile_b.p;
                sa.tile_count = (uint64_t *)ctx->d_tile_c.p;
                sa.soff = (uint64_t *)ctx->d_soff.p;
                HIP_TRY(launch_select(c, sa, Nc));
                GatherArgs ga;
                memset(&ga, 0, sizeof(ga));
                ga.plan = (const DevPlan *)ctx->d_plan.p;
                ga.mode = kSelNonZero;
                ga.from_dense = 1;
                ga.C = ctx->cfg.chunk_bytes;
                ga.src = (const uint64_t *)ctx->d_addr.p;
                ga.size = (const uint64_t *)ctx->d_size.p;
                ga.off = (const uint64_t *)ctx->d_off.p;
                ga.cb = (const uint64_t *)ctx->d_cb.p;
                ga.map = (const uint32_t *)ctx->d_map.p;
                ga.dense = (const uint8_t *)ctx->d_dense.p;
                ga.flags = (const uint8_t *)ctx->d_flags.p;
                ga.soff = (const uint64_t *)ctx->d_soff.p;
                ga.out_host = 1;
                ga.out_addr = (const uint64_t *)ctx->d_drain.p;
                ga.out_chunk0 = (const uint64_t *)ctx->d_drain.p + oc;
                ga.row_out = (const uint32_t *)((const uint64_t *)ctx->d_drain.p + 2 * oc);
                HIP_TRY(launch_gather(c, ga, 2 * ctx->cu_count));
            }
            return CKPT_OK;
        };
        const int rc = capture();
        const hipError_t e = hipStreamEndCapture(c, &graph);
        if (rc != CKPT_OK) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess)
            return hip_fail(e, "hipStreamEndCapture", __LINE__);
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess)
            return hip_fail(ei, "hipGraphInstantiate", __LINE__);
        ctx->g_exec = exec;
        ctx->g_n = nc;
        ctx->g_N = Nc;
        ctx->g_D = Dc;
        ctx->g_drain = drain != nullptr;
        ctx->g_outs = oc;
        ctx->g_nt = nontemporal;
        ctx->g_ptrs = buffers();
        ctx->graph_captures++;
    }
    // New descriptor contents in the captured upload buffer.  The previous
    // call on this context has finished with it (every call synchronizes).
    uint8_t *up = (uint8_t *)ctx->h_up.p;
    auto *plan = (DevPlan *)up;
    memset(plan, 0, sizeof(DevPlan));
    plan->n_allocs = n;
    auto *addr = (uint64_t *)(up + sizeof(DevPlan));
    auto *size = addr + ctx->g_n;
    for (uint64_t k = 0; k < n; k++) {
        addr[k] = rows[k].ptr;
        size[k] = rows[k].size;
    }
    if (drain) {
        uint64_t *out_addr = size + ctx->g_n, *out_chunk0 = out_addr + ctx->g_outs;
        auto *row_out = (uint32_t *)(out_chunk0 + ctx->g_outs);
        for (size_t i = 0; i < nout; i++) {
            out_addr[i] = (uint64_t)(uintptr_t)(*drain->data)[i].p;
            out_chunk0[i] = drain->part_chunk[i];
            for (uint64_t k = drain->part_row[i]; k < drain->part_row[i + 1]; k++)
                row_out[k] = (uint32_t)i;
        }
    }
    HIP_TRY(hipGraphLaunch(ctx->g_exec, s));
    return CKPT_OK;
}

// ---------------------------------------------------------------- checkpoint
//
// rows: the table to drain, possibly the concatenation of several contexts'
// tables (batched form); parts[i] = first row of output i (parts.size() =
// number of outputs).  Each output's image is the one its rows alone give.

// The load/store hint of a pack.  With load_hint 0, non-temporal, unless most
// live bytes sit in allocations whose dense image starts off a 128-byte line:
// then the line two neighbouring chunks share is written in two parts by two
// waves, and regular stores let the two parts meet in the L2 instead of going
// to HBM one by one (many allocations of arbitrary sizes, as in a batch).
bool ckpt::pack_hint(const ckpt_ctx *ctx, const std::vector<Row> &rows, const std::vector<uint64_t> &off)
{
    if (!ctx->hint_auto)
        return ctx->cfg.load_hint == 2;
    uint64_t live = 0, off_line = 0;
    for (size_t k = 0; k < rows.size(); k++) {
        live += rows[k].size;
        if (off[k] % 128)
            off_line += rows[k].size;
    }
    return 2 * off_line <= live;
}

int ckpt::run_checkpoint(ckpt_ctx *ctx, hipStream_t s, int mode, const ckpt_image *base, const std::vector<Row> &rows,
                         const std::vector<size_t> &parts, std::vector<ckpt_image *> &outs, bool use_graph)
{
    const ckpt_config &cfg = ctx->cfg;
    const uint32_t C = cfg.chunk_bytes;
    const bool timing = cfg.flags & CKPT_TIMING;
    const bool no_drain = cfg.flags & CKPT_NO_DRAIN;
    const bool keep_dense = cfg.flags & CKPT_KEEP_DENSE;
    const bool direct = cfg.flags & CKPT_DRAIN_DIRECT;
    const bool incremental = mode == CKPT_INCREMENTAL;
    const Layout L = host_layout(rows, C);
    const uint64_t n = rows.size(), N = L.N;
    ckpt_timing &T = ctx->timing;
    memset(&T, 0, sizeof(T));
    const auto t_call = std::chrono::steady_clock::now();

    image_wait(base);
    if (base && base->C != C)
        return set_error(CKPT_E_MISMATCH, "base image has chunk size %u, context %u", base->C, C);
    // A base with another allocation table is matched by registration id:
    // base_cb[k] is the base's first chunk of allocation k when the base has
    // an allocation with its id, size and kind, else kNoBase (every chunk DIRTY).
    const bool remap = base && !same_table(base, rows, C);
    std::vector<uint64_t> base_cb;
    if (remap) {
        base_cb.assign(n, kNoBase);
        size_t j = 0;
        for (uint64_t k = 0; k < n; k++) {
            while (j < base->allocs.size() && base->allocs[j].id < rows[k].id)
                j++;
            if (j < base->allocs.size() && base->allocs[j].id == rows[k].id &&
                base->allocs[j].size == rows[k].size && base->allocs[j].kind == rows[k].kind)
                base_cb[k] = base->allocs[j].cb;
        }
    }
    if (!incremental && cfg.staging_budget && L.data_bytes > cfg.staging_budget)
        return set_error(CKPT_E_BUDGET, "dense image %llu B exceeds the staging budget %llu B",
                         (unsigned long long)L.data_bytes, (unsigned long long)cfg.staging_budget);

    // Drain pending device work first (CheCUDA's step (a)), unless the caller
    // asked for stream order only.
    if (!(cfg.flags & CKPT_STREAM_ORDERED)) {
        const auto t0 = std::chrono::steady_clock::now();
        HIP_TRY(hipDeviceSynchronize());
        T.order_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    // The previous call's host copies may still be running on the side stream;
    // they read only the snapshot buffers (d_prev_crc, d_snap_flags), which
    // this call writes only after waiting for them (order_after_meta below), so
    // this call's table upload and pack overlap them.
    if (ctx->managed_prefetch)
        for (const Row &r : rows)
            if (r.kind == CKPT_MANAGED && r.size)
                HIP_TRY(hipMemPrefetchAsync((const void *)r.ptr, r.size, cfg.device, s));

    const bool graph = use_graph && !incremental && !base && !keep_dense;
    // A replayed graph also holds the drain when there is one: select, then a
    // gather that stores each output's chunks straight into its pinned host
    // buffer (sized to the output's dense bytes, which bound its serialized bytes).
    const bool graph_drain = graph && !no_drain && !direct;
    // Per-output slices: rows [parts[i], parts[i+1]) -> chunks [cb_i, cb_i+1)
    // -> serialized bytes [soff(cb_i), soff(cb_i+1)).
    const size_t nout = outs.size();
    std::vector<uint64_t> part_row(nout + 1), part_chunk(nout + 1), part_data(nout + 1, 0);
    for (size_t i = 0; i < nout; i++)
        part_row[i] = parts[i];
    part_row[nout] = n;
    for (size_t i = 0; i <= nout; i++)
        part_chunk[i] = L.cb[part_row[i]];
    std::vector<PinnedBuf> data(nout);
    uint8_t *dense = nullptr;
    void *dense_owned = nullptr;
    struct DenseGuard {
        void *p;
        ~DenseGuard() { if (p) (void)hipFree(p); }
    } dense_guard{nullptr};
    if (timing)
        HIP_TRY(hipEventRecord(ctx->ev[0], s));
    if (graph) {
        // the replayed graph holds the upload, scan, map and pack (and the
        // drain's select and gather): ev[0] -> ev[2] spans all of it (layout_ms
        // is reported as 0)
        GraphDrain gd{nout, part_row.data(), part_chunk.data(), &data};
        if (graph_drain)
            for (size_t i = 0; i < nout; i++)
                CKPT_TRY(data[i].ensure(std::max<uint64_t>(L.off[part_row[i + 1]] - L.off[part_row[i]], 16)));
        CKPT_TRY(graph_prologue(ctx, s, rows, N, L.data_bytes, graph_drain ? &gd : nullptr, pack_hint(ctx, rows, L.off)));
        dense = (uint8_t *)ctx->d_dense.p;
        if (timing) {
            HIP_TRY(hipEventRecord(ctx->ev[2], s));
        }
    } else {
    CKPT_TRY(upload_table(ctx, s, rows, false, N, 0));
    CKPT_TRY(ctx->d_crc.ensure(std::max<uint64_t>(N, 1) * 4));
    CKPT_TRY(ctx->d_flags.ensure(std::max<uint64_t>(N, 1)));

    // DIRTY is judged against the base's CRC array; the context keeps the last
    // image's array on the device, so a chain of increments uploads nothing.
    const uint32_t *d_base = nullptr;
    const uint64_t *d_base_cb = nullptr;
    if (base) {
        const uint64_t bN = base->N;
        if (base->serial == ctx->prev_serial && ctx->d_prev_crc.cap >= bN * 4) {
            d_base = (const uint32_t *)ctx->d_prev_crc.p;
        } else {
            CKPT_TRY(ctx->d_base_crc.ensure(std::max<uint64_t>(bN, 1) * 4));
            if (bN)
                HIP_TRY(hipMemcpyAsync(ctx->d_base_crc.p, base->crc, bN * 4, hipMemcpyHostToDevice, s));
            d_base = (const uint32_t *)ctx->d_base_crc.p;
        }
        if (remap) {
            CKPT_TRY(ctx->h_base_cb.ensure(std::max<uint64_t>(n, 1) * 8));
            CKPT_TRY(ctx->d_base_cb.ensure(std::max<uint64_t>(n, 1) * 8));
            if (n) {
                memcpy(ctx->h_base_cb.p, base_cb.data(), n * 8);
                HIP_TRY(hipMemcpyAsync(ctx->d_base_cb.p, ctx->h_base_cb.p, n * 8, hipMemcpyHostToDevice, s));
            }
            d_base_cb = (const uint64_t *)ctx->d_base_cb.p;
        }
    }

    // Dense image: the context's staging, or a buffer the image will own.
    if (!incremental) {
        if (keep_dense) {
            hipError_t e = hipMalloc(&dense_owned, std::max<uint64_t>(L.data_bytes, 16));
            if (e != hipSuccess)
                return hip_fail(e, "hipMalloc(dense image)", __LINE__);
            dense_guard.p = dense_owned;
            dense = (uint8_t *)dense_owned;
        } else {
            int rc = ctx->d_dense.ensure(std::max<uint64_t>(L.data_bytes, 16));
            if (rc != CKPT_OK)
                return rc;
            dense = (uint8_t *)ctx->d_dense.p;
        }
    }
    if (timing)
        HIP_TRY(hipEventRecord(ctx->ev[1], s));
    ChunkArgs a = chunk_args(ctx);
    a.src = (const uint64_t *)ctx->d_addr.p;
    a.dense = dense;
    a.crc = (uint32_t *)ctx->d_crc.p;
    a.flags = (uint8_t *)ctx->d_flags.p;
    a.base_crc = d_base;
    a.base_cb = d_base_cb;
    if (!incremental)
        a.nontemporal = pack_hint(ctx, rows, L.off) ? 1 : 0;
    if (N)
        HIP_TRY(launch_chunks(s, incremental ? kModeHash : kModePack, a, ctx->grid_chunks, cfg.block_threads));
    if (timing)
        HIP_TRY(hipEventRecord(ctx->ev[2], s));
    }
    ChunkArgs a = chunk_args(ctx);
    a.flags = (uint8_t *)ctx->d_flags.p;
    T.pack_read_bytes = 0;
    for (const Row &r : rows)
        T.pack_read_bytes += r.size;
    T.pack_write_bytes = incremental ? 0 : L.data_bytes;
    T.pack_write_bytes += 5 * N;

    CKPT_TRY(ctx->d_soff.ensure(std::max<uint64_t>(N, 1) * 8));
    CKPT_TRY(ctx->d_ids.ensure(std::max<uint64_t>(N, 1) * 8));
    uint64_t *d_soff = (uint64_t *)ctx->d_soff.p;
    DevPlan P;
    uint8_t *d_out = nullptr;        // where the gather writes (device compact or pinned host)

    hipStream_t ds = ctx->side;      // drain stream: the copies to the host
    hipStream_t gs = ctx->side;      // the stream the gather runs on
    bool snap = false;               // the host copies read the snapshot buffers
    if (incremental) {
        // The delta is gathered from the allocations themselves, so it must be
        // taken before `s` may run new work: hash, select and gather on s.
        // The copies to the host then run on the side stream.
        CKPT_TRY(run_select(ctx, s, kSelDirtyNonZero, a.flags, nullptr, N, d_soff, (uint64_t *)ctx->d_ids.p, N));
        CKPT_TRY(read_plan(ctx, s, &P));
        gs = s;
    } else {
        if (no_drain && N) {
            // Snapshot the CRC and flag arrays for the host copies, which then
            // run on the side stream after this call returns: the next pack may
            // overwrite d_crc / d_flags at once.  The CRC snapshot is also the
            // base of the next increment.
            CKPT_TRY(order_after_meta(ctx, s));
            CKPT_TRY(ctx->d_prev_crc.ensure(N * 4));
            CKPT_TRY(ctx->d_snap_flags.ensure(N));
            HIP_TRY(hipMemcpyAsync(ctx->d_prev_crc.p, ctx->d_crc.p, N * 4, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(ctx->d_snap_flags.p, ctx->d_flags.p, N, hipMemcpyDeviceToDevice, s));
            snap = true;
        }
        HIP_TRY(hipEventRecord(ctx->ev[3], s));   // packed: the caller's stream is free
        HIP_TRY(hipStreamWaitEvent(ctx->side, ctx->ev[3], 0));
        if (no_drain) {
            P.sel_bytes = 0;
            P.sel_count = 0;
        } else if (graph_drain) {
            CKPT_TRY(read_plan(ctx, ds, &P));   // the graph has selected and gathered
        } else {
            CKPT_TRY(run_select(ctx, ds, kSelNonZero, a.flags, nullptr, N, d_soff, nullptr, 0));
            CKPT_TRY(read_plan(ctx, ds, &P));
        }
    }
    if (timing)
        HIP_TRY(hipEventRecord(ctx->ev[4], gs));

    const uint64_t sel_bytes = no_drain ? 0 : P.sel_bytes;
    // A full checkpoint drains in segments of seg_chunks chunks: each
    // segment's gather (on the gather stream, into one of kSegSlots device
    // slots) overlaps the copy of earlier segments to the host (on the side
    // stream), and at most kSegSlots segments are staged.  An increment is
    // gathered on s in one pass (it is small, and s must not wait for the host
    // link); CKPT_DRAIN_DIRECT stores to the host from the gather itself.
    const uint64_t seg_b = segment_bytes(cfg);
    const uint64_t seg_chunks = seg_b ? std::max<uint64_t>(1, seg_b / C) : 0;
    const uint64_t n_seg = (!no_drain && sel_bytes && !incremental && !direct && !graph_drain && seg_b)
                               ? (N + seg_chunks - 1) / seg_chunks : 0;
    const bool segmented = n_seg > 1;
    const uint64_t slot_bytes = seg_chunks * C;   // a segment's serialized bytes never exceed this
    std::vector<uint64_t> seg_data;               // serialized offset of each segment's first chunk
    if (!no_drain) {
        if (nout == 1 && !segmented) {
            part_data[1] = sel_bytes;
        } else {
            // serialized offsets (soff) at the outputs' and segments' first chunks
            std::vector<uint64_t> want(part_chunk.begin(), part_chunk.end());
            if (segmented)
                for (uint64_t k = 0; k <= n_seg; k++)
                    want.push_back(std::min<uint64_t>(N, k * seg_chunks));
            const size_t m = want.size();
            CKPT_TRY(ctx->d_pick.ensure(m * 16));
            std::vector<uint64_t> idx(m), val(m);
            for (size_t i = 0; i < m; i++)
                idx[i] = std::min<uint64_t>(want[i], N ? N - 1 : 0);
            uint64_t *d_idx = (uint64_t *)ctx->d_pick.p, *d_val = d_idx + m;
            HIP_TRY(hipMemcpyAsync(d_idx, idx.data(), m * 8, hipMemcpyHostToDevice, ds));
            HIP_TRY(launch_pick_u64(ds, d_soff, d_idx, d_val, (uint32_t)m));
            HIP_TRY(hipMemcpyAsync(val.data(), d_val, m * 8, hipMemcpyDeviceToHost, ds));
            HIP_TRY(hipStreamSynchronize(ds));
            for (size_t i = 0; i < m; i++)
                val[i] = want[i] >= N ? sel_bytes : val[i];
            for (size_t i = 0; i <= nout; i++)
                part_data[i] = val[i];
            seg_data.assign(val.begin() + (nout + 1), val.end());
        }
    }

    // Drain: gather the selected chunks, then copy them to pinned host memory.
    uint64_t n_timed = 0;   // segments with per-segment gather events
    if (!no_drain && sel_bytes && !graph_drain) {
        const uint64_t stage = segmented ? std::min<uint64_t>(sel_bytes, kSegSlots * slot_bytes) : sel_bytes;
        if (cfg.staging_budget && !direct && (incremental ? 0 : L.data_bytes) + stage > cfg.staging_budget)
            return set_error(CKPT_E_BUDGET, "drain staging %llu B exceeds the budget",
                             (unsigned long long)((incremental ? 0 : L.data_bytes) + stage));
        if (direct) {
            if (nout != 1)
                return set_error(CKPT_E_INVAL, "CKPT_DRAIN_DIRECT is not available for batches");
            CKPT_TRY(data[0].ensure(sel_bytes));
            d_out = (uint8_t *)data[0].p;
        } else {
            // with a reservation, after the dense image when that is the
            // context's staging
            CKPT_TRY(serial_staging(ctx, dense == (uint8_t *)ctx->d_dense.p ? L.data_bytes : 0, stage, &d_out));
            for (size_t i = 0; i < nout; i++)
                CKPT_TRY(data[i].ensure(part_data[i + 1] - part_data[i]));
        }
        GatherArgs ga;
        memset(&ga, 0, sizeof(ga));
        ga.plan = (const DevPlan *)ctx->d_plan.p;
        ga.mode = incremental ? kSelDirtyNonZero : kSelNonZero;
        ga.from_dense = incremental ? 0 : 1;
        ga.C = C;
        ga.src = (const uint64_t *)ctx->d_addr.p;
        ga.size = (const uint64_t *)ctx->d_size.p;
        ga.off = (const uint64_t *)ctx->d_off.p;
        ga.cb = (const uint64_t *)ctx->d_cb.p;
        ga.map = (const uint32_t *)ctx->d_map.p;
        ga.dense = dense;
        ga.flags = a.flags;
        ga.soff = d_soff;
        ga.out = d_out;
        ga.out_host = direct ? 1 : 0;
        if (segmented) {
            // The pack and the select are complete (the side stream was
            // synchronized above).  slot_full[j]: slot j gathered; slot_free[j]:
            // slot j copied out.
            CKPT_TRY(seg_events(ctx, 2 * kSegSlots + (timing ? 2 * n_seg : 0)));
            hipEvent_t *slot_full = ctx->seg_ev.data(), *slot_free = slot_full + kSegSlots;
            hipEvent_t *tev = slot_free + kSegSlots;
            hipStream_t gst = ctx->gat;
            uint64_t used = 0;
            for (uint64_t k = 0; k < n_seg; k++) {
                const uint64_t b0 = seg_data[k], b1 = seg_data[k + 1];
                if (b1 == b0)
                    continue;   // only ZERO chunks
                const int j = (int)(used % kSegSlots);
                if (used >= (uint64_t)kSegSlots)
                    HIP_TRY(hipStreamWaitEvent(gst, slot_free[j], 0));
                ga.g_begin = k * seg_chunks;
                ga.g_end = std::min<uint64_t>(N, (k + 1) * seg_chunks);
                ga.out = d_out + (uint64_t)j * slot_bytes;
                ga.soff_base = b0;
                if (timing)
                    HIP_TRY(hipEventRecord(tev[2 * used], gst));
                // One 1024-thread workgroup per CU: the runtime's copies to the
                // host are kernels too, and each of their workgroups holds a CU
                // slot for the whole copy.  A second gather workgroup per CU
                // would not fit beside one and would wait for the copy to end.
                HIP_TRY(launch_gather(gst, ga, ctx->cu_count));
                if (timing)
                    HIP_TRY(hipEventRecord(tev[2 * used + 1], gst));
                HIP_TRY(hipEventRecord(slot_full[j], gst));
                HIP_TRY(hipStreamWaitEvent(ds, slot_full[j], 0));
                if (timing && used == 0)
                    HIP_TRY(hipEventRecord(ctx->ev[7], ds));
                for (size_t i = 0; i < nout; i++) {   // the segment's bytes, cut at the outputs' bounds
                    const uint64_t lo = std::max(b0, part_data[i]), hi = std::min(b1, part_data[i + 1]);
                    if (lo < hi)
                        HIP_TRY(hipMemcpyAsync((uint8_t *)data[i].p + (lo - part_data[i]), ga.out + (lo - b0), hi - lo,
                                               hipMemcpyDeviceToHost, ds));
                }
                HIP_TRY(hipEventRecord(slot_free[j], ds));
                used++;
            }
            n_timed = timing ? used : 0;
            if (timing)
                HIP_TRY(hipEventRecord(ctx->ev[5], gst));
        } else {
            HIP_TRY(launch_gather(gs, ga, 2 * ctx->cu_count));
            if (incremental) {
                HIP_TRY(hipEventRecord(ctx->ev[3], s));   // delta taken: the caller's stream is free
                HIP_TRY(hipStreamWaitEvent(ds, ctx->ev[3], 0));
            }
            if (timing) {
                HIP_TRY(hipEventRecord(ctx->ev[5], gs));
                HIP_TRY(hipStreamWaitEvent(ds, ctx->ev[5], 0));
                HIP_TRY(hipEventRecord(ctx->ev[7], ds));
            }
            if (!direct)
                for (size_t i = 0; i < nout; i++) {
                    const uint64_t b = part_data[i + 1] - part_data[i];
                    if (b)
                        HIP_TRY(hipMemcpyAsync(data[i].p, d_out + part_data[i], b, hipMemcpyDeviceToHost, ds));
                }
        }
    } else {
        if (incremental) {
            HIP_TRY(hipEventRecord(ctx->ev[3], s));
            HIP_TRY(hipStreamWaitEvent(ds, ctx->ev[3], 0));
        }
        if (timing) {
            HIP_TRY(hipEventRecord(ctx->ev[5], gs));
            HIP_TRY(hipStreamWaitEvent(ds, ctx->ev[5], 0));
            HIP_TRY(hipEventRecord(ctx->ev[7], ds));
        }
    }

    // Metadata: CRC, flags, dirty ids, layout.
    std::vector<ckpt_image *> imgs(nout, nullptr);
    struct ImgGuard {
        std::vector<ckpt_image *> &v;
        bool keep = false;
        ~ImgGuard() { if (!keep) for (auto *p : v) delete p; }
    } img_guard{imgs};
    // one pinned block for every output's CRC and flags, filled by two copies
    auto meta = std::make_shared<PinnedBuf>();
    CKPT_TRY(meta->ensure(std::max<uint64_t>(5 * N, 8)));
    if (N) {
        const void *crc_src = snap ? ctx->d_prev_crc.p : ctx->d_crc.p;
        const void *flags_src = snap ? ctx->d_snap_flags.p : ctx->d_flags.p;
        HIP_TRY(hipMemcpyAsync(meta->p, crc_src, N * 4, hipMemcpyDeviceToHost, ds));
        HIP_TRY(hipMemcpyAsync((uint8_t *)meta->p + 4 * N, flags_src, N, hipMemcpyDeviceToHost, ds));
    }
    for (size_t i = 0; i < nout; i++) {
        auto *img = new ckpt_image();
        imgs[i] = img;
        img->device = cfg.device;
        img->mode = incremental ? CKPT_INCREMENTAL : CKPT_FULL;
        img->C = C;
        img->N = part_chunk[i + 1] - part_chunk[i];
        img->data_bytes = L.off[part_row[i + 1]] - L.off[part_row[i]];
        img->ser_bytes = part_data[i + 1] - part_data[i];
        img->serial = next_serial();
        img->base_serial = base ? base->serial : 0;
        img->drained = !no_drain;
        img->meta = meta;
        img->crc = (uint32_t *)meta->p + part_chunk[i];
        img->flags = (uint8_t *)meta->p + 4 * N + part_chunk[i];
        img->data = std::move(data[i]);
        const uint64_t r0 = part_row[i], r1 = part_row[i + 1];
        img->allocs.resize(r1 - r0);
        img->addrs.resize(r1 - r0);
        for (uint64_t k = r0; k < r1; k++) {
            img->addrs[k - r0] = rows[k].ptr;
            ckpt_alloc_rec &rec = img->allocs[k - r0];
            rec.id = rows[k].id;
            rec.kind = rows[k].kind;
            rec.pad = 0;
            rec.size = rows[k].size;
            rec.off = L.off[k] - L.off[r0];
            rec.cb = L.cb[k] - L.cb[r0];
        }
    }
    if (incremental) {
        imgs[0]->n_dirty = P.sel_count;
        CKPT_TRY(imgs[0]->ids_buf.ensure(std::max<uint64_t>(P.sel_count, 1) * 8));
        if (P.sel_count)
            HIP_TRY(hipMemcpyAsync(imgs[0]->ids_buf.p, ctx->d_ids.p, P.sel_count * 8, hipMemcpyDeviceToHost, ds));
    }
    // keep this CRC array on the device as the base of the next increment
    // (the snapshot already is)
    if (nout == 1 && N && !snap) {
        // on the side stream, after the earlier host copies that may read d_prev_crc
        CKPT_TRY(ctx->d_prev_crc.ensure(N * 4));
        HIP_TRY(hipMemcpyAsync(ctx->d_prev_crc.p, ctx->d_crc.p, N * 4, hipMemcpyDeviceToDevice, ds));
    }
    if (timing)
        HIP_TRY(hipEventRecord(ctx->ev[6], ds));
    // Without a drain the image is complete once the pack is: the CRC and
    // flag copies to the host finish on the side stream while the caller goes
    // on.  Each image waits for its own copy before it exposes host sections,
    // and the next call on this context orders its work after them.
    // (An increment's copies read d_crc / d_flags themselves, which the next
    // call overwrites, so an increment always waits for them.)
    const bool async_meta = no_drain && !incremental;
    if (async_meta) {
        auto ev = std::make_shared<MetaEvent>();
        HIP_TRY(hipEventCreateWithFlags(&ev->e, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(ev->e, ds));
        for (ckpt_image *img : imgs)
            img->meta_ready = ev;
        HIP_TRY(hipEventRecord(ctx->meta_ev, ds));
        ctx->meta_pending = true;
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        HIP_TRY(hipStreamSynchronize(ds));
        HIP_TRY(hipStreamSynchronize(s));
    }
    ctx->prev_serial = nout == 1 && N ? imgs[0]->serial : 0;

    if (timing) {
        T.layout_ms = graph ? 0.f : ev_ms(ctx->ev[0], ctx->ev[1]);
        T.pack_ms = graph ? ev_ms(ctx->ev[0], ctx->ev[2]) : ev_ms(ctx->ev[1], ctx->ev[2]);
        if (!async_meta) {
            T.select_ms = incremental ? ev_ms(ctx->ev[2], ctx->ev[4]) : ev_ms(ctx->ev[3], ctx->ev[4]);
            if (n_timed) {
                for (uint64_t u = 0; u < n_timed; u++)
                    T.gather_ms += ev_ms(ctx->seg_ev[2 * kSegSlots + 2 * u], ctx->seg_ev[2 * kSegSlots + 2 * u + 1]);
            } else {
                T.gather_ms = ev_ms(ctx->ev[4], ctx->ev[5]);
            }
            T.d2h_ms = ev_ms(ctx->ev[7], ctx->ev[6]);
        }
    }
    T.link_bytes = sel_bytes + 5 * N;
    T.total_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t_call).count();

    for (size_t i = 0; i < nout; i++) {
        ckpt_image *img = imgs[i];
        if (keep_dense && nout == 1) {
            img->dense = dense_owned;
            img->dense_owned = true;
            dense_guard.p = nullptr;
        } else if (no_drain) {
            // the context's staging: valid until its next checkpoint
            img->dense = dense + L.off[part_row[i]];
        }
        outs[i] = img;
    }
    img_guard.keep = true;
    return CKPT_OK;
}

extern "C" int ckpt_checkpoint(ckpt_ctx *ctx, void *stream, int mode, const ckpt_image *base, ckpt_image **out)
{
    if (!ctx || !out)
        return set_error(CKPT_E_INVAL, "ctx or out is NULL");
    if (mode != CKPT_FULL && mode != CKPT_INCREMENTAL)
        return set_error(CKPT_E_INVAL, "unknown mode %d", mode);
    if (mode == CKPT_INCREMENTAL && !base)
        return set_error(CKPT_E_INVAL, "an incremental checkpoint needs a base image");
    HookGuard hg(ctx);
    DeviceGuard g(ctx->cfg.device);
    if (!g.ok())
        return set_error(CKPT_E_HIP, "cannot select device %d", ctx->cfg.device);
    CKPT_TRY(ctx_ready(ctx));
    std::vector<Row> rows(ctx->live.begin(), ctx->live.end());
    std::vector<size_t> parts{0};
    std::vector<ckpt_image *> outs(1, nullptr);
    int rc = run_checkpoint(ctx, (hipStream_t)stream, mode, base, rows, parts, outs,
                            (ctx->cfg.flags & CKPT_GRAPH) != 0);
    if (rc == CKPT_OK)
        *out = outs[0];
    return rc;
}

extern "C" int ckpt_checkpoint_batch(ckpt_ctx *const *ctxs, size_t n, void *stream, ckpt_image **outs)
{
    if (!ctxs || !outs || n == 0)
        return set_error(CKPT_E_INVAL, "empty batch");
    ckpt_ctx *c0 = ctxs[0];
    const ckpt_ctx *hooked = nullptr;
    for (size_t i = 0; i < n; i++)
        if (ctxs[i] && ctxs[i]->hooked.load())
            hooked = ctxs[i];
    HookGuard hg(hooked);
    for (size_t i = 0; i < n; i++) {
        if (!ctxs[i])
            return set_error(CKPT_E_INVAL, "ctxs[%zu] is NULL", i);
        if (ctxs[i]->cfg.device != c0->cfg.device || ctxs[i]->cfg.chunk_bytes != c0->cfg.chunk_bytes)
            return set_error(CKPT_E_INVAL, "batched contexts differ in device or chunk size");
    }
    if (c0->cfg.flags & (CKPT_KEEP_DENSE | CKPT_DRAIN_DIRECT))
        return set_error(CKPT_E_INVAL, "batches keep no dense image and drain through staging");
    DeviceGuard g(c0->cfg.device);
    CKPT_TRY(ctx_ready(c0));
    std::vector<Row> rows;
    std::vector<size_t> parts(n);
    for (size_t i = 0; i < n; i++) {
        parts[i] = rows.size();
        rows.insert(rows.end(), ctxs[i]->live.begin(), ctxs[i]->live.end());
    }
    std::vector<ckpt_image *> o(n, nullptr);
    int rc = run_checkpoint(c0, (hipStream_t)stream, CKPT_FULL, nullptr, rows, parts, o,
                            !(c0->cfg.flags & CKPT_NO_GRAPH));
    if (rc == CKPT_OK)
        for (size_t i = 0; i < n; i++)
            outs[i] = o[i];
    return rc;
}

// ------------------------------------------------------------------ restore

extern "C" int ckpt_restore(ckpt_ctx *ctx, void *stream, const ckpt_image *img, const ckpt_image *delta,
                            void *const *dst, const size_t *dst_bytes, size_t n_dst, ckpt_verify_report *rep)
{
    return restore_impl(ctx, stream, img, delta, dst, dst_bytes, n_dst, rep, false);
}

int ckpt::restore_impl(ckpt_ctx *ctx, void *stream, const ckpt_image *img, const ckpt_image *delta,
                       void *const *dst, const size_t *dst_bytes, size_t n_dst, ckpt_verify_report *rep,
                       bool fresh_dst)
{
    if (!ctx || !img)
        return set_error(CKPT_E_INVAL, "ctx or image is NULL");
    if (!img->drained || img->mode != CKPT_FULL)
        return set_error(CKPT_E_INVAL, "restore needs a drained full image");
    if (img->C != ctx->cfg.chunk_bytes)
        return set_error(CKPT_E_MISMATCH, "image chunk size %u, context %u", img->C, ctx->cfg.chunk_bytes);
    if (delta && delta->mode == CKPT_INCREMENTAL && delta->drained && delta->base_serial == img->serial &&
        !same_table(img, delta)) {
        // the allocation table changed between the two: restore the merged image
        std::unique_ptr<ckpt_image> merged;
        CKPT_TRY(fold_delta(img, delta, &merged));
        return restore_impl(ctx, stream, merged.get(), nullptr, dst, dst_bytes, n_dst, rep, fresh_dst);
    }
    const uint64_t n = img->allocs.size();
    if (n_dst != n)
        return set_error(CKPT_E_MISMATCH, "%zu destinations for %llu allocations", n_dst, (unsigned long long)n);
    if (n && !dst)
        return set_error(CKPT_E_INVAL, "dst is NULL");
    std::vector<Row> rows(n);
    for (uint64_t k = 0; k < n; k++) {
        const uint64_t d = (uint64_t)(uintptr_t)dst[k], sz = img->allocs[k].size;
        if (dst_bytes && dst_bytes[k] != sz)
            return set_error(CKPT_E_MISMATCH, "dst[%llu] has %zu bytes, the allocation %llu", (unsigned long long)k,
                             dst_bytes[k], (unsigned long long)sz);
        if (d % 16 != 0 || (sz && d == 0))
            return set_error(CKPT_E_INVAL, "dst[%llu] is NULL or not 16-byte aligned", (unsigned long long)k);
        rows[k].id = img->allocs[k].id;
        rows[k].kind = img->allocs[k].kind;
        rows[k].ptr = d;
        rows[k].size = sz;
    }
    if (delta) {
        if (delta->mode != CKPT_INCREMENTAL || !delta->drained)
            return set_error(CKPT_E_INVAL, "delta is not a drained incremental image");
        if (delta->base_serial != img->serial || !same_table(img, delta))
            return set_error(CKPT_E_MISMATCH, "delta was not taken against this image");
        // ids index chunk arrays on the device: they must be ascending and < N
        const uint64_t *ids = (const uint64_t *)delta->ids_buf.p;
        for (uint64_t i = 0; i < delta->n_dirty; i++)
            if (ids[i] >= img->N || (i && ids[i] <= ids[i - 1]))
                return set_error(CKPT_E_INVAL, "delta id list is not ascending below %llu",
                                 (unsigned long long)img->N);
    }
    const uint64_t N = img->N;
    // The base image is refilled in segments of seg_chunks chunks: each
    // segment's copy to the device (side stream, into one of kSegSlots slots)
    // overlaps the scatter of earlier segments (on `stream`), and at most
    // kSegSlots segments are staged.
    const uint64_t seg_b = segment_bytes(ctx->cfg);
    const uint64_t seg_chunks = seg_b ? std::max<uint64_t>(1, seg_b / img->C) : 0;
    const uint64_t n_seg = seg_b && N ? (N + seg_chunks - 1) / seg_chunks : 0;
    bool segmented = n_seg > 1;
    // Destinations the caller has just mapped (a restore at the recorded
    // addresses that re-created them): a segmented refill measured 66 ms
    // slower there than into the same memory mapped earlier (16 GiB), and one
    // pass 4 ms -- new memory is readied before its first use, and one pass
    // copies the image to the device meanwhile.  One pass when its staging fits.
    if (segmented && fresh_dst) {
        const uint64_t whole = img->ser_bytes + (delta ? delta->ser_bytes : 0);
        const uint64_t room = ctx->reserved ? ctx->d_dense.cap : ctx->cfg.staging_budget;
        if (!room || whole <= room)
            segmented = false;
    }
    const uint64_t slot_bytes = seg_chunks * img->C;   // a segment's serialized bytes never exceed this
    const uint64_t base_stage = segmented ? std::min<uint64_t>(img->ser_bytes, kSegSlots * slot_bytes) : img->ser_bytes;
    const uint64_t stage = base_stage + (delta ? delta->ser_bytes : 0);
    if (ctx->cfg.staging_budget && stage > ctx->cfg.staging_budget)
        return set_error(CKPT_E_BUDGET, "restore staging %llu B exceeds the budget", (unsigned long long)stage);

    DeviceGuard g(ctx->cfg.device);
    CKPT_TRY(ctx_ready(ctx));
    hipStream_t s = (hipStream_t)stream;
    CKPT_TRY(order_after_meta(ctx, s));
    image_wait(img);
    if (delta)
        image_wait(delta);
    const bool timing = ctx->cfg.flags & CKPT_TIMING;
    ckpt_timing &T = ctx->timing;
    memset(&T, 0, sizeof(T));
    const auto t_call = std::chrono::steady_clock::now();

    if (timing)
        HIP_TRY(hipEventRecord(ctx->ev[0], s));
    CKPT_TRY(upload_table(ctx, s, rows, true, N, N));
    CKPT_TRY(ctx->d_crc.ensure(std::max<uint64_t>(N, 1) * 4));
    CKPT_TRY(ctx->d_flags.ensure(std::max<uint64_t>(N, 1)));
    CKPT_TRY(ctx->d_bad.ensure(std::max<uint64_t>(N, 1)));
    CKPT_TRY(ctx->d_soff.ensure(std::max<uint64_t>(N, 1) * 8));
    uint8_t *staging = nullptr;
    CKPT_TRY(serial_staging(ctx, 0, stage, &staging));
    if (N) {
        HIP_TRY(hipMemcpyAsync(ctx->d_crc.p, img->crc, N * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ctx->d_flags.p, img->flags, N, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_fill_u64(s, (uint64_t *)ctx->d_bad.p, (N + 7) / 8, 0));
    }
    if (img->ser_bytes && !segmented)
        HIP_TRY(hipMemcpyAsync(staging, img->data.p, img->ser_bytes, hipMemcpyHostToDevice, s));
    if (timing)
        HIP_TRY(hipEventRecord(ctx->ev[1], s));

    ChunkArgs a = chunk_args(ctx);
    a.dst = (const uint64_t *)ctx->d_addr.p;
    a.staging = staging;
    a.soff = (const uint64_t *)ctx->d_soff.p;
    a.want_crc = (const uint32_t *)ctx->d_crc.p;
    a.want_flags = (const uint8_t *)ctx->d_flags.p;
    a.zero_crc = ctx->zero_crc;
    a.bad = (uint8_t *)ctx->d_bad.p;
    DevPlan P;
    if (N) {
        CKPT_TRY(run_select(ctx, s, kSelNonZero, (const uint8_t *)ctx->d_flags.p, nullptr, N,
                            (uint64_t *)ctx->d_soff.p, nullptr, 0));
        // The flags decide which chunks are read from staging: they must account
        // for exactly the serialized bytes, or the scatter would read past them.
        CKPT_TRY(read_plan(ctx, s, &P));
        if (P.sel_bytes != img->ser_bytes)
            return set_error(CKPT_E_INVAL, "flags select %llu serialized bytes, image holds %llu",
                             (unsigned long long)P.sel_bytes, (unsigned long long)img->ser_bytes);
        if (!segmented) {
            HIP_TRY(launch_chunks(s, kModeRestore, a, ctx->grid_chunks, ctx->cfg.block_threads));
        } else {
            // serialized offset of each segment's first chunk
            std::vector<uint64_t> idx(n_seg + 1), seg_data(n_seg + 1);
            for (uint64_t k = 0; k <= n_seg; k++)
                idx[k] = std::min<uint64_t>(k * seg_chunks, N - 1);
            CKPT_TRY(ctx->d_pick.ensure((n_seg + 1) * 16));
            uint64_t *d_idx = (uint64_t *)ctx->d_pick.p, *d_val = d_idx + n_seg + 1;
            HIP_TRY(hipMemcpyAsync(d_idx, idx.data(), (n_seg + 1) * 8, hipMemcpyHostToDevice, s));
            HIP_TRY(launch_pick_u64(s, (const uint64_t *)ctx->d_soff.p, d_idx, d_val, (uint32_t)(n_seg + 1)));
            HIP_TRY(hipMemcpyAsync(seg_data.data(), d_val, (n_seg + 1) * 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            seg_data[n_seg] = img->ser_bytes;
            // slot_full[j]: slot j copied in; slot_free[j]: slot j scattered
            CKPT_TRY(seg_events(ctx, 2 * kSegSlots + (timing ? 2 * n_seg : 0)));
            hipEvent_t *slot_full = ctx->seg_ev.data(), *slot_free = slot_full + kSegSlots;
            hipEvent_t *tev = slot_free + kSegSlots;
            hipStream_t cs = ctx->side;
            HIP_TRY(hipEventRecord(ctx->ev[3], s));   // the staging's earlier readers are done
            HIP_TRY(hipStreamWaitEvent(cs, ctx->ev[3], 0));
            if (timing)
                HIP_TRY(hipEventRecord(ctx->ev[7], cs));
            for (uint64_t k = 0; k < n_seg; k++) {
                const uint64_t b0 = seg_data[k], b1 = seg_data[k + 1];
                const int j = (int)(k % kSegSlots);
                if (k >= (uint64_t)kSegSlots)
                    HIP_TRY(hipStreamWaitEvent(cs, slot_free[j], 0));
                uint8_t *slot = staging + (uint64_t)j * slot_bytes;
                if (b1 > b0)
                    HIP_TRY(hipMemcpyAsync(slot, (const uint8_t *)img->data.p + b0, b1 - b0, hipMemcpyHostToDevice, cs));
                HIP_TRY(hipEventRecord(slot_full[j], cs));
                HIP_TRY(hipStreamWaitEvent(s, slot_full[j], 0));
                ChunkArgs sa = a;
                sa.item_begin = k * seg_chunks;
                sa.item_end = std::min<uint64_t>(N, (k + 1) * seg_chunks);
                sa.staging = slot;
                sa.soff_base = b0;
                if (timing)
                    HIP_TRY(hipEventRecord(tev[2 * k], s));
                HIP_TRY(launch_chunks(s, kModeRestore, sa, ctx->grid_chunks, ctx->cfg.block_threads));
                if (timing)
                    HIP_TRY(hipEventRecord(tev[2 * k + 1], s));
                HIP_TRY(hipEventRecord(slot_free[j], s));
            }
            if (timing)
                HIP_TRY(hipEventRecord(ctx->ev[6], cs));
        }
    } else if (img->ser_bytes) {
        return set_error(CKPT_E_INVAL, "image without chunks holds serialized bytes");
    }
    if (delta && delta->n_dirty) {
        const uint64_t nd = delta->n_dirty;
        CKPT_TRY(ctx->d_crc2.ensure(std::max<uint64_t>(N, 1) * 4));
        CKPT_TRY(ctx->d_flags2.ensure(std::max<uint64_t>(N, 1)));
        CKPT_TRY(ctx->d_ids.ensure(nd * 8));
        CKPT_TRY(ctx->d_soff2.ensure(nd * 8));
        if (timing)
            HIP_TRY(hipEventRecord(ctx->ev[4], s));
        uint8_t *staging2 = staging + base_stage;
        HIP_TRY(hipMemcpyAsync(ctx->d_crc2.p, delta->crc, N * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ctx->d_flags2.p, delta->flags, N, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ctx->d_ids.p, delta->ids_buf.p, nd * 8, hipMemcpyHostToDevice, s));
        if (delta->ser_bytes)
            HIP_TRY(hipMemcpyAsync(staging2, delta->data.p, delta->ser_bytes, hipMemcpyHostToDevice, s));
        // n_items = the delta's id count (plan field written from pinned memory)
        auto *hp = (DevPlan *)ctx->h_plan.p;
        HIP_TRY(hipStreamSynchronize(s));   // h_plan is reused below; keep the copy ordered
        hp->n_items = nd;
        HIP_TRY(hipMemcpyAsync((uint8_t *)ctx->d_plan.p + offsetof(DevPlan, n_items), &hp->n_items, 8,
                               hipMemcpyHostToDevice, s));
        CKPT_TRY(run_select(ctx, s, kSelIdsNonZero, (const uint8_t *)ctx->d_flags2.p, (const uint64_t *)ctx->d_ids.p,
                            nd, (uint64_t *)ctx->d_soff2.p, nullptr, 0));
        CKPT_TRY(read_plan(ctx, s, &P));
        if (P.sel_bytes != delta->ser_bytes)
            return set_error(CKPT_E_INVAL, "delta flags select %llu bytes, delta holds %llu",
                             (unsigned long long)P.sel_bytes, (unsigned long long)delta->ser_bytes);
        ChunkArgs b = a;
        b.staging = staging2;
        b.soff = (const uint64_t *)ctx->d_soff2.p;
        b.want_crc = (const uint32_t *)ctx->d_crc2.p;
        b.want_flags = (const uint8_t *)ctx->d_flags2.p;
        b.ids = (const uint64_t *)ctx->d_ids.p;
        HIP_TRY(launch_chunks(s, kModeRestore, b, ctx->grid_chunks, ctx->cfg.block_threads));
    }
    if (timing)
        HIP_TRY(hipEventRecord(ctx->ev[2], s));
    CKPT_TRY(read_plan(ctx, s, &P));
    uint64_t n_bad = 0, n_ids = 0;
    uint64_t ids[CKPT_REPORT_MAX];
    if (P.bad_count) {
        CKPT_TRY(ctx->d_ids.ensure(CKPT_REPORT_MAX * 8));
        CKPT_TRY(run_select(ctx, s, kSelBad, (const uint8_t *)ctx->d_bad.p, nullptr, N, nullptr,
                            (uint64_t *)ctx->d_ids.p, CKPT_REPORT_MAX));
        CKPT_TRY(read_plan(ctx, s, &P));
        n_bad = P.sel_count;
        n_ids = std::min<uint64_t>(n_bad, CKPT_REPORT_MAX);
        HIP_TRY(hipMemcpy(ids, ctx->d_ids.p, n_ids * 8, hipMemcpyDeviceToHost));
    }
    if (timing) {
        if (segmented) {
            T.h2d_ms = ev_ms(ctx->ev[7], ctx->ev[6]);
            for (uint64_t k = 0; k < n_seg; k++)
                T.scatter_ms += ev_ms(ctx->seg_ev[2 * kSegSlots + 2 * k], ctx->seg_ev[2 * kSegSlots + 2 * k + 1]);
            if (delta && delta->n_dirty)
                T.scatter_ms += ev_ms(ctx->ev[4], ctx->ev[2]);
        } else {
            T.h2d_ms = ev_ms(ctx->ev[0], ctx->ev[1]);
            T.scatter_ms = ev_ms(ctx->ev[1], ctx->ev[2]);
        }
    }
    T.link_bytes = stage + 5 * N;
    T.total_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t_call).count();
    if (rep) {
        memset(rep, 0, sizeof(*rep));
        rep->n_bad = n_bad;
        rep->n_ids = n_ids;
        memcpy(rep->ids, ids, n_ids * 8);
    }
    return n_bad ? set_error(CKPT_E_CORRUPT, "%llu chunks failed verification", (unsigned long long)n_bad)
                 : CKPT_OK;
}

// -------------------------------------------------------------------- image

// --------------------------------------------------------------- merging
//
// A full image and an incremental image taken against it fold into the full
// image a checkpoint would have produced at the increment's time: the
// increment's allocation table, CRC and flags (every chunk DIRTY, as in a
// full image without a base), and each non-ZERO chunk's bytes from the
// increment when it is DIRTY there, else from the same chunk of the base
// allocation with the same id.  All on the host, from the images' DATA.
extern "C" int ckpt_image_merge(const ckpt_image *base, const ckpt_image *delta, ckpt_image **out)
{
    if (!base || !delta || !out)
        return set_error(CKPT_E_INVAL, "NULL argument");
    image_wait(base);
    image_wait(delta);
    if (!base->drained || !delta->drained)
        return set_error(CKPT_E_INVAL, "merging needs images with host DATA");
    if (base->mode != CKPT_FULL || delta->mode != CKPT_INCREMENTAL)
        return set_error(CKPT_E_INVAL, "merge takes a full image and an incremental image");
    if (delta->base_serial != base->serial || delta->C != base->C)
        return set_error(CKPT_E_MISMATCH, "the incremental image was not taken against this base");
    const uint32_t C = delta->C;
    const uint64_t n = delta->allocs.size(), N = delta->N, bn = base->allocs.size();

    // base: the serialized offset of each chunk (ZERO chunks have none)
    std::vector<uint64_t> boff(base->N + 1, 0);
    for (uint64_t j = 0, g = 0, o = 0; j < bn; j++) {
        const uint64_t sz = base->allocs[j].size;
        for (uint64_t c = 0; c * C < sz; c++, g++) {
            boff[g] = o;
            if (!(base->flags[g] & kFlagZero))
                o += ru16(std::min<uint64_t>(C, sz - c * C));
        }
    }
    // the source of every chunk of the result: 0 none (ZERO), 1 delta, 2 base
    struct Src {
        uint64_t off, len;   // offset in the source DATA, bytes (a multiple of 16)
        uint8_t from;
    };
    std::vector<Src> src(N);
    uint64_t total = 0, doff = 0;
    size_t j = 0;
    for (uint64_t k = 0, g = 0; k < n; k++) {
        const ckpt_alloc_rec &r = delta->allocs[k];
        while (j < bn && base->allocs[j].id < r.id)
            j++;
        const bool matched =
            j < bn && base->allocs[j].id == r.id && base->allocs[j].size == r.size && base->allocs[j].kind == r.kind;
        for (uint64_t c = 0; c * C < r.size; c++, g++) {
            const uint64_t len = ru16(std::min<uint64_t>(C, r.size - c * C));
            const uint8_t f = delta->flags[g];
            Src &x = src[g];
            x.len = len;
            if (f & kFlagZero) {
                x.from = 0;
                x.len = 0;
            } else if (f & kFlagDirty) {
                x.from = 1;
                x.off = doff;
                doff += len;
            } else {
                const uint64_t bg = matched ? base->allocs[j].cb + c : kNoBase;
                if (bg == kNoBase || (base->flags[bg] & kFlagZero) || base->crc[bg] != delta->crc[g])
                    return set_error(CKPT_E_CORRUPT, "chunk %llu is clean in the increment but has no equal base chunk",
                                     (unsigned long long)g);
                x.from = 2;
                x.off = boff[bg];
            }
            total += x.len;
        }
    }
    if (doff != delta->ser_bytes)
        return set_error(CKPT_E_CORRUPT, "increment DATA holds %llu bytes, its flags describe %llu",
                         (unsigned long long)delta->ser_bytes, (unsigned long long)doff);

    auto *img = new ckpt_image();
    std::unique_ptr<ckpt_image> guard(img);
    img->device = delta->device;
    img->mode = CKPT_FULL;
    img->C = C;
    img->N = N;
    img->data_bytes = delta->data_bytes;
    img->ser_bytes = total;
    // the merged image stands for the increment's state (same CRC array), so
    // it takes the increment's serial: an increment taken against the
    // increment can be merged into it next
    img->serial = delta->serial;
    img->base_serial = 0;
    img->drained = true;
    img->allocs = delta->allocs;
    img->addrs = delta->addrs;
    CKPT_TRY(alloc_meta(img, N));
    if (N) {
        memcpy(img->crc, delta->crc, N * 4);
        for (uint64_t g = 0; g < N; g++)
            img->flags[g] = (uint8_t)((delta->flags[g] & kFlagZero) | kFlagDirty);
    }
    CKPT_TRY(img->ids_buf.ensure(8));
    CKPT_TRY(img->data.ensure(std::max<uint64_t>(total, 1)));
    // copy in parallel over contiguous chunk ranges
    const unsigned T = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(8, total >> 26));
    std::vector<uint64_t> start(T + 1, 0), out_off(T + 1, 0);
    for (unsigned t = 0; t <= T; t++)
        start[t] = N * t / T;
    for (unsigned t = 0; t < T; t++) {
        uint64_t o = 0;
        for (uint64_t g = start[t]; g < start[t + 1]; g++)
            o += src[g].len;
        out_off[t + 1] = out_off[t] + o;
    }
    auto copy_range = [&](unsigned t) {
        uint8_t *dst = (uint8_t *)img->data.p + out_off[t];
        for (uint64_t g = start[t]; g < start[t + 1]; g++) {
            const Src &x = src[g];
            if (x.from == 0)
                continue;
            const uint8_t *from = (const uint8_t *)(x.from == 1 ? delta->data.p : base->data.p) + x.off;
            memcpy(dst, from, x.len);
            dst += x.len;
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < T; t++)
        pool.emplace_back(copy_range, t);
    copy_range(0);
    for (auto &th : pool)
        th.join();
    *out = guard.release();
    return CKPT_OK;
}

int ckpt::fold_delta(const ckpt_image *img, const ckpt_image *delta, std::unique_ptr<ckpt_image> *merged)
{
    merged->reset();
    if (!img || !delta || same_table(img, delta))
        return CKPT_OK;
    ckpt_image *m = nullptr;
    CKPT_TRY(ckpt_image_merge(img, delta, &m));
    merged->reset(m);
    return CKPT_OK;
}

extern "C" int ckpt_image_info(const ckpt_image *img, ckpt_image_meta *out)
{
    if (!img || !out)
        return set_error(CKPT_E_INVAL, "image or out is NULL");
    image_wait(img);
    memset(out, 0, sizeof(*out));
    out->mode = img->mode;
    out->chunk_bytes = img->C;
    out->n_allocs = img->allocs.size();
    out->n_chunks = img->N;
    out->data_bytes = img->data_bytes;
    out->serialized_bytes = img->ser_bytes;
    out->n_dirty = img->n_dirty;
    out->serial = img->serial;
    out->base_serial = img->base_serial;
    out->crc_digest = crc_digest(img->crc, img->N * 4);
    out->has_dense = img->dense != nullptr;
    out->drained = img->drained;
    return CKPT_OK;
}

extern "C" int ckpt_image_view(const ckpt_image *img, int section, const void **p, size_t *bytes)
{
    if (!img || !p || !bytes)
        return set_error(CKPT_E_INVAL, "NULL argument");
    image_wait(img);
    switch (section) {
    case CKPT_SEC_ALLOCS:
        *p = img->allocs.empty() ? nullptr : img->allocs.data();
        *bytes = img->allocs.size() * sizeof(ckpt_alloc_rec);
        break;
    case CKPT_SEC_CRC:
        *p = img->N ? img->crc : nullptr;
        *bytes = img->N * 4;
        break;
    case CKPT_SEC_FLAGS:
        *p = img->N ? img->flags : nullptr;
        *bytes = img->N;
        break;
    case CKPT_SEC_DATA:
        *p = img->ser_bytes ? img->data.p : nullptr;
        *bytes = img->ser_bytes;
        break;
    case CKPT_SEC_DIRTY_IDS:
        *p = img->n_dirty ? img->ids_buf.p : nullptr;
        *bytes = img->n_dirty * 8;
        break;
    case CKPT_SEC_DENSE:
        *p = img->dense;
        *bytes = img->dense ? img->data_bytes : 0;
        break;
    case CKPT_SEC_ADDRS:
        *p = img->addrs.empty() ? nullptr : img->addrs.data();
        *bytes = img->addrs.size() * 8;
        break;
    default:
        return set_error(CKPT_E_INVAL, "unknown section %d", section);
    }
    return CKPT_OK;
}

// Serialized form, all little-endian:
//   header (kHeaderBytes): magic "CKPTIMG1", version, mode, C, align (16),
//   n, N, data_bytes, ser_bytes, n_dirty, serial, base_serial, digest
//   ALLOCS n x 40, ADDRS n x 8 (version 2 on), CRC N x 4, FLAGS N (padded
//   to 8), DIRTY_IDS n_dirty x 8, DATA.  Version 1 data (no ADDRS) still loads,
//   with every address 0.
namespace {
constexpr char kMagic[8] = {'C', 'K', 'P', 'T', 'I', 'M', 'G', '1'};
constexpr uint32_t kVersion = 2;
constexpr size_t kHeaderBytes = 8 + 4 * 4 + 8 * 8;
size_t pad8(size_t x) { return (x + 7) & ~size_t(7); }

size_t serialized_size(uint32_t version, uint64_t n, uint64_t N, uint64_t n_dirty, uint64_t ser)
{
    return kHeaderBytes + n * sizeof(ckpt_alloc_rec) + (version >= 2 ? n * 8 : 0) + N * 4 + pad8(N) +
           n_dirty * 8 + ser;
}
}  // namespace

size_t ckpt::serialized_head_bytes(const ckpt_image *img)
{
    return serialized_size(kVersion, img->allocs.size(), img->N, img->n_dirty, 0);
}

void ckpt::serialize_head(const ckpt_image *img, uint8_t *p)
{
    const uint64_t n = img->allocs.size();
    memcpy(p, kMagic, 8);
    uint32_t h32[4] = {kVersion, img->mode, img->C, 16};
    memcpy(p + 8, h32, 16);
    uint64_t h64[8] = {n, img->N, img->data_bytes, img->ser_bytes, img->n_dirty, img->serial, img->base_serial,
                       crc_digest(img->crc, img->N * 4)};
    memcpy(p + 24, h64, 64);
    p += kHeaderBytes;
    if (n)
        memcpy(p, img->allocs.data(), n * sizeof(ckpt_alloc_rec));
    p += n * sizeof(ckpt_alloc_rec);
    for (uint64_t k = 0; k < n; k++) {
        const uint64_t a = k < img->addrs.size() ? img->addrs[k] : 0;
        memcpy(p + 8 * k, &a, 8);
    }
    p += n * 8;
    if (img->N) {
        memcpy(p, img->crc, img->N * 4);
        memcpy(p + img->N * 4, img->flags, img->N);
    }
    memset(p + img->N * 4 + img->N, 0, pad8(img->N) - img->N);
    p += img->N * 4 + pad8(img->N);
    if (img->n_dirty)
        memcpy(p, img->ids_buf.p, img->n_dirty * 8);
}

extern "C" int ckpt_image_serialize(const ckpt_image *img, void *buf, size_t cap, size_t *need)
{
    if (!img || !need)
        return set_error(CKPT_E_INVAL, "NULL argument");
    image_wait(img);
    if (!img->drained)
        return set_error(CKPT_E_INVAL, "image holds no host data");
    const size_t head = serialized_head_bytes(img);
    const size_t total = head + img->ser_bytes;
    *need = total;
    if (!buf)
        return CKPT_OK;
    if (cap < total)
        return set_error(CKPT_E_INVAL, "buffer holds %zu of %zu bytes", cap, total);
    serialize_head(img, (uint8_t *)buf);
    if (img->ser_bytes)
        memcpy((uint8_t *)buf + head, img->data.p, img->ser_bytes);
    return CKPT_OK;
}

int ckpt::head_layout(const void *hdr, size_t hdr_bytes, uint64_t avail, uint64_t *head_bytes, uint64_t *ser_bytes)
{
    if (hdr_bytes < kHeaderBytes || avail < kHeaderBytes)
        return set_error(CKPT_E_INVAL, "truncated image header (%llu bytes)",
                         (unsigned long long)std::min<uint64_t>(hdr_bytes, avail));
    const uint8_t *p = (const uint8_t *)hdr;
    if (memcmp(p, kMagic, 8) != 0)
        return set_error(CKPT_E_INVAL, "bad magic");
    uint32_t h32[4];
    uint64_t h64[8];
    memcpy(h32, p + 8, 16);
    memcpy(h64, p + 24, 64);
    if ((h32[0] != 1 && h32[0] != 2) || (h32[1] != CKPT_FULL && h32[1] != CKPT_INCREMENTAL) || h32[2] == 0 ||
        h32[2] % 16 != 0 || h32[3] != 16)
        return set_error(CKPT_E_INVAL, "bad header fields");
    const uint64_t n = h64[0], N = h64[1], nd = h64[4], ser = h64[3];
    // bound every count by the image's size before multiplying
    if (n > avail / sizeof(ckpt_alloc_rec) || N > avail / 5 || nd > avail / 8 || ser > avail)
        return set_error(CKPT_E_INVAL, "truncated image");
    const uint64_t total = serialized_size(h32[0], n, N, nd, ser);
    if (avail < total)
        return set_error(CKPT_E_INVAL, "truncated image: %llu of %llu bytes", (unsigned long long)avail,
                         (unsigned long long)total);
    *head_bytes = total - ser;
    *ser_bytes = ser;
    return CKPT_OK;
}

int ckpt::parse_head(const void *buf, size_t bytes, ImageHead *h, uint64_t data_apart)
{
    uint64_t head = 0, ser = 0;
    CKPT_TRY(head_layout(buf, bytes, bytes + data_apart, &head, &ser));
    if (data_apart && (data_apart != ser || bytes < head))
        return set_error(CKPT_E_INVAL, "image sections do not match the header");
    const uint8_t *p = (const uint8_t *)buf;
    uint32_t h32[4];
    uint64_t h64[8];
    memcpy(h32, p + 8, 16);
    memcpy(h64, p + 24, 64);
    const uint64_t n = h64[0];
    h->version = h32[0];
    h->mode = h32[1];
    h->C = h32[2];
    h->N = h64[1];
    h->data_bytes = h64[2];
    h->ser_bytes = ser;
    h->n_dirty = h64[4];
    h->serial = h64[5];
    h->base_serial = h64[6];
    h->digest = h64[7];
    h->head_bytes = head;
    p += kHeaderBytes;
    h->allocs.resize(n);
    if (n)
        memcpy(h->allocs.data(), p, n * sizeof(ckpt_alloc_rec));
    p += n * sizeof(ckpt_alloc_rec);
    // the table must be self-consistent: offsets and chunk bases are prefix sums
    uint64_t o = 0, g = 0;
    for (uint64_t k = 0; k < n; k++) {
        const ckpt_alloc_rec &r = h->allocs[k];
        if (r.off != o || r.cb != g || (r.kind != CKPT_DEVICE && r.kind != CKPT_MANAGED))
            return set_error(CKPT_E_INVAL, "inconsistent allocation table at row %llu", (unsigned long long)k);
        o += ru16(r.size);
        g += (r.size + h->C - 1) / h->C;
    }
    if (o != h->data_bytes || g != h->N)
        return set_error(CKPT_E_INVAL, "allocation table does not match the header totals");
    h->addrs.assign(n, 0);
    if (h->version >= 2) {
        if (n)
            memcpy(h->addrs.data(), p, n * 8);
        p += n * 8;
    }
    h->rest = p;
    return CKPT_OK;
}

int ckpt::image_from_head(ckpt_ctx *ctx, ImageHead *h, ckpt_image **out)
{
    auto *img = new ckpt_image();
    std::unique_ptr<ckpt_image> guard(img);
    img->device = ctx ? ctx->cfg.device : 0;
    img->mode = h->mode;
    img->C = h->C;
    img->N = h->N;
    img->data_bytes = h->data_bytes;
    img->ser_bytes = h->ser_bytes;
    img->n_dirty = h->n_dirty;
    img->serial = h->serial;
    img->base_serial = h->base_serial;
    img->drained = true;
    img->allocs = std::move(h->allocs);
    img->addrs = std::move(h->addrs);
    const uint8_t *p = h->rest;
    const uint64_t N = h->N, nd = h->n_dirty, ser = h->ser_bytes;
    CKPT_TRY(alloc_meta(img, N));
    if (N) {
        memcpy(img->crc, p, N * 4);
        memcpy(img->flags, p + N * 4, N);
    }
    p += N * 4 + pad8(N);
    CKPT_TRY(img->ids_buf.ensure(std::max<uint64_t>(nd, 1) * 8));
    if (nd)
        memcpy(img->ids_buf.p, p, nd * 8);
    if (crc_digest(img->crc, N * 4) != h->digest)
        return set_error(CKPT_E_INVAL, "CRC section digest mismatch");
    CKPT_TRY(img->data.ensure(std::max<uint64_t>(ser, 1)));
    *out = guard.release();
    return CKPT_OK;
}

extern "C" int ckpt_image_load(ckpt_ctx *ctx, const void *buf, size_t bytes, ckpt_image **out)
{
    if (!buf || !out)
        return set_error(CKPT_E_INVAL, "NULL argument");
    ImageHead h;
    CKPT_TRY(parse_head(buf, bytes, &h));
    ckpt_image *img = nullptr;
    CKPT_TRY(image_from_head(ctx, &h, &img));
    if (h.ser_bytes)
        memcpy(img->data.p, (const uint8_t *)buf + h.head_bytes, h.ser_bytes);
    *out = img;
    return CKPT_OK;
}

extern "C" void ckpt_image_free(ckpt_image *img) { delete img; }
