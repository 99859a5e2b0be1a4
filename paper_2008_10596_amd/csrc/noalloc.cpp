// noalloc.cpp -- ckpt_checkpoint_noalloc: the device pass of a checkpoint
// (size scan, chunk map, fused pack + CRC-32C + flags, or the hash-only pass)
// into buffers the caller passes, for callers that cannot allocate.
//
// ckpt_checkpoint keeps its descriptor tables in device buffers it grows on
// demand.  This variant takes them from one file-scope device array instead:
// the plan header, the uploaded allocation table, its address and size
// arrays, the prefix sums and the chunk -> allocation map.  The array holds at
// most kNaMaxAllocs allocations and kNaMaxChunks chunks; each device the
// library runs on keeps its own copy until the process ends.  Host code must
// never hand the array's name to a kernel or a copy (on the host it names a
// stand-in, not device memory): ckpt_init looks up each device's address once
// with hipGetSymbolAddress, and every use goes through that address.
#include <cstddef>
#include <cstring>
#include <mutex>

#include "ckpt.h"
#include "ckpt_runtime.h"

using namespace ckpt;

namespace {

constexpr uint64_t a256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

constexpr uint64_t kNaMaxAllocs = 65536;
constexpr uint64_t kNaMaxChunks = uint64_t(1) << 23;
constexpr uint64_t kRowBytes = 32;   // the host table's rows: id, kind, address, size

// Parts of the array, 256-byte aligned.
constexpr uint64_t kOffPlan = 0;
constexpr uint64_t kOffRows = a256(sizeof(DevPlan));
constexpr uint64_t kOffAddr = kOffRows + a256(kRowBytes * kNaMaxAllocs);
constexpr uint64_t kOffSize = kOffAddr + a256(8 * kNaMaxAllocs);
constexpr uint64_t kOffOff = kOffSize + a256(8 * kNaMaxAllocs);
constexpr uint64_t kOffCb = kOffOff + a256(8 * (kNaMaxAllocs + 1));
constexpr uint64_t kOffMap = kOffCb + a256(8 * (kNaMaxAllocs + 1));
constexpr uint64_t kScratchBytes = kOffMap + a256(4 * kNaMaxChunks);   // 36 MiB

static_assert(sizeof(Row) == kRowBytes && offsetof(Row, ptr) == 16 && offsetof(Row, size) == 24,
              "k_table_split reads the address and size at words 2 and 3 of each row");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t *g_scratch[kMaxDevices];   // each device's address of `scratch`

}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Called by ckpt_init with `device` current.
int ckpt::noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return set_error(CKPT_E_INVAL, "device %d: the allocation-free path serves devices 0..%d", device,
                         kMaxDevices - 1);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device])
        return CKPT_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return hip_fail(e, "hipGetSymbolAddress(scratch)", __LINE__);
    if (!p)
        return set_error(CKPT_E_HIP, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch[device] = (uint8_t *)p;
    return CKPT_OK;
}

extern "C" int ckpt_checkpoint_noalloc(ckpt_ctx *ctx, void *stream, int mode, const uint32_t *base_crc,
                                       void *dense, uint64_t dense_bytes, uint32_t *crc, uint8_t *flags,
                                       uint64_t chunk_cap, uint64_t *n_chunks, uint64_t *data_bytes)
{
    if (!ctx)
        return set_error(CKPT_E_INVAL, "ctx is NULL");
    HookGuard hg(ctx);
    const ckpt_config &cfg = ctx->cfg;
    if (mode != CKPT_FULL && mode != CKPT_INCREMENTAL)
        return set_error(CKPT_E_INVAL, "unknown mode %d", mode);
    if (mode == CKPT_INCREMENTAL && !base_crc)
        return set_error(CKPT_E_INVAL, "an incremental pass needs the base's CRC array");
    uint8_t *sp = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        sp = cfg.device >= 0 && cfg.device < kMaxDevices ? g_scratch[cfg.device] : nullptr;
    }
    if (!sp)
        return set_error(CKPT_E_INVAL, "the device array of device %d was not set up", cfg.device);

    // The layout's totals on the host, from the log (no allocation).
    const uint32_t C = cfg.chunk_bytes;
    const uint64_t n = ctx->live.size();
    uint64_t N = 0, D = 0;
    for (const Reg &r : ctx->live) {
        N += (r.size + C - 1) / C;
        D += (r.size + 15) & ~uint64_t(15);
    }
    if (n > kNaMaxAllocs || N > kNaMaxChunks)
        return set_error(CKPT_E_BUDGET,
                         "%llu allocations and %llu chunks; the allocation-free path holds at most %llu "
                         "allocations and %llu chunks",
                         (unsigned long long)n, (unsigned long long)N, (unsigned long long)kNaMaxAllocs,
                         (unsigned long long)kNaMaxChunks);
    const bool pack = mode == CKPT_FULL;
    if ((pack && dense_bytes < D) || chunk_cap < N) {
        if (n_chunks)
            *n_chunks = N;
        if (data_bytes)
            *data_bytes = D;
        return set_error(CKPT_E_MISMATCH, "outputs hold %llu dense bytes and %llu chunks; the pass needs %llu and %llu",
                         (unsigned long long)dense_bytes, (unsigned long long)chunk_cap,
                         (unsigned long long)(pack ? D : 0), (unsigned long long)N);
    }
    if ((pack && D && (!dense || (uintptr_t)dense % 16)) || (N && (!crc || !flags || (uintptr_t)crc % 4)) ||
        (base_crc && (uintptr_t)base_crc % 4))
        return set_error(CKPT_E_INVAL, "NULL or misaligned output (dense: 16 bytes, crc and base_crc: 4 bytes)");

    hipStream_t s = (hipStream_t)stream;
    DeviceGuard g(cfg.device);
    if (!(cfg.flags & CKPT_STREAM_ORDERED))
        HIP_TRY(hipDeviceSynchronize());
    if (ctx->managed_prefetch)
        for (const Reg &r : ctx->live)
            if (r.kind == CKPT_MANAGED && r.size)
                HIP_TRY(hipMemPrefetchAsync((const void *)r.ptr, r.size, cfg.device, s));

    auto *plan = (DevPlan *)(sp + kOffPlan);
    auto *rows = (uint64_t *)(sp + kOffRows);
    auto *addr = (uint64_t *)(sp + kOffAddr);
    auto *size = (uint64_t *)(sp + kOffSize);
    auto *off = (uint64_t *)(sp + kOffOff);
    auto *cb = (uint64_t *)(sp + kOffCb);
    auto *map = (uint32_t *)(sp + kOffMap);
    // Every part is rewritten before it is read: the table (n rows), the plan
    // (k_table_split), off/cb (scan), map (every chunk id below N).
    if (n)
        HIP_TRY(hipMemcpyAsync(rows, ctx->live.data(), n * kRowBytes, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_table_split(s, rows, n, plan, addr, size));
    HIP_TRY(launch_layout_scan(s, plan, size, C, off, cb));
    if (N) {
        HIP_TRY(launch_chunk_map(s, plan, cb, map, ctx->grid_small));
        ChunkArgs a;
        memset(&a, 0, sizeof(a));
        a.plan = plan;
        a.plan_rw = plan;
        a.tables = ctx->tables;
        a.tables_quad = ctx->tables + kRepWords;
        a.C = C;
        a.waves_per_chunk = cfg.waves_per_chunk;
        a.nontemporal = cfg.load_hint == 2;
        a.zero_crc = ctx->zero_crc;
        a.src = addr;
        a.size = size;
        a.off = off;
        a.cb = cb;
        a.map = map;
        a.dense = pack ? (uint8_t *)dense : nullptr;
        a.crc = crc;
        a.flags = flags;
        a.base_crc = base_crc;
        HIP_TRY(launch_chunks(s, pack ? kModePack : kModeHash, a, ctx->grid_chunks, cfg.block_threads));
    }
    if (n_chunks)
        *n_chunks = N;
    if (data_bytes)
        *data_bytes = D;
    return CKPT_OK;
}
