// ckpt_runtime.h -- host-side types of libckpt (not part of the public ABI).
#pragma once

#include <atomic>
#include <cstddef>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ckpt.h"
#include "internal.h"

namespace ckpt {

int set_error(int status, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what, int line);

#define HIP_TRY(expr)                                                   \
    do {                                                                \
        hipError_t e_ = (expr);                                         \
        if (e_ != hipSuccess)                                           \
            return ::ckpt::hip_fail(e_, #expr, __LINE__);               \
    } while (0)

#define CKPT_TRY(expr)                                                  \
    do {                                                                \
        int rc_ = (expr);                                               \
        if (rc_ != CKPT_OK)                                             \
            return rc_;                                                 \
    } while (0)

// Grow-only device buffer.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    int ensure(size_t bytes);
    void release();
};

// Pinned host buffer from the process-wide pool; returned to the pool when
// released or destroyed.
struct PinnedBuf {
    void *p = nullptr;
    size_t cap = 0;
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf &) = delete;
    PinnedBuf &operator=(const PinnedBuf &) = delete;
    PinnedBuf(PinnedBuf &&o) noexcept : p(o.p), cap(o.cap) { o.p = nullptr; o.cap = 0; }
    PinnedBuf &operator=(PinnedBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p;
            cap = o.cap;
            o.p = nullptr;
            o.cap = 0;
        }
        return *this;
    }
    ~PinnedBuf() { release(); }
    int ensure(size_t bytes);
    void release();
};

// Pinned host bytes handed out by the process-wide pool (images' sections,
// staging) and not yet returned; the buffers it keeps for reuse are not
// counted.
uint64_t pinned_live_bytes();

// Completion of an asynchronous copy into host memory, shared by the images
// it fills.
struct MetaEvent {
    hipEvent_t e = nullptr;
    std::atomic<bool> done{false};
    void wait()
    {
        if (e && !done.load()) {
            (void)hipEventSynchronize(e);
            done.store(true);
        }
    }
    ~MetaEvent()
    {
        wait();
        if (e)
            (void)hipEventDestroy(e);
    }
};

class DeviceGuard {
public:
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
    bool ok() const { return ok_; }

private:
    int prev_ = 0;
    bool ok_ = false;
};

// One row of a table to drain or refill.
struct Row {
    uint64_t id = 0;
    uint32_t kind = 0;
    uint64_t ptr = 0;    // source (checkpoint) or destination (restore) address
    uint64_t size = 0;
};
using Reg = Row;

struct RangeEnd {
    uint64_t end;
    uint64_t id;
};

// A virtual range the context reserved and backed with device memory
// (ckpt_vmm_alloc, ckpt_restore_at); released when its last registration goes.
struct VmmRange {
    uint64_t bytes = 0;                    // multiple of the allocation granularity
    hipMemGenericAllocationHandle_t h{};   // the physical memory mapped there
    uint32_t refs = 0;                     // live registrations inside the range
    bool in_window = false;                // its addresses belong to a VmmWindow
};

// A large region of virtual addresses the context picked once; address-stable
// allocations without a requested address are placed in it from the bottom
// up (each with its own reservation), far below the addresses the runtime
// hands out for its own use.
struct VmmWindow {
    uint64_t base = 0, usable = 0;        // [base, base + usable)
    std::map<uint64_t, uint64_t> free;    // spots not booked: start -> bytes
};

// Registration with a given id when it is still unissued in the context (at or
// above next_id), else with the next id; fails on overlap as ckpt_register does.
int add_registration(ckpt_ctx *ctx, uint64_t start, uint64_t bytes, uint32_t kind, uint64_t want_id,
                     uint64_t *id);
int drop_registration(ckpt_ctx *ctx, uint64_t start);
void vmm_release_all(ckpt_ctx *ctx);
// When delta's allocation table differs from img's, *merged = the two folded
// into one full image (ckpt_image_merge); else *merged stays empty.
int fold_delta(const ckpt_image *img, const ckpt_image *delta, std::unique_ptr<ckpt_image> *merged);
// A serialized image's header and tables, checked, without the CRC, flag,
// id and DATA sections (the first three start at `rest`; DATA follows them,
// head_bytes from the image's start).  Host memory only.
struct ImageHead {
    uint32_t version = 0, mode = 0, C = 0;
    uint64_t N = 0, data_bytes = 0, ser_bytes = 0, n_dirty = 0, serial = 0, base_serial = 0, digest = 0;
    uint64_t head_bytes = 0;
    std::vector<ckpt_alloc_rec> allocs;
    std::vector<uint64_t> addrs;
    const uint8_t *rest = nullptr;
};
// Checks the fixed header at hdr (hdr_bytes readable) of an image of `avail`
// bytes and gives the size of everything before DATA and of DATA.
int head_layout(const void *hdr, size_t hdr_bytes, uint64_t avail, uint64_t *head_bytes, uint64_t *ser_bytes);
// Parses buf[0, bytes).  data_apart = 0: buf is the whole image; else buf holds
// at least everything before DATA and the caller holds DATA (data_apart bytes,
// which must be ser_bytes) elsewhere.
int parse_head(const void *buf, size_t bytes, ImageHead *h, uint64_t data_apart = 0);
// A new drained image with h's tables and CRC/flag/id sections (the digest
// checked; h's tables are moved out) and room for DATA, not yet filled.
int image_from_head(ckpt_ctx *ctx, ImageHead *h, ckpt_image **out);
// An image file opened for reading: its head read and checked, DATA not yet.
struct ImageFile {
    int fd = -1;
    std::string path;
    std::vector<uint8_t> head;
    ImageHead h;
    // a compressed container (CKPT_FILE_DEFLATE): DATA in blocks of zblock
    // bytes, block b stored at zoff[b] as zlen[b] bytes, raw when zraw[b]
    bool deflated = false;
    uint32_t zblock = 0;
    std::vector<uint64_t> zoff, zlen;
    std::vector<uint8_t> zraw, zplanes;   // zplanes: element width of the byte planes (1: none)
    ImageFile() = default;
    ImageFile(const ImageFile &) = delete;
    ImageFile &operator=(const ImageFile &) = delete;
    ~ImageFile();
};
int open_image_file(const char *path, ImageFile *f);
// image_from_head, then DATA read from the file straight into the image's
// pinned memory by several threads.
int load_image_file(ckpt_ctx *ctx, ImageFile *f, ckpt_image **out);

// Digest of an image's CRC section (ckpt_image_meta.crc_digest).
uint64_t crc_digest(const void *p, size_t n);

// The serialized form up to (not including) DATA, which follows it.
size_t serialized_head_bytes(const ckpt_image *img);
void serialize_head(const ckpt_image *img, uint8_t *out);

// The allocation hook (ckpt_hook_*) and the calls on the context it logs into
// are serialized by one process-wide lock, held only for a hooked context.
std::recursive_mutex &hook_mutex();
void hook_forget(ckpt_ctx *ctx);
// Releases the hook's cached blocks when ctx is the installed context.
void hook_trim_for(ckpt_ctx *ctx);
// An address-stable block of `bytes` (a granularity multiple) placed by the
// context, mapped but not registered; unmapped again by vmm_block_unmap (or
// with the context's other ranges when it is destroyed).
int vmm_block_map(ckpt_ctx *ctx, uint64_t bytes, uint64_t *base);
void vmm_block_unmap(ckpt_ctx *ctx, uint64_t base);

}  // namespace ckpt

struct ckpt_ctx {
    ckpt_config cfg{};
    int cu_count = 0;
    int grid_chunks = 0;   // persistent workgroups of the chunk kernels
    int grid_small = 0;    // grid of the map / gather kernels
    bool managed_prefetch = false;
    bool ready = false;           // streams, events, tables made (ctx_ready)
    hipStream_t side = nullptr;   // drain stream
    hipStream_t cap = nullptr;    // graph capture stream
    hipStream_t gat = nullptr;    // gather stream of a segmented drain
    hipEvent_t ev[8] = {};
    std::vector<hipEvent_t> seg_ev;   // segment pipelines: slot ordering and timing
    hipEvent_t meta_ev = nullptr;   // last asynchronous CRC/flag copy to the host
    bool meta_pending = false;

    // captured prologue (graph_prologue) and what it was captured for
    hipGraphExec_t g_exec = nullptr;
    uint64_t g_n = 0, g_N = 0, g_D = 0;
    bool g_drain = false;        // the graph also holds the drain (select + gather into host memory)
    uint64_t g_outs = 0;         // outputs the drain tables hold
    bool g_nt = false;           // the captured pack's hint (non-temporal)
    std::vector<void *> g_ptrs;
    uint64_t graph_captures = 0;

    // the log: live registrations in id order, and their ranges by start
    std::vector<ckpt::Reg> live;
    std::map<uint64_t, ckpt::RangeEnd> ranges;
    uint64_t next_id = 1;

    // address-stable memory the context owns: ranges by base, and the range
    // base of each registration made inside one
    std::map<uint64_t, ckpt::VmmRange> vmm;
    std::map<uint64_t, uint64_t> vmm_of;
    std::vector<ckpt::VmmWindow> windows;
    std::atomic<bool> hooked{false};   // the allocation hook logs into this context

    // device buffers
    const uint32_t *tables = nullptr;   // shared CRC operator tables (shared_tables)
    ckpt::DevBuf d_plan, d_addr, d_size, d_off, d_cb, d_map;
    ckpt::DevBuf d_crc, d_flags, d_base_crc, d_prev_crc, d_soff, d_ids, d_tile_b, d_tile_c;
    ckpt::DevBuf d_dense, d_compact, d_bad, d_pick, d_crc2, d_flags2, d_soff2, d_base_cb, d_snap_flags;
    ckpt::DevBuf d_drain;   // the graph's drain tables: out_addr, out_chunk0, row_out
    ckpt::PinnedBuf h_up, h_plan, h_base_cb;
    bool reserved = false;      // CKPT_RESERVE_STAGING: d_dense is the reserved block
    bool hint_auto = false;     // load_hint was 0: the pack picks its hint (pack_hint)
    uint64_t prev_serial = 0;   // image whose CRC array is in d_prev_crc
    uint32_t zero_crc = 0;      // CRC-32C of chunk_bytes zero bytes (made at ckpt_init)

    ckpt_timing timing{};

    std::vector<ckpt::DevBuf *> all_dev()
    {
        return {&d_plan, &d_addr, &d_size, &d_off, &d_cb, &d_map, &d_crc, &d_flags, &d_base_crc,
                &d_prev_crc, &d_soff, &d_ids, &d_tile_b, &d_tile_c, &d_dense, &d_compact, &d_bad, &d_pick,
                &d_crc2, &d_flags2, &d_soff2, &d_base_cb, &d_snap_flags, &d_drain};
    }
};

struct ckpt_image {
    int device = 0;
    uint32_t mode = CKPT_FULL;
    uint32_t C = 0;
    uint64_t N = 0, data_bytes = 0, ser_bytes = 0, n_dirty = 0;
    uint64_t serial = 0, base_serial = 0;
    bool drained = false;
    std::vector<ckpt_alloc_rec> allocs;
    std::vector<uint64_t> addrs;   // device address of each allocation when taken
    // CRC and flag sections: slices of a pinned block that the images of one
    // batch share (one copy from the device for all of them)
    std::shared_ptr<ckpt::PinnedBuf> meta;
    uint32_t *crc = nullptr;
    uint8_t *flags = nullptr;
    ckpt::PinnedBuf ids_buf, data;
    void *dense = nullptr;
    bool dense_owned = false;
    std::shared_ptr<ckpt::MetaEvent> meta_ready;   // host CRC/flags valid once this completes
    ~ckpt_image();
};

namespace ckpt {

int ctx_setup(ckpt_ctx *ctx);
// Looks up, once per device, the device address of the allocation-free
// path's file-scope array (ckpt_checkpoint_noalloc); `device` must be current.
int noalloc_setup(int device);
// The device CRC operator tables for cfg (device, layout, pieces, rounds per
// wave), made on first use and shared; NULL and *rc set on failure.
const uint32_t *shared_tables(const ckpt_config &cfg, int *rc);
// A private pinned block for an image's CRC (4N bytes) and flags (N bytes).
int alloc_meta(ckpt_image *img, uint64_t N);
void image_wait(const ckpt_image *img);
int order_after_meta(ckpt_ctx *ctx, hipStream_t s);
int ctx_ready(ckpt_ctx *ctx);
// Device staging of `bytes` serialized bytes (a drain's gather output, a
// restore's copy from the host): with a reservation, the reserved block from
// `used` bytes on (rounded up to 256); else the context's compact buffer.
int serial_staging(ckpt_ctx *ctx, uint64_t used, uint64_t bytes, uint8_t **out);
// ckpt_restore; fresh_dst: the destinations were mapped by the caller just
// before (one pass instead of segments where the staging fits).
int restore_impl(ckpt_ctx *ctx, void *stream, const ckpt_image *img, const ckpt_image *delta, void *const *dst,
                 const size_t *dst_bytes, size_t n_dst, ckpt_verify_report *rep, bool fresh_dst);
// Segment size of drains and restores (0: one pass) and the device slots.
uint64_t segment_bytes(const ckpt_config &cfg);
constexpr int kSegSlots = 4;
// At least n events in ctx->seg_ev.
int seg_events(ckpt_ctx *ctx, size_t n);
// The drain a replayed graph may hold: the selected chunks of output i go
// straight into pinned host buffer (*data)[i], which holds at least output
// i's dense bytes.
struct GraphDrain {
    size_t nout;
    const uint64_t *part_row;     // nout + 1: each output's first row, then n
    const uint64_t *part_chunk;   // nout + 1: each output's first chunk, then N
    std::vector<PinnedBuf> *data;
};
int graph_prologue(ckpt_ctx *ctx, hipStream_t s, const std::vector<Row> &rows, uint64_t N, uint64_t data_bytes,
                   const GraphDrain *drain, bool nontemporal);
// The pack's load/store hint for these rows and their dense offsets (runtime.cpp).
bool pack_hint(const ckpt_ctx *ctx, const std::vector<Row> &rows, const std::vector<uint64_t> &off);
int upload_table(ckpt_ctx *ctx, hipStream_t s, const std::vector<Row> &rows, bool dst_side, uint64_t N_host,
                 uint64_t n_items);
int read_plan(ckpt_ctx *ctx, hipStream_t s, DevPlan *out);
int run_select(ckpt_ctx *ctx, hipStream_t s, int mode, const uint8_t *flags, const uint64_t *ids,
               uint64_t max_items, uint64_t *soff, uint64_t *ids_out, uint64_t ids_cap);
ChunkArgs chunk_args(ckpt_ctx *ctx);
int run_checkpoint(ckpt_ctx *ctx, hipStream_t s, int mode, const ckpt_image *base, const std::vector<Row> &rows,
                   const std::vector<size_t> &parts, std::vector<ckpt_image *> &outs, bool use_graph);

}  // namespace ckpt

namespace ckpt {
// Holds the hook lock while a call works on a hooked context.
class HookGuard {
public:
    explicit HookGuard(const ckpt_ctx *ctx)
    {
        if (ctx && ctx->hooked.load())
            lk_ = std::unique_lock<std::recursive_mutex>(hook_mutex());
    }

private:
    std::unique_lock<std::recursive_mutex> lk_;
};
}  // namespace ckpt
