// server.cpp -- the serving loop of libckpt: continuous batching of
// checkpoint and restore requests on one GPU.
//
// Requests are admitted in arrival order when a slot is free and their
// device staging fits the budget.  Admitted requests are prepared by an
// auxiliary worker (allocation table upload, size scan, chunk map; for a
// restore also the image upload, selection scan and consistency check), then
// join the step loop: each step is ONE launch of the row-mode chunk kernel
// that processes up to step_bytes of every stepping request, packing some and
// restoring others.  A request whose chunks are all processed is finished by
// an auxiliary worker (checkpoint: selection scan, gather, copy of the
// serialized image to pinned host memory; restore: the verification count)
// while later steps keep the GPU busy with the other requests.  Requests that
// arrive meanwhile join at the next step.  Admission (admission.h) counts the
// device staging of every request and, for a checkpoint, the pinned host
// memory of the image it will produce.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.h"
#include "ckpt.h"
#include "ckpt_runtime.h"

using namespace ckpt;
using Clock = std::chrono::steady_clock;

namespace {

uint64_t r256(uint64_t x) { return (x + 255) & ~uint64_t(255); }
uint64_t ru16(uint64_t x) { return (x + 15) & ~uint64_t(15); }
double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// The staging budget: one device block, carved by an ArenaMap.
class Arena {
public:
    int init(uint64_t bytes)
    {
        CKPT_TRY(mem_.ensure(bytes));
        map_.reset(bytes);
        return CKPT_OK;
    }
    void release() { mem_.release(); map_.reset(0); }
    uint64_t size() const { return map_.size(); }
    uint64_t alloc(uint64_t bytes) { return map_.alloc(bytes); }
    void free(uint64_t off, uint64_t bytes) { map_.free(off, bytes); }
    const ArenaMap &map() const { return map_; }
    uint8_t *base() const { return (uint8_t *)mem_.p; }

private:
    DevBuf mem_;
    ArenaMap map_;
};

enum State { kQueued, kPrep, kStepping, kFinish, kDone };

struct Req {
    uint64_t ticket = 0;
    uint32_t op = CKPT_REQ_CHECKPOINT;
    std::vector<Row> rows;          // ptr = source (checkpoint) or destination (restore)
    const ckpt_image *image = nullptr;
    std::vector<uint64_t> off, cb;  // host layout, n + 1 each
    uint64_t N = 0, data_bytes = 0, live = 0, ser_bytes = 0;
    uint64_t host_charge = 0;       // checkpoint: most pinned bytes its image can take
    bool waited_host = false;       // was held back for host memory
    bool mem_waited = false;        // a step of it waited for memory
    Clock::time_point t_mem_wait{};
    // device block and its parts
    uint64_t block_off = 0, block_bytes = 0;
    uint64_t *d_addr = nullptr, *d_size = nullptr, *d_off = nullptr, *d_cb = nullptr, *d_soff = nullptr;
    uint64_t *d_tile_b = nullptr, *d_tile_c = nullptr;
    uint32_t *d_map = nullptr, *d_crc = nullptr;
    uint8_t *d_flags = nullptr, *d_bad = nullptr, *d_dense = nullptr, *d_compact = nullptr, *d_staging = nullptr;
    DevPlan *d_plan = nullptr;
    uint64_t next_chunk = 0;
    State state = kQueued;
    Clock::time_point t_submit, t_admit, t_done;
    ckpt_result result{};
};

struct Task {
    Req *req;
    bool prep;                      // prep or finish
    Clock::time_point not_before{}; // a finish waiting for pinned host memory
};

// finish_request: the image's pinned host memory could not be allocated now
// (the request keeps its staging and is finished again later)
constexpr int kRetryHost = 1;
// how long a request (or a step) may wait for memory before it fails
constexpr double kHostWaitLimitMs = 30000.0;
constexpr int kHostRetryMs = 2;

}  // namespace

struct ckpt_server {
    ckpt_server_config cfg{};
    int cu_count = 0;
    bool managed_prefetch = false;
    Arena arena;
    DevBuf d_tables;
    hipStream_t step_stream = nullptr;

    std::mutex mu;
    std::condition_variable cv_step, cv_aux, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<Req *> queue;                      // submitted, not admitted
    std::vector<Req *> active;                    // admitted, not done
    std::unordered_map<uint64_t, Req *> by_ticket;
    std::deque<Task> aux_tasks;
    AdmitState adm;                               // slots and host reservations
    bool host_blocked = false;                    // a checkpoint waits for host memory
    const Req *held = nullptr;                    // that checkpoint, held back since t_held
    Clock::time_point t_held{};

    // step buffers (owned by the step thread)
    PinnedBuf h_step;
    DevBuf d_step, d_map;

    std::thread step_thread;
    std::vector<std::thread> aux_threads;

    // statistics
    uint64_t submitted = 0, completed = 0, failed = 0, bytes = 0, steps = 0;
    uint64_t host_waits = 0, host_peak = 0;
    char last_error[160] = {};                    // message of the latest failure
    Clock::time_point t_step_wait{};              // a step waits for memory since
    bool step_waiting = false;
    uint32_t max_concurrent = 0;
    std::vector<double> lat_ms;
    bool have_first = false;
    Clock::time_point t_first, t_last;
};

namespace {

int hip_err(Req *r, hipError_t e, const char *what)
{
    r->result.status = hip_fail(e, what, __LINE__);
    return r->result.status;
}

#define REQ_HIP(r, expr)                                 \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess)                            \
            return hip_err((r), e_, #expr);              \
    } while (0)

// Parts of a request's device block, 256-byte aligned.  Returns total bytes.
uint64_t plan_block(Req *r, uint8_t *base)
{
    const uint64_t n = r->rows.size(), N = r->N;
    const uint64_t tiles = std::max<uint64_t>((N + kSelTile - 1) / kSelTile, 1);
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint8_t *p = base ? base + o : nullptr;
        o += r256(std::max<uint64_t>(bytes, 16));
        return p;
    };
    r->d_plan = (DevPlan *)take(sizeof(DevPlan));
    r->d_addr = (uint64_t *)take(8 * n);
    r->d_size = (uint64_t *)take(8 * n);
    r->d_off = (uint64_t *)take(8 * (n + 1));
    r->d_cb = (uint64_t *)take(8 * (n + 1));
    r->d_map = (uint32_t *)take(4 * N);
    r->d_crc = (uint32_t *)take(4 * N);
    r->d_flags = (uint8_t *)take(N);
    r->d_soff = (uint64_t *)take(8 * N);
    r->d_tile_b = (uint64_t *)take(8 * tiles);
    r->d_tile_c = (uint64_t *)take(8 * tiles);
    if (r->op == CKPT_REQ_CHECKPOINT) {
        r->d_dense = take(r->data_bytes);
        r->d_compact = take(r->data_bytes);
    } else {
        r->d_bad = take(N);
        r->d_staging = take(r->ser_bytes);
    }
    return o;
}

SelArgs sel_args(Req *r, int mode, const uint8_t *flags)
{
    SelArgs a;
    memset(&a, 0, sizeof(a));
    a.plan = r->d_plan;
    a.mode = mode;
    a.size = r->d_size;
    a.cb = r->d_cb;
    a.map = r->d_map;
    a.flags = flags;
    a.tile_bytes = r->d_tile_b;
    a.tile_count = r->d_tile_c;
    a.soff = r->d_soff;
    return a;
}

// Upload the table, scan, map; restore: stage the image and check it.
int prep_request(ckpt_server *sv, Req *r, hipStream_t s, PinnedBuf &up)
{
    const uint64_t n = r->rows.size(), N = r->N;
    const size_t bytes = sizeof(DevPlan) + 16 * n;
    CKPT_TRY(up.ensure(bytes));
    auto *plan = (DevPlan *)up.p;
    memset(plan, 0, sizeof(DevPlan));
    plan->n_allocs = n;
    plan->n_items = N;
    auto *addr = (uint64_t *)((uint8_t *)up.p + sizeof(DevPlan));
    for (uint64_t k = 0; k < n; k++) {
        addr[k] = r->rows[k].ptr;
        addr[n + k] = r->rows[k].size;
    }
    REQ_HIP(r, hipMemcpyAsync(r->d_plan, plan, sizeof(DevPlan), hipMemcpyHostToDevice, s));
    if (n) {
        REQ_HIP(r, hipMemcpyAsync(r->d_addr, addr, 8 * n, hipMemcpyHostToDevice, s));
        REQ_HIP(r, hipMemcpyAsync(r->d_size, addr + n, 8 * n, hipMemcpyHostToDevice, s));
    }
    REQ_HIP(r, launch_layout_scan(s, r->d_plan, r->d_size, sv->cfg.chunk_bytes, r->d_off, r->d_cb));
    if (N)
        REQ_HIP(r, launch_chunk_map(s, r->d_plan, r->d_cb, r->d_map, sv->cu_count));
    if (r->op == CKPT_REQ_CHECKPOINT) {
        if (sv->managed_prefetch)
            for (const Row &row : r->rows)
                if (row.kind == CKPT_MANAGED && row.size)
                    REQ_HIP(r, hipMemPrefetchAsync((const void *)row.ptr, row.size, sv->cfg.device, s));
    } else {
        const ckpt_image *img = r->image;
        if (N) {
            REQ_HIP(r, hipMemcpyAsync(r->d_crc, img->crc, 4 * N, hipMemcpyHostToDevice, s));
            REQ_HIP(r, hipMemcpyAsync(r->d_flags, img->flags, N, hipMemcpyHostToDevice, s));
            REQ_HIP(r, hipMemsetAsync(r->d_bad, 0, N, s));
        }
        if (r->ser_bytes)
            REQ_HIP(r, hipMemcpyAsync(r->d_staging, img->data.p, r->ser_bytes, hipMemcpyHostToDevice, s));
        if (N) {
            SelArgs a = sel_args(r, kSelNonZero, r->d_flags);
            a.C = sv->cfg.chunk_bytes;
            REQ_HIP(r, launch_select(s, a, N));
        }
    }
    REQ_HIP(r, hipMemcpyAsync(up.p, r->d_plan, sizeof(DevPlan), hipMemcpyDeviceToHost, s));
    REQ_HIP(r, hipStreamSynchronize(s));
    if (r->op == CKPT_REQ_RESTORE && N && plan->sel_bytes != r->ser_bytes) {
        r->result.status = set_error(CKPT_E_INVAL, "image flags select %llu bytes, data holds %llu",
                                     (unsigned long long)plan->sel_bytes, (unsigned long long)r->ser_bytes);
        return r->result.status;
    }
    return CKPT_OK;
}

// Checkpoint: select, gather, copy to pinned memory, build the image.
// Restore: read the verification count.
int finish_request(ckpt_server *sv, Req *r, hipStream_t s, PinnedBuf &up)
{
    const uint64_t N = r->N;
    const uint32_t C = sv->cfg.chunk_bytes;
    CKPT_TRY(up.ensure(sizeof(DevPlan)));
    auto *plan = (DevPlan *)up.p;
    if (r->op == CKPT_REQ_RESTORE) {
        REQ_HIP(r, hipMemcpyAsync(plan, r->d_plan, sizeof(DevPlan), hipMemcpyDeviceToHost, s));
        REQ_HIP(r, hipStreamSynchronize(s));
        r->result.n_bad = plan->bad_count;
        r->result.status = plan->bad_count ? CKPT_E_CORRUPT : CKPT_OK;
        r->result.bytes = r->live + r->ser_bytes;
        return CKPT_OK;
    }
    std::unique_ptr<ckpt_image> img(new ckpt_image());
    // On an error return, wait for the copies already queued into the image's
    // pinned buffers before they go back to the pool (declared after img, so
    // it runs before img is destroyed).
    struct SyncOnError {
        hipStream_t s;
        bool ok = false;
        ~SyncOnError()
        {
            if (!ok)
                (void)hipStreamSynchronize(s);
        }
    } sync_on_error{s};
    img->device = sv->cfg.device;
    img->mode = CKPT_FULL;
    img->C = C;
    img->N = N;
    img->data_bytes = r->data_bytes;
    img->drained = true;
    img->allocs.resize(r->rows.size());
    img->addrs.resize(r->rows.size());
    for (size_t k = 0; k < r->rows.size(); k++) {
        img->addrs[k] = r->rows[k].ptr;
        ckpt_alloc_rec &a = img->allocs[k];
        a.id = k + 1;
        a.kind = r->rows[k].kind;
        a.pad = 0;
        a.size = r->rows[k].size;
        a.off = r->off[k];
        a.cb = r->cb[k];
    }
    uint64_t sel = 0;
    if (N) {
        SelArgs a = sel_args(r, kSelNonZero, r->d_flags);
        a.C = C;
        REQ_HIP(r, launch_select(s, a, N));
        REQ_HIP(r, hipMemcpyAsync(plan, r->d_plan, sizeof(DevPlan), hipMemcpyDeviceToHost, s));
        REQ_HIP(r, hipStreamSynchronize(s));
        sel = plan->sel_bytes;
    }
    img->ser_bytes = sel;
    if (alloc_meta(img.get(), N) || img->data.ensure(std::max<uint64_t>(sel, 1))) {
        // nothing is queued into the image's buffers yet: give them back and
        // let the caller try again once host memory may have been released
        sync_on_error.ok = true;
        return kRetryHost;
    }
    if (sel) {
        GatherArgs g;
        memset(&g, 0, sizeof(g));
        g.plan = r->d_plan;
        g.mode = kSelNonZero;
        g.from_dense = 1;
        g.C = C;
        g.src = r->d_addr;
        g.size = r->d_size;
        g.off = r->d_off;
        g.cb = r->d_cb;
        g.map = r->d_map;
        g.dense = r->d_dense;
        g.flags = r->d_flags;
        g.soff = r->d_soff;
        g.out = r->d_compact;
        REQ_HIP(r, launch_gather(s, g, sv->cu_count));
        REQ_HIP(r, hipMemcpyAsync(img->data.p, r->d_compact, sel, hipMemcpyDeviceToHost, s));
    }
    if (N) {
        REQ_HIP(r, hipMemcpyAsync(img->crc, r->d_crc, 4 * N, hipMemcpyDeviceToHost, s));
        REQ_HIP(r, hipMemcpyAsync(img->flags, r->d_flags, N, hipMemcpyDeviceToHost, s));
    }
    REQ_HIP(r, hipStreamSynchronize(s));
    sync_on_error.ok = true;
    static std::atomic<uint64_t> serial{0};
    img->serial = (0x5E5Full << 48) | (++serial);
    r->result.image = img.release();
    r->result.status = CKPT_OK;
    r->result.bytes = r->live + r->data_bytes;
    return CKPT_OK;
}

void complete(ckpt_server *sv, Req *r)
{
    // caller holds sv->mu; no device work of r is queued any more
    r->t_done = Clock::now();
    r->state = kDone;
    r->result.latency_ms = ms_between(r->t_submit, r->t_done);
    r->result.queue_ms = ms_between(r->t_submit, r->t_admit);
    sv->arena.free(r->block_off, r->block_bytes);
    if (r->op == CKPT_REQ_CHECKPOINT)
        sv->adm.host_reserved -= r->host_charge;
    sv->active.erase(std::remove(sv->active.begin(), sv->active.end(), r), sv->active.end());
    sv->adm.n_active--;
    sv->t_last = r->t_done;
    if (r->result.status == CKPT_OK || r->result.status == CKPT_E_CORRUPT) {
        sv->completed++;
        sv->bytes += r->live;
        sv->lat_ms.push_back(r->result.latency_ms);
    } else {
        sv->failed++;
    }
    sv->cv_done.notify_all();
    sv->cv_step.notify_all();
}

// Keeps the failing thread's message (caller holds sv->mu).
void note_failure(ckpt_server *sv)
{
    snprintf(sv->last_error, sizeof(sv->last_error), "%s", ckpt_last_error());
}

AdmitInfo admit_info(const Req *r)
{
    AdmitInfo a;
    a.checkpoint = r->op == CKPT_REQ_CHECKPOINT;
    a.dev_bytes = r->block_bytes;
    a.host_bytes = r->host_charge;
    return a;
}

// A queued request that was never admitted ends with `status` (caller holds
// sv->mu): it has no staging block and no device work.
void fail_queued(ckpt_server *sv, Req *r, int status)
{
    sv->queue.erase(std::remove(sv->queue.begin(), sv->queue.end(), r), sv->queue.end());
    r->t_done = Clock::now();
    r->t_admit = r->t_done;
    r->state = kDone;
    r->result.status = status;
    r->result.latency_ms = ms_between(r->t_submit, r->t_done);
    r->result.queue_ms = r->result.latency_ms;
    sv->failed++;
    sv->t_last = r->t_done;
    sv->cv_done.notify_all();
}

// Admit queued requests (admission.h): in arrival order while a slot and
// staging are free; restores may pass a checkpoint that waits for host memory.
// A checkpoint held back for host memory longer than kHostWaitLimitMs fails
// with CKPT_E_NOMEM: the memory it waits for may be held by finished
// checkpoints' images that the caller has not claimed while it waits for this
// one.
void admit_locked(ckpt_server *sv)
{
    for (;;) {
        const uint64_t host_live = pinned_live_bytes();
        bool blocked = false;
        const long i = next_admissible(sv->queue, sv->adm, sv->arena.map(), host_live, admit_info, &blocked);
        sv->host_blocked = blocked;
        Req *held = nullptr;   // when blocked, the first queued checkpoint is the one held back
        if (blocked)
            for (Req *q : sv->queue)
                if (q->op == CKPT_REQ_CHECKPOINT) {
                    held = q;
                    break;
                }
        const auto now = Clock::now();
        if (held != sv->held) {   // a new hold (or none): its clock starts now
            sv->held = held;
            sv->t_held = now;
            if (held && !held->waited_host) {
                held->waited_host = true;
                sv->host_waits++;
            }
        } else if (held && ms_between(sv->t_held, now) >= kHostWaitLimitMs) {
            set_error(CKPT_E_NOMEM, "checkpoint held back %.0f s for host memory: %llu pinned bytes held, budget %llu",
                      kHostWaitLimitMs / 1000, (unsigned long long)host_live, (unsigned long long)sv->adm.host_budget);
            note_failure(sv);
            fail_queued(sv, held, CKPT_E_NOMEM);
            sv->held = nullptr;
            continue;   // the queue changed: look again
        }
        if (i < 0)
            return;
        Req *r = sv->queue[(size_t)i];
        const uint64_t off = sv->arena.alloc(r->block_bytes);
        if (off == UINT64_MAX)
            return;   // cannot happen: next_admissible checked that it fits
        sv->queue.erase(sv->queue.begin() + i);
        if (r == sv->held)
            sv->held = nullptr;
        r->block_off = off;
        plan_block(r, sv->arena.base() + off);
        r->state = kPrep;
        r->t_admit = Clock::now();
        if (r->op == CKPT_REQ_CHECKPOINT) {
            sv->adm.host_reserved += r->host_charge;
            sv->host_peak = std::max(sv->host_peak, host_live + sv->adm.host_reserved);
        }
        sv->active.push_back(r);
        sv->adm.n_active++;
        sv->max_concurrent = std::max(sv->max_concurrent, sv->adm.n_active);
        sv->aux_tasks.push_back({r, true});
        sv->cv_aux.notify_one();
    }
}

void aux_loop(ckpt_server *sv)
{
    DeviceGuard g(sv->cfg.device);
    hipStream_t s = nullptr;
    (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    PinnedBuf up;
    for (;;) {
        Task t{nullptr, false, {}};
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            for (;;) {
                if (sv->aux_tasks.empty() && sv->stop)
                    break;
                // the first task that may run now; else wait for the earliest
                const auto now = Clock::now();
                auto it = std::find_if(sv->aux_tasks.begin(), sv->aux_tasks.end(),
                                       [&](const Task &x) { return x.not_before <= now; });
                if (it != sv->aux_tasks.end()) {
                    t = *it;
                    sv->aux_tasks.erase(it);
                    break;
                }
                if (sv->aux_tasks.empty()) {
                    sv->cv_aux.wait(lk);
                } else {
                    auto first = sv->aux_tasks.front().not_before;
                    for (const Task &x : sv->aux_tasks)
                        first = std::min(first, x.not_before);
                    sv->cv_aux.wait_until(lk, first);
                }
            }
            if (!t.req)
                break;   // stopping
        }
        Req *r = t.req;
        int rc = t.prep ? prep_request(sv, r, s, up) : finish_request(sv, r, s, up);
        if (rc != CKPT_OK)
            (void)hipStreamSynchronize(s);   // nothing of r may still be queued when its block is freed
        if (rc == kRetryHost || rc == CKPT_E_NOMEM) {
            // Memory is short right now: pinned host memory for the image
            // (kRetryHost) or for a staging buffer, or device memory.  The
            // request keeps its staging block (a checkpoint: its packed image)
            // and the same step is run again shortly.  A short image buffer
            // also makes admission take the pinned bytes held now as the
            // host's capacity, so later checkpoints queue.
            const auto now = Clock::now();
            std::lock_guard<std::mutex> lk(sv->mu);
            if (!r->mem_waited) {
                r->mem_waited = true;
                r->t_mem_wait = now;
                sv->host_waits++;
            }
            if (rc == kRetryHost)
                sv->adm.host_budget = std::min<uint64_t>(sv->adm.host_budget ? sv->adm.host_budget : UINT64_MAX,
                                                         std::max<uint64_t>(pinned_live_bytes(), uint64_t(1) << 30));
            if (ms_between(r->t_mem_wait, now) < kHostWaitLimitMs) {
                r->result.status = CKPT_OK;
                sv->aux_tasks.push_back({r, t.prep, now + std::chrono::milliseconds(kHostRetryMs)});
                sv->cv_aux.notify_one();
                continue;
            }
            rc = set_error(CKPT_E_NOMEM, "memory for the request was not available for %.0f s",
                           kHostWaitLimitMs / 1000);
            r->result.status = rc;
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        if (rc != CKPT_OK || !t.prep) {
            if (rc != CKPT_OK && r->result.status == CKPT_OK)
                r->result.status = rc;
            if (rc != CKPT_OK)
                note_failure(sv);
            complete(sv, r);
        } else {
            r->state = r->N ? kStepping : kFinish;
            if (r->state == kFinish)
                sv->aux_tasks.push_back({r, false});
            sv->cv_step.notify_all();
            sv->cv_aux.notify_one();
        }
    }
    if (s)
        (void)hipStreamDestroy(s);
}

// Build and run one step over every stepping request.
// Where a step row came from: request, allocation, first chunk, chunk count.
struct RowSrc {
    size_t req;
    size_t k;
    uint64_t c, nc;
};

bool inside(uint64_t p, uint64_t bytes, uint64_t lo, uint64_t lo_bytes)
{
    return p >= lo && bytes <= lo_bytes && p - lo <= lo_bytes - bytes;
}

// Checks every address a step will hand the row kernel against the request
// it belongs to: each stepping request's block lies in the arena, is not part
// of a free hole and overlaps no other stepping request's block; every row's
// per-chunk arrays, dense image, staging and source or destination ranges lie
// inside that request's block or its allocations.  A violation is reported as
// an error instead of being launched.
int audit_step(const ckpt_server *sv, const std::vector<Req *> &reqs, const std::vector<StepRow> &rows,
               const std::vector<RowSrc> &src)
{
    const uint32_t C = sv->cfg.chunk_bytes;
    const uint64_t base = (uint64_t)sv->arena.base(), asz = sv->arena.size();
    std::vector<std::pair<uint64_t, uint64_t>> blocks;
    for (const Req *r : reqs) {
        if (r->state != kStepping || !inside(r->block_off, r->block_bytes, 0, asz))
            return set_error(CKPT_E_INVAL, "step audit: request %llu is not stepping in the arena",
                             (unsigned long long)r->ticket);
        for (const auto &h : sv->arena.map().holes())
            if (h.first < r->block_off + r->block_bytes && r->block_off < h.first + h.second)
                return set_error(CKPT_E_INVAL, "step audit: request %llu's block is free in the arena",
                                 (unsigned long long)r->ticket);
        blocks.emplace_back(r->block_off, r->block_bytes);
    }
    std::sort(blocks.begin(), blocks.end());
    for (size_t i = 1; i < blocks.size(); i++)
        if (blocks[i - 1].first + blocks[i - 1].second > blocks[i].first)
            return set_error(CKPT_E_INVAL, "step audit: two stepping requests share arena bytes");
    for (size_t j = 0; j < rows.size(); j++) {
        const StepRow &row = rows[j];
        const RowSrc &rs = src[j];
        const Req *r = reqs[rs.req];
        const uint64_t blk = base + r->block_off, N = r->N;
        const Row &al = r->rows[rs.k];
        const uint64_t start = (rs.c - r->cb[rs.k]) * C;
        const uint64_t span = std::min<uint64_t>(row.rem, rs.nc * C);   // data bytes of the row's chunks
        bool ok = inside((uint64_t)r->d_crc, 4 * N, blk, r->block_bytes) &&
                  inside((uint64_t)r->d_flags, N, blk, r->block_bytes) && rs.c + rs.nc <= N &&
                  rs.c >= r->cb[rs.k] && rs.c + rs.nc <= r->cb[rs.k + 1] && row.rem == al.size - start &&
                  row.crc == (uint64_t)(r->d_crc + rs.c) && row.flags == (uint64_t)(r->d_flags + rs.c);
        if (ok && row.mode == kModePack) {
            ok = r->op == CKPT_REQ_CHECKPOINT && inside(row.src, span, al.ptr, al.size) &&
                 inside((uint64_t)r->d_dense, r->data_bytes, blk, r->block_bytes) &&
                 inside(row.dst, ru16(span), (uint64_t)r->d_dense, r->data_bytes);
        } else if (ok) {
            ok = row.mode == kModeRestore && r->op == CKPT_REQ_RESTORE && inside(row.dst, span, al.ptr, al.size) &&
                 row.src == (uint64_t)r->d_staging &&
                 inside((uint64_t)r->d_staging, std::max<uint64_t>(r->ser_bytes, 1), blk, r->block_bytes) &&
                 inside((uint64_t)r->d_soff, 8 * N, blk, r->block_bytes) &&
                 inside((uint64_t)r->d_bad, N, blk, r->block_bytes) && row.soff == (uint64_t)(r->d_soff + rs.c) &&
                 row.bad == (uint64_t)(r->d_bad + rs.c) && row.bad_count == (uint64_t)&r->d_plan->bad_count &&
                 inside((uint64_t)r->d_plan, sizeof(DevPlan), blk, r->block_bytes);
        }
        if (!ok)
            return set_error(CKPT_E_INVAL, "step audit: row %zu of request %llu (allocation %zu, chunks %llu+%llu) "
                             "points outside its request", j, (unsigned long long)r->ticket, rs.k,
                             (unsigned long long)rs.c, (unsigned long long)rs.nc);
    }
    return CKPT_OK;
}

int run_step(ckpt_server *sv, const std::vector<Req *> &reqs, std::vector<uint64_t> &ends)
{
    const uint32_t C = sv->cfg.chunk_bytes;
    const uint64_t q = std::max<uint64_t>(1, sv->cfg.step_bytes / C);
    std::vector<StepRow> rows;
    std::vector<RowSrc> row_src;
    std::vector<uint64_t> row_cb;
    uint64_t items = 0;
    ends.resize(reqs.size());
    for (size_t i = 0; i < reqs.size(); i++) {
        Req *r = reqs[i];
        const uint64_t lo = r->next_chunk, hi = std::min(r->N, lo + q);
        ends[i] = hi;
        // allocation containing chunk lo: the last k with cb[k] <= lo
        size_t k = std::upper_bound(r->cb.begin(), r->cb.end() - 1, lo) - r->cb.begin() - 1;
        for (uint64_t c = lo; c < hi; k++) {
            const uint64_t c1 = std::min(hi, r->cb[k + 1]);
            if (c1 <= c)
                continue;
            const uint64_t first = c - r->cb[k], start = first * C;
            StepRow row;
            memset(&row, 0, sizeof(row));
            row.rem = r->rows[k].size - start;
            row.item0 = items;
            row.crc = (uint64_t)(r->d_crc + c);
            row.flags = (uint64_t)(r->d_flags + c);
            if (r->op == CKPT_REQ_CHECKPOINT) {
                row.mode = kModePack;
                row.src = r->rows[k].ptr + start;
                row.dst = (uint64_t)(r->d_dense + r->off[k] + start);
            } else {
                row.mode = kModeRestore;
                row.src = (uint64_t)r->d_staging;
                row.dst = r->rows[k].ptr + start;
                row.soff = (uint64_t)(r->d_soff + c);
                row.bad = (uint64_t)(r->d_bad + c);
                row.bad_count = (uint64_t)&r->d_plan->bad_count;
            }
            rows.push_back(row);
            row_src.push_back({i, k, c, c1 - c});
            row_cb.push_back(items);
            items += c1 - c;
            c = c1;
        }
    }
    if (!items)
        return CKPT_OK;
    {
        // the step thread reads the arena's holes while aux threads may
        // free other requests' blocks
        std::lock_guard<std::mutex> lk(sv->mu);
        CKPT_TRY(audit_step(sv, reqs, rows, row_src));
    }
    const uint64_t nr = rows.size();
    row_cb.push_back(items);
    const size_t bytes = sizeof(DevPlan) + nr * sizeof(StepRow) + (nr + 1) * 8;
    CKPT_TRY(sv->h_step.ensure(bytes));
    CKPT_TRY(sv->d_step.ensure(bytes));
    CKPT_TRY(sv->d_map.ensure(items * 4));
    uint8_t *h = (uint8_t *)sv->h_step.p;
    DevPlan plan;
    memset(&plan, 0, sizeof(plan));
    plan.n_allocs = nr;
    memcpy(h, &plan, sizeof(plan));
    memcpy(h + sizeof(DevPlan), rows.data(), nr * sizeof(StepRow));
    memcpy(h + sizeof(DevPlan) + nr * sizeof(StepRow), row_cb.data(), (nr + 1) * 8);
    uint8_t *d = (uint8_t *)sv->d_step.p;
    hipStream_t s = sv->step_stream;
    HIP_TRY(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_chunk_map(s, (const DevPlan *)d, (const uint64_t *)(d + sizeof(DevPlan) + nr * sizeof(StepRow)),
                             (uint32_t *)sv->d_map.p, sv->cu_count));
    RowArgs a;
    memset(&a, 0, sizeof(a));
    a.tables = (const uint32_t *)sv->d_tables.p;
    a.C = C;
    a.nontemporal = 1;
    a.n_items = items;
    a.rows = (const StepRow *)(d + sizeof(DevPlan));
    a.map = (const uint32_t *)sv->d_map.p;
    a.tile_ctr = &((DevPlan *)d)->tile_next;
    HIP_TRY(launch_rows(s, a, sv->cu_count, sv->cfg.block_threads));
    HIP_TRY(hipStreamSynchronize(s));
    return CKPT_OK;
}

void step_loop(ckpt_server *sv)
{
    DeviceGuard g(sv->cfg.device);
    std::vector<Req *> reqs;
    std::vector<uint64_t> ends;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            for (;;) {
                admit_locked(sv);
                reqs.clear();
                for (Req *r : sv->active)
                    if (r->state == kStepping)
                        reqs.push_back(r);
                if (sv->stop || !reqs.empty())
                    break;
                // host memory is released by whoever frees an image: poll
                // while a checkpoint waits for it
                if (sv->host_blocked)
                    sv->cv_step.wait_for(lk, std::chrono::milliseconds(1));
                else
                    sv->cv_step.wait(lk);
            }
            if (sv->stop)
                break;
        }
        int rc = run_step(sv, reqs, ends);
        if (rc != CKPT_OK)
            (void)hipStreamSynchronize(sv->step_stream);
        if (rc == CKPT_E_NOMEM) {
            // a step buffer could not grow: the requests keep their place and
            // the step runs again shortly, for as long as a request may wait
            const auto now = Clock::now();
            std::unique_lock<std::mutex> lk(sv->mu);
            if (!sv->step_waiting) {
                sv->step_waiting = true;
                sv->t_step_wait = now;
            }
            if (ms_between(sv->t_step_wait, now) < kHostWaitLimitMs) {
                sv->cv_step.wait_for(lk, std::chrono::milliseconds(kHostRetryMs));
                continue;
            }
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->step_waiting = false;
        if (rc != CKPT_OK)
            note_failure(sv);
        sv->steps++;
        for (size_t i = 0; i < reqs.size(); i++) {
            Req *r = reqs[i];
            if (rc != CKPT_OK) {
                r->result.status = rc;
                complete(sv, r);
                continue;
            }
            r->next_chunk = ends[i];
            if (r->next_chunk >= r->N) {
                r->state = kFinish;
                sv->aux_tasks.push_back({r, false});
                sv->cv_aux.notify_one();
            }
        }
    }
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" int ckpt_server_create(const ckpt_server_config *cfg_in, ckpt_server **out)
{
    if (!out)
        return set_error(CKPT_E_INVAL, "out is NULL");
    ckpt_server_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    if (cfg_in)
        cfg = *cfg_in;
    if (cfg.chunk_bytes == 0)
        cfg.chunk_bytes = 4096;
    if (cfg.chunk_bytes % 16 != 0 || cfg.chunk_bytes > (1u << 30))
        return set_error(CKPT_E_INVAL, "chunk_bytes %u", cfg.chunk_bytes);
    if (cfg.staging_budget == 0)
        cfg.staging_budget = uint64_t(64) << 30;
    if (cfg.step_bytes == 0)
        cfg.step_bytes = uint64_t(256) << 20;
    if (cfg.max_active == 0)
        cfg.max_active = 16;
    if (cfg.host_budget == 0)
        cfg.host_budget = uint64_t(64) << 30;
    if (cfg.lane_pieces == 0)
        cfg.lane_pieces = 1;
    if (cfg.lane_pieces != 1)
        return set_error(CKPT_E_INVAL, "lane_pieces %u: only 1", cfg.lane_pieces);
    if (cfg.block_threads == 0)
        cfg.block_threads = 1024;
    if (cfg.block_threads != 64 && cfg.block_threads != 128 && cfg.block_threads != 256 &&
        cfg.block_threads != 512 && cfg.block_threads != 1024)
        return set_error(CKPT_E_INVAL, "block_threads %u", cfg.block_threads);
    if (cfg.aux_threads == 0)
        cfg.aux_threads = 2;
    if (cfg.aux_threads > 16)
        return set_error(CKPT_E_INVAL, "aux_threads %u", cfg.aux_threads);
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDeviceCount", __LINE__);
    if (cfg.device < 0 || cfg.device >= ndev)
        return set_error(CKPT_E_INVAL, "device %d of %d", cfg.device, ndev);

    DeviceGuard g(cfg.device);
    auto *sv = new ckpt_server();
    sv->cfg = cfg;
    sv->adm.max_active = cfg.max_active;
    sv->adm.host_budget = cfg.host_budget;
    auto fail = [&](int rc) {
        ckpt_server_destroy(sv);
        return rc;
    };
    if ((e = hipDeviceGetAttribute(&sv->cu_count, hipDeviceAttributeMultiprocessorCount, cfg.device)) != hipSuccess)
        return fail(hip_fail(e, "hipDeviceGetAttribute", __LINE__));
    int managed = 0;
    if (hipDeviceGetAttribute(&managed, hipDeviceAttributeConcurrentManagedAccess, cfg.device) == hipSuccess)
        sv->managed_prefetch = managed != 0;
    if ((e = hipStreamCreateWithFlags(&sv->step_stream, hipStreamNonBlocking)) != hipSuccess)
        return fail(hip_fail(e, "hipStreamCreateWithFlags", __LINE__));
    int rc = sv->arena.init(cfg.staging_budget);
    if (rc != CKPT_OK)
        return fail(rc);
    // the replicated tables (one 1024-thread workgroup per CU)
    std::vector<uint32_t> tabs(kRepWords);
    const uint32_t rounds = (cfg.chunk_bytes + kRoundBytes - 1) / kRoundBytes;
    build_tables_replicated(tabs.data(), rounds);
    if ((rc = sv->d_tables.ensure(tabs.size() * 4)) != CKPT_OK)
        return fail(rc);
    if ((e = hipMemcpy(sv->d_tables.p, tabs.data(), tabs.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(hip_fail(e, "hipMemcpy(tables)", __LINE__));
    sv->step_thread = std::thread(step_loop, sv);
    for (uint32_t i = 0; i < cfg.aux_threads; i++)
        sv->aux_threads.emplace_back(aux_loop, sv);
    *out = sv;
    return CKPT_OK;
}

extern "C" int ckpt_server_submit(ckpt_server *sv, const ckpt_request *req, uint64_t *ticket)
{
    if (!sv || !req || !ticket)
        return set_error(CKPT_E_INVAL, "NULL argument");
    if (req->op != CKPT_REQ_CHECKPOINT && req->op != CKPT_REQ_RESTORE)
        return set_error(CKPT_E_INVAL, "unknown op %u", req->op);
    if (req->n && (!req->ptrs || !req->sizes))
        return set_error(CKPT_E_INVAL, "ptrs or sizes is NULL");
    const uint32_t C = sv->cfg.chunk_bytes;
    std::unique_ptr<Req> r(new Req());
    r->op = req->op;
    r->rows.resize(req->n);
    for (uint32_t k = 0; k < req->n; k++) {
        Row &row = r->rows[k];
        row.id = k + 1;
        row.kind = req->kinds ? req->kinds[k] : CKPT_DEVICE;
        row.ptr = (uint64_t)(uintptr_t)req->ptrs[k];
        row.size = req->sizes[k];
        if (row.kind != CKPT_DEVICE && row.kind != CKPT_MANAGED)
            return set_error(CKPT_E_INVAL, "allocation %u: unknown kind %u", k, row.kind);
        if (row.ptr % 16 != 0 || (row.size && row.ptr == 0))
            return set_error(CKPT_E_INVAL, "allocation %u: NULL or not 16-byte aligned", k);
    }
    r->off.resize(req->n + 1);
    r->cb.resize(req->n + 1);
    for (uint32_t k = 0; k < req->n; k++) {
        r->off[k + 1] = r->off[k] + ru16(r->rows[k].size);
        r->cb[k + 1] = r->cb[k] + (r->rows[k].size + C - 1) / C;
        r->live += r->rows[k].size;
    }
    r->N = r->cb[req->n];
    r->data_bytes = r->off[req->n];
    if (req->op == CKPT_REQ_RESTORE) {
        const ckpt_image *img = req->image;
        if (!img || !img->drained || img->mode != CKPT_FULL)
            return set_error(CKPT_E_INVAL, "restore needs a drained full image");
        if (img->C != C || img->allocs.size() != req->n)
            return set_error(CKPT_E_MISMATCH, "image chunk size or allocation count differs");
        for (uint32_t k = 0; k < req->n; k++)
            if (img->allocs[k].size != r->rows[k].size)
                return set_error(CKPT_E_MISMATCH, "allocation %u: %llu bytes, image has %llu", k,
                                 (unsigned long long)r->rows[k].size, (unsigned long long)img->allocs[k].size);
        r->image = img;
        r->ser_bytes = img->ser_bytes;
    }
    r->block_bytes = plan_block(r.get(), nullptr);
    if (r->block_bytes > sv->arena.size())
        return set_error(CKPT_E_BUDGET, "request needs %llu B of staging, the budget is %llu B",
                         (unsigned long long)r->block_bytes, (unsigned long long)sv->arena.size());
    if (r->op == CKPT_REQ_CHECKPOINT) {
        // the image's DATA (at most the dense bytes) and CRC/flag block, as
        // the pinned pool may hand them out: rounded up to 2 MiB, or a reused
        // buffer up to a quarter and 4 MiB larger
        const uint64_t meta = 5 * r->N;
        r->host_charge = r->data_bytes + r->data_bytes / 4 + meta + meta / 4 + (uint64_t(8) << 20) + 64;
        if (r->host_charge > sv->cfg.host_budget)
            return set_error(CKPT_E_BUDGET, "the image may need %llu B of pinned memory, the host budget is %llu B",
                             (unsigned long long)r->host_charge, (unsigned long long)sv->cfg.host_budget);
    }
    r->result.op = r->op;
    std::lock_guard<std::mutex> lk(sv->mu);
    r->ticket = sv->next_ticket++;
    r->t_submit = Clock::now();
    if (!sv->have_first) {
        sv->t_first = r->t_submit;
        sv->have_first = true;
    }
    sv->submitted++;
    *ticket = r->ticket;
    sv->by_ticket[r->ticket] = r.get();
    sv->queue.push_back(r.release());
    sv->cv_step.notify_all();
    return CKPT_OK;
}

static int take_result(ckpt_server *sv, uint64_t ticket, ckpt_result *out, bool wait)
{
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->by_ticket.find(ticket);
    if (it == sv->by_ticket.end())
        return set_error(CKPT_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Req *r = it->second;
    if (wait)
        sv->cv_done.wait(lk, [&] { return r->state == kDone; });
    if (r->state != kDone)
        return CKPT_E_AGAIN;
    if (out)
        *out = r->result;
    else if (r->result.image)
        ckpt_image_free(r->result.image);
    sv->by_ticket.erase(it);
    delete r;
    return CKPT_OK;
}

extern "C" int ckpt_server_poll(ckpt_server *sv, uint64_t ticket, ckpt_result *out)
{
    if (!sv)
        return set_error(CKPT_E_INVAL, "server is NULL");
    return take_result(sv, ticket, out, false);
}

extern "C" int ckpt_server_wait(ckpt_server *sv, uint64_t ticket, ckpt_result *out)
{
    if (!sv)
        return set_error(CKPT_E_INVAL, "server is NULL");
    return take_result(sv, ticket, out, true);
}

extern "C" int ckpt_server_stats(const ckpt_server *csv, ckpt_stats *out)
{
    if (!csv || !out)
        return set_error(CKPT_E_INVAL, "NULL argument");
    auto *sv = const_cast<ckpt_server *>(csv);
    std::lock_guard<std::mutex> lk(sv->mu);
    memset(out, 0, sizeof(*out));
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->failed = sv->failed;
    out->bytes = sv->bytes;
    out->steps = sv->steps;
    out->max_concurrent = sv->max_concurrent;
    out->host_waits = sv->host_waits;
    out->host_peak = sv->host_peak;
    memcpy(out->last_error, sv->last_error, sizeof(out->last_error));
    std::vector<double> v = sv->lat_ms;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        // nearest-rank percentiles
        auto pct = [&](double p) {
            size_t i = (size_t)std::ceil(p / 100.0 * v.size());
            return v[std::min(v.size() - 1, i ? i - 1 : 0)];
        };
        out->p50_ms = pct(50);
        out->p99_ms = pct(99);
        double s = 0;
        for (double x : v)
            s += x;
        out->mean_ms = s / v.size();
        out->max_ms = v.back();
    }
    if (sv->have_first && sv->completed) {
        out->makespan_s = std::chrono::duration<double>(sv->t_last - sv->t_first).count();
        if (out->makespan_s > 0)
            out->gbps = sv->bytes / out->makespan_s / 1e9;
    }
    return CKPT_OK;
}

extern "C" int ckpt_server_reset_stats(ckpt_server *sv)
{
    if (!sv)
        return set_error(CKPT_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->submitted = sv->completed = sv->failed = sv->bytes = sv->steps = 0;
    sv->max_concurrent = sv->adm.n_active;
    sv->host_waits = 0;
    sv->host_peak = 0;
    sv->last_error[0] = 0;
    sv->lat_ms.clear();
    sv->have_first = false;
    return CKPT_OK;
}

extern "C" void ckpt_server_destroy(ckpt_server *sv)
{
    if (!sv)
        return;
    {
        // let admitted work finish: wait until nothing is active, then stop
        std::unique_lock<std::mutex> lk(sv->mu);
        for (Req *r : sv->queue) {
            r->result.status = CKPT_E_AGAIN;
            r->state = kDone;
        }
        sv->queue.clear();
        if (sv->step_thread.joinable())
            sv->cv_done.wait(lk, [&] { return sv->adm.n_active == 0; });
        sv->stop = true;
        sv->cv_step.notify_all();
        sv->cv_aux.notify_all();
    }
    if (sv->step_thread.joinable())
        sv->step_thread.join();
    for (auto &t : sv->aux_threads)
        if (t.joinable())
            t.join();
    {
        DeviceGuard g(sv->cfg.device);
        if (sv->step_stream)
            (void)hipStreamDestroy(sv->step_stream);
        sv->arena.release();
        sv->d_tables.release();
        sv->d_step.release();
        sv->d_map.release();
        sv->h_step.release();
    }
    for (auto &kv : sv->by_ticket) {
        if (kv.second->result.image)
            ckpt_image_free(kv.second->result.image);
        delete kv.second;
    }
    delete sv;
}
