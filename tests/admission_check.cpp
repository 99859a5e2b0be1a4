// admission_check.cpp -- drives the serving loop's admission policy
// (paper_2008_10596_amd/csrc/admission.h) on the CPU, the way the server's
// step thread and workers do, with the device calls left out: requests are
// submitted, admitted, finished, and their images released by a simulated
// caller.  Built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_server_admission.py.  After every event it checks:
//   - admitted requests' staging blocks lie in the arena, are not free there,
//     and do not overlap; the arena's used bytes are their sum;
//   - at most max_active requests are admitted;
//   - the host reservation is the sum of the admitted checkpoints' charges,
//     and no checkpoint was admitted past the host budget;
//   - checkpoints are admitted in arrival order, and a request passes an
//     earlier one only when it is a restore passing a checkpoint that waits
//     for host memory;
// and at the end that every request was admitted and finished.
// Exit status 0 when every check holds; the first failing check is printed.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "admission.h"

using namespace ckpt;

namespace {

struct SimReq {
    uint64_t seq = 0;
    bool checkpoint = false;
    uint64_t dev = 0, host = 0;
    uint64_t off = 0;
    uint64_t image = 0;   // bytes of the image it produced (checkpoint)
};

int g_fail = 0;

#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            std::fprintf(stderr, "check failed: %s: ", #cond); \
            std::fprintf(stderr, __VA_ARGS__);             \
            std::fprintf(stderr, "\n");                    \
            g_fail = 1;                                    \
            return false;                                  \
        }                                                  \
    } while (0)

struct Sim {
    AdmitState st;
    ArenaMap arena;
    std::deque<SimReq *> queue;
    std::vector<SimReq *> active;
    std::vector<uint64_t> held;     // images the caller keeps (pinned bytes)
    uint64_t host_live = 0;
    uint64_t last_ckpt_seq = 0;     // arrival order of admitted checkpoints
    uint64_t submitted = 0, admitted = 0, finished = 0;
    bool blocked = false;

    bool invariants()
    {
        CHECK(st.n_active == active.size() && st.n_active <= st.max_active, "%u active", st.n_active);
        uint64_t used = 0, reserved = 0;
        std::vector<std::pair<uint64_t, uint64_t>> blocks;
        for (const SimReq *r : active) {
            used += r->dev;
            if (r->checkpoint)
                reserved += r->host;
            CHECK(r->off <= arena.size() && r->dev <= arena.size() - r->off, "block out of the arena");
            for (const auto &h : arena.holes())
                CHECK(!(h.first < r->off + r->dev && r->off < h.first + h.second), "admitted block is free");
            blocks.emplace_back(r->off, r->dev);
        }
        std::sort(blocks.begin(), blocks.end());
        for (size_t i = 1; i < blocks.size(); i++)
            CHECK(blocks[i - 1].first + blocks[i - 1].second <= blocks[i].first, "blocks overlap");
        CHECK(used == arena.used(), "arena used %llu, blocks %llu", (unsigned long long)arena.used(),
              (unsigned long long)used);
        CHECK(reserved == st.host_reserved, "reservation drift");
        uint64_t holes = 0;
        for (const auto &h : arena.holes())
            holes += h.second;
        CHECK(holes + used == arena.size(), "holes and blocks do not cover the arena");
        return true;
    }

    // The server's admission loop.
    bool admit()
    {
        for (;;) {
            const long i = next_admissible(queue, st, arena, host_live, info, &blocked);
            if (i < 0)
                return true;
            SimReq *r = queue[(size_t)i];
            // everything earlier in the queue must be a checkpoint held back for host memory
            for (long j = 0; j < i; j++) {
                const SimReq *e = queue[(size_t)j];
                CHECK(e->checkpoint && !r->checkpoint, "request %llu passed request %llu",
                      (unsigned long long)r->seq, (unsigned long long)e->seq);
            }
            if (i > 0) {
                const SimReq *e = queue[0];   // the checkpoints behind it wait in order
                CHECK(st.host_budget && host_live + st.host_reserved + e->host > st.host_budget,
                      "passed checkpoint %llu was not held back", (unsigned long long)e->seq);
            }
            const uint64_t off = arena.alloc(r->dev);
            CHECK(off != UINT64_MAX, "next_admissible chose a block that does not fit");
            queue.erase(queue.begin() + i);
            r->off = off;
            if (r->checkpoint) {
                CHECK(r->seq > last_ckpt_seq, "checkpoint %llu admitted out of order", (unsigned long long)r->seq);
                last_ckpt_seq = r->seq;
                st.host_reserved += r->host;
                CHECK(!st.host_budget || host_live + st.host_reserved <= st.host_budget, "host budget exceeded");
            }
            active.push_back(r);
            st.n_active++;
            admitted++;
            if (!invariants())
                return false;
        }
    }

    static AdmitInfo info(const SimReq *r)
    {
        AdmitInfo a;
        a.checkpoint = r->checkpoint;
        a.dev_bytes = r->dev;
        a.host_bytes = r->host;
        return a;
    }

    void finish(size_t i, std::mt19937_64 &rng)
    {
        SimReq *r = active[i];
        active.erase(active.begin() + (long)i);
        arena.free(r->off, r->dev);
        st.n_active--;
        if (r->checkpoint) {
            st.host_reserved -= r->host;
            r->image = r->host ? rng() % (r->host + 1) : 0;   // zero-chunk elision can shrink it
            held.push_back(r->image);
            host_live += r->image;
        }
        finished++;
        delete r;
    }
};

bool run(uint64_t seed, uint32_t max_active, uint64_t arena_bytes, uint64_t host_budget, int events)
{
    std::mt19937_64 rng(seed);
    Sim s;
    s.st.max_active = max_active;
    s.st.host_budget = host_budget;
    s.arena.reset(arena_bytes);
    auto rnd = [&](uint64_t lo, uint64_t hi) { return lo + rng() % (hi - lo + 1); };
    for (int ev = 0; ev < events || !s.queue.empty() || !s.active.empty(); ev++) {
        const int what = (int)(rng() % 10);
        if (ev < events && what < 4) {
            auto *r = new SimReq();
            r->seq = ++s.submitted;
            r->checkpoint = rng() % 10 < 7;
            r->dev = rnd(1, arena_bytes / 3);
            if (r->checkpoint)
                r->host = host_budget ? rnd(1, host_budget / 2) : rnd(1, 1000);
            s.queue.push_back(r);
        } else if (what < 8 && !s.active.empty()) {
            s.finish(rng() % s.active.size(), rng);
        } else if (!s.held.empty()) {
            // the caller releases an image (more eagerly once no work is left)
            const size_t i = rng() % s.held.size();
            s.host_live -= s.held[i];
            s.held.erase(s.held.begin() + (long)i);
        }
        if (!s.admit() || !s.invariants())
            return false;
        if (ev > 100 * events + 100000) {
            std::fprintf(stderr, "seed %llu: the queue did not drain (queued %zu, active %zu)\n",
                         (unsigned long long)seed, s.queue.size(), s.active.size());
            return false;
        }
    }
    if (s.admitted != s.submitted || s.finished != s.submitted) {
        std::fprintf(stderr, "seed %llu: submitted %llu admitted %llu finished %llu\n", (unsigned long long)seed,
                     (unsigned long long)s.submitted, (unsigned long long)s.admitted,
                     (unsigned long long)s.finished);
        return false;
    }
    return true;
}

// Hand-made cases with known outcomes.
bool cases()
{
    Sim s;
    s.st.max_active = 4;
    s.st.host_budget = 100;
    s.arena.reset(1000);
    s.host_live = 60;                               // images the caller holds
    auto mk = [&](bool ck, uint64_t dev, uint64_t host) {
        auto *r = new SimReq();
        r->seq = ++s.submitted;
        r->checkpoint = ck;
        r->dev = dev;
        r->host = host;
        s.queue.push_back(r);
        return r;
    };
    mk(true, 100, 50);    // 1: waits for host memory (60 + 50 > 100)
    mk(false, 100, 0);    // 2: restore passes it
    mk(true, 100, 10);    // 3: checkpoint behind a waiting one waits too, though it would fit
    mk(false, 901, 0);    // 4: restore whose block does not fit: stops admission
    mk(false, 10, 0);     // 5: waits behind 4
    if (!s.admit())
        return false;
    CHECK(s.active.size() == 1 && s.active[0]->seq == 2 && s.blocked, "case A: %zu admitted", s.active.size());
    s.host_live = 0;                                 // the caller frees its images
    if (!s.admit())
        return false;
    CHECK(s.active.size() == 3 && s.queue.size() == 2 && s.queue[0]->seq == 4, "case B");
    std::mt19937_64 rng(1);
    while (!s.active.empty())
        s.finish(0, rng);
    s.host_live = 0;
    if (!s.admit())
        return false;
    CHECK(s.active.size() == 2 && s.queue.empty(), "case C");
    // max_active bounds admission even when memory is free
    s.st.max_active = 2;
    mk(false, 1, 0);
    if (!s.admit())
        return false;
    CHECK(s.queue.size() == 1, "case D");
    while (!s.active.empty())
        s.finish(0, rng);
    while (!s.queue.empty()) {
        delete s.queue.front();
        s.queue.pop_front();
    }
    return true;
}

}  // namespace

int main()
{
    if (!cases())
        return 1;
    for (uint64_t seed = 1; seed <= 300; seed++) {
        const uint32_t max_active = 1 + (uint32_t)(seed % 16);
        const uint64_t host_budget = seed % 5 == 0 ? 0 : 1000 + seed * 37;
        if (!run(seed, max_active, 5000 + seed * 101, host_budget, 2000))
            return 1;
    }
    std::printf("admission: all checks held\n");
    return g_fail;
}
