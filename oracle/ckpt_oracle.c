/*
 * ckpt_oracle.c -- plain CPU oracle for the device-memory checkpoint path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load or call this code.  The product
 * library (paper_2008_10596_amd/) never includes, links or calls it, and it
 * shares no source, header, table or constant generator with the HIP path.
 *
 * What it computes, and where each rule comes from:
 *
 *  - The paper (CRAC, Jain & Cooperman, Sec. 3.2 "Saving the library-allocated
 *    arena") saves only the memory of the *active mallocs* -- allocations made
 *    and not yet freed at checkpoint time -- and never the allocator's arena.
 *    Sec. 3.2 "restoring the CUDA library-allocated regions" copies that
 *    memory back at restart, and Sec. 3.1 "Log-and-replay" handles regions in
 *    the order they were allocated.  So the image holds exactly the live
 *    allocations' bytes, in allocation order (oracle_layout, oracle_pack).
 *  - The paper fixes no image format, checksum, chunking or delta scheme.
 *    Those are this library's own choices, restated here as plain rules:
 *      * CRC-32C (Castagnoli; reflected polynomial 0x82F63B78, init and
 *        xorout 0xFFFFFFFF) over each chunk, bitwise definition below;
 *      * a dense image: allocation k at offset off_k, where offsets are the
 *        exclusive prefix sum of the sizes rounded up to 16 bytes, pad bytes 0;
 *      * a per-allocation chunk grid of C bytes (the last chunk of an
 *        allocation may be shorter); global chunk id g = cb_k + c where cb is
 *        the exclusive prefix sum of ceil(size_k / C);
 *      * flags[g] = ZERO | DIRTY << 1: ZERO when every byte of the chunk is 0,
 *        DIRTY when there is no base checkpoint or crc[g] differs from it;
 *      * the drained (serialized) data: non-ZERO chunks in ascending g, each
 *        padded with zeros to a multiple of 16 bytes;
 *      * an incremental (delta) image: the ascending list of DIRTY ids and the
 *        DIRTY, non-ZERO chunks' bytes, each padded to 16;
 *      * restore: every chunk is written back (ZERO chunks as zeros) and its
 *        CRC recomputed and compared with the stored one; mismatches are still
 *        written, counted, and the smallest 64 ids reported in ascending order.
 *
 * Everything is done the slow, obvious way: one byte at a time through a
 * 256-entry table (Sarwate's method), which is itself generated from, and
 * tested against, the bit-at-a-time definition.  Threads (pthreads) only split
 * the chunk range, so a timing run can use the host's cores; the result does
 * not depend on the thread count.
 */
#include <pthread.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_POLY_REFLECTED 0x82F63B78u
#define ORACLE_ALIGN 16u
#define ORACLE_FLAG_ZERO 1u
#define ORACLE_FLAG_DIRTY 2u
#define ORACLE_MAX_REPORT 64

/* ---------------------------------------------------------------- CRC-32C */

/* One byte into the register, eight single-bit steps: the definition. */
static uint32_t crc_bitwise_byte(uint32_t r, uint8_t b)
{
    r ^= b;
    for (int i = 0; i < 8; i++)
        r = (r & 1u) ? (r >> 1) ^ ORACLE_POLY_REFLECTED : (r >> 1);
    return r;
}

uint32_t oracle_crc32c_bitwise(const uint8_t *p, size_t n)
{
    uint32_t r = 0xFFFFFFFFu;
    for (size_t i = 0; i < n; i++)
        r = crc_bitwise_byte(r, p[i]);
    return r ^ 0xFFFFFFFFu;
}

static uint32_t crc_table[256];
static pthread_once_t crc_table_once = PTHREAD_ONCE_INIT;

/* table[b] = register after feeding byte b into a zero register. */
static void crc_table_build(void)
{
    for (int b = 0; b < 256; b++)
        crc_table[b] = crc_bitwise_byte(0u, (uint8_t)b);
}

void oracle_crc32c_table(uint32_t out[256])
{
    pthread_once(&crc_table_once, crc_table_build);
    memcpy(out, crc_table, sizeof(crc_table));
}

/* Sarwate: the low byte of (register ^ data byte) indexes the table; the
 * rest of the register moves down by one byte. */
uint32_t oracle_crc32c(const uint8_t *p, size_t n)
{
    pthread_once(&crc_table_once, crc_table_build);
    uint32_t r = 0xFFFFFFFFu;
    for (size_t i = 0; i < n; i++)
        r = crc_table[(r ^ p[i]) & 0xFFu] ^ (r >> 8);
    return r ^ 0xFFFFFFFFu;
}

/* ---------------------------------------------------------------- layout */

static uint64_t round_up16(uint64_t x) { return (x + ORACLE_ALIGN - 1) / ORACLE_ALIGN * ORACLE_ALIGN; }
static uint64_t chunks_of(uint64_t size, uint64_t C) { return (size + C - 1) / C; }

/*
 * Dense layout and chunk grid.  ext_k = roundup16(size_k); off = exclusive
 * prefix sum of ext; nc_k = ceil(size_k / C); cb = exclusive prefix sum of nc.
 * Any output pointer may be NULL.  Returns 0, or -1 when C is not a positive
 * multiple of 16.
 */
int oracle_layout(size_t n, const uint64_t *sizes, uint64_t C,
                  uint64_t *off, uint64_t *cb,
                  uint64_t *data_bytes, uint64_t *n_chunks)
{
    if (C == 0 || C % ORACLE_ALIGN != 0)
        return -1;
    uint64_t o = 0, g = 0;
    for (size_t k = 0; k < n; k++) {
        if (off) off[k] = o;
        if (cb) cb[k] = g;
        o += round_up16(sizes[k]);
        g += chunks_of(sizes[k], C);
    }
    if (data_bytes) *data_bytes = o;
    if (n_chunks) *n_chunks = g;
    return 0;
}

/* Bytes in chunk c of an allocation of `size` bytes: C, except the last. */
static uint64_t chunk_len(uint64_t size, uint64_t C, uint64_t c)
{
    uint64_t rest = size - c * C;
    return rest < C ? rest : C;
}

/* Visits chunk c of allocation k, for every chunk of every allocation in
 * registration order, with g (the global chunk id) counting up from 0. */
#define FOR_EACH_CHUNK(n, sizes, C, k, c, g)                                   \
    for (uint64_t g = 0, k = 0; k < (uint64_t)(n); k++)                        \
        for (uint64_t c = 0; c < chunks_of((sizes)[k], (C)); c++, g++)

static int all_zero(const uint8_t *p, uint64_t n)
{
    for (uint64_t i = 0; i < n; i++)
        if (p[i] != 0)
            return 0;
    return 1;
}

/* --------------------------------------------------------- per-chunk pass */

typedef struct {
    size_t n;
    const uint8_t *const *src;
    const uint64_t *sizes;
    uint64_t C;
    const uint32_t *base_crc;   /* NULL: first checkpoint, every chunk DIRTY */
    uint32_t *crc;
    uint8_t *flags;
    uint64_t g_begin, g_end;
} chunk_job;

static void *chunk_worker(void *arg)
{
    chunk_job *j = (chunk_job *)arg;
    FOR_EACH_CHUNK(j->n, j->sizes, j->C, k, c, g) {
        uint64_t len = chunk_len(j->sizes[k], j->C, c);
        if (g < j->g_begin || g >= j->g_end)
            continue;
        const uint8_t *p = j->src[k] + c * j->C;
        uint32_t crc = oracle_crc32c(p, len);
        uint8_t f = 0;
        if (all_zero(p, len))
            f |= ORACLE_FLAG_ZERO;
        if (j->base_crc == NULL || j->base_crc[g] != crc)
            f |= ORACLE_FLAG_DIRTY;
        j->crc[g] = crc;
        j->flags[g] = f;
    }
    return NULL;
}

/* Runs chunk_worker over [0, N) split into `threads` equal ranges. */
static int run_chunks(chunk_job *proto, uint64_t N, int threads)
{
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > N) threads = N ? (int)N : 1;
    pthread_t *tid = calloc((size_t)threads, sizeof(pthread_t));
    chunk_job *jobs = calloc((size_t)threads, sizeof(chunk_job));
    if (!tid || !jobs) { free(tid); free(jobs); return -1; }
    for (int t = 0; t < threads; t++) {
        jobs[t] = *proto;
        jobs[t].g_begin = N * (uint64_t)t / (uint64_t)threads;
        jobs[t].g_end = N * (uint64_t)(t + 1) / (uint64_t)threads;
    }
    int started = 0, rc = 0;
    for (int t = 1; t < threads; t++) {
        if (pthread_create(&tid[t], NULL, chunk_worker, &jobs[t]) != 0) { rc = -1; break; }
        started = t;
    }
    chunk_worker(&jobs[0]);
    for (int t = 1; t <= started; t++)
        pthread_join(tid[t], NULL);
    if (rc != 0) /* a thread failed to start: do its range here */
        for (int t = started + 1; t < threads; t++)
            chunk_worker(&jobs[t]);
    free(tid);
    free(jobs);
    return 0;
}

/*
 * Full checkpoint.  Inputs: n host copies of the live allocations in
 * registration order (src[k], sizes[k]), chunk size C, optional base CRC array
 * (N entries) for DIRTY.  Outputs (each may be NULL except crc/flags):
 *   dense[data_bytes]      allocation bytes at off_k, pad bytes zero;
 *   crc[N], flags[N];
 *   ser[...]               non-ZERO chunks, ascending g, each padded to 16;
 *   *ser_bytes             its length.
 * Returns 0, -1 on bad C, -2 on allocation failure.
 */
int oracle_checkpoint(size_t n, const uint8_t *const *src, const uint64_t *sizes,
                      uint64_t C, const uint32_t *base_crc, int threads,
                      uint8_t *dense, uint32_t *crc, uint8_t *flags,
                      uint8_t *ser, uint64_t *ser_bytes)
{
    uint64_t data_bytes = 0, N = 0;
    if (oracle_layout(n, sizes, C, NULL, NULL, &data_bytes, &N) != 0)
        return -1;

    chunk_job proto = {n, src, sizes, C, base_crc, crc, flags, 0, 0};
    if (run_chunks(&proto, N, threads) != 0)
        return -2;

    if (dense) {
        uint64_t o = 0;
        for (size_t k = 0; k < n; k++) {
            memcpy(dense + o, src[k], sizes[k]);
            memset(dense + o + sizes[k], 0, round_up16(sizes[k]) - sizes[k]);
            o += round_up16(sizes[k]);
        }
    }

    uint64_t s = 0;
    FOR_EACH_CHUNK(n, sizes, C, k, c, g) {
        uint64_t len = chunk_len(sizes[k], C, c);
        if (flags[g] & ORACLE_FLAG_ZERO)
            continue;
        if (ser) {
            memcpy(ser + s, src[k] + c * C, len);
            memset(ser + s + len, 0, round_up16(len) - len);
        }
        s += round_up16(len);
    }
    if (ser_bytes) *ser_bytes = s;
    return 0;
}

/*
 * Incremental checkpoint against a base with the same allocation table and C.
 * crc/flags get the full new arrays; dirty_ids gets the ascending ids with
 * crc != base_crc (every DIRTY chunk, ZERO or not); delta gets the DIRTY,
 * non-ZERO chunks' bytes, each padded to 16.  dirty_ids / delta may be NULL.
 */
int oracle_delta(size_t n, const uint8_t *const *src, const uint64_t *sizes,
                 uint64_t C, const uint32_t *base_crc, int threads,
                 uint32_t *crc, uint8_t *flags,
                 uint64_t *dirty_ids, uint64_t *n_dirty,
                 uint8_t *delta, uint64_t *delta_bytes)
{
    if (base_crc == NULL)
        return -1;
    uint64_t N = 0;
    if (oracle_layout(n, sizes, C, NULL, NULL, NULL, &N) != 0)
        return -1;
    chunk_job proto = {n, src, sizes, C, base_crc, crc, flags, 0, 0};
    if (run_chunks(&proto, N, threads) != 0)
        return -2;

    uint64_t nd = 0, s = 0;
    FOR_EACH_CHUNK(n, sizes, C, k, c, g) {
        uint64_t len = chunk_len(sizes[k], C, c);
        if (!(flags[g] & ORACLE_FLAG_DIRTY))
            continue;
        if (dirty_ids) dirty_ids[nd] = g;
        nd++;
        if (flags[g] & ORACLE_FLAG_ZERO)
            continue;
        if (delta) {
            memcpy(delta + s, src[k] + c * C, len);
            memset(delta + s + len, 0, round_up16(len) - len);
        }
        s += round_up16(len);
    }
    if (n_dirty) *n_dirty = nd;
    if (delta_bytes) *delta_bytes = s;
    return 0;
}

/* ---------------------------------------------------------------- restore */

/* Keeps the count of bad chunks and the smallest ORACLE_MAX_REPORT ids. */
typedef struct {
    uint64_t count;
    uint64_t n_ids;
    uint64_t ids[ORACLE_MAX_REPORT];
} bad_report;

static void report_bad(bad_report *rep, uint64_t g)
{
    /* ids arrive in ascending order in this oracle, so the first 64 are the
     * smallest 64 */
    if (rep->n_ids < ORACLE_MAX_REPORT)
        rep->ids[rep->n_ids++] = g;
    rep->count++;
}

/* One chunk back: ZERO -> zeros; else the next serialized piece.  The CRC of
 * what was written is recomputed and compared with the stored one. */
static void restore_chunk(uint8_t *dst, uint64_t len, uint8_t flag, uint32_t want,
                          const uint8_t *piece, uint64_t g, bad_report *rep)
{
    if (flag & ORACLE_FLAG_ZERO)
        memset(dst, 0, len);
    else
        memcpy(dst, piece, len);
    if (oracle_crc32c(dst, len) != want)
        report_bad(rep, g);
}

/*
 * Full restore into n destination buffers (host memory here), dst[k] of
 * sizes[k] bytes, from crc/flags and the serialized data.  Returns 0 when all
 * chunks verify, 1 when some do not (bad count / ids written), -1 when the
 * serialized data is shorter than the flags require.
 */
int oracle_restore(size_t n, const uint64_t *sizes, uint64_t C,
                   const uint32_t *crc, const uint8_t *flags,
                   const uint8_t *ser, uint64_t ser_bytes,
                   uint8_t *const *dst,
                   uint64_t *bad_count, uint64_t *bad_ids, uint64_t *n_bad_ids)
{
    uint64_t N = 0;
    if (oracle_layout(n, sizes, C, NULL, NULL, NULL, &N) != 0)
        return -1;
    bad_report rep;
    memset(&rep, 0, sizeof(rep));
    uint64_t s = 0;
    FOR_EACH_CHUNK(n, sizes, C, k, c, g) {
        uint64_t len = chunk_len(sizes[k], C, c);
        const uint8_t *piece = NULL;
        if (!(flags[g] & ORACLE_FLAG_ZERO)) {
            if (s + round_up16(len) > ser_bytes)
                return -1;
            piece = ser + s;
            s += round_up16(len);
        }
        restore_chunk(dst[k] + c * C, len, flags[g], crc[g], piece, g, &rep);
    }
    if (bad_count) *bad_count = rep.count;
    if (n_bad_ids) *n_bad_ids = rep.n_ids;
    if (bad_ids) memcpy(bad_ids, rep.ids, rep.n_ids * sizeof(uint64_t));
    return rep.count ? 1 : 0;
}

/*
 * Delta overlay: after a full restore of the base, each DIRTY id in ascending
 * order gets the delta's rule (ZERO -> zeros, else the next delta piece) and
 * is verified against the delta's CRC.  Same return convention.
 */
int oracle_restore_delta(size_t n, const uint64_t *sizes, uint64_t C,
                         const uint32_t *crc, const uint8_t *flags,
                         const uint64_t *dirty_ids, uint64_t n_dirty,
                         const uint8_t *delta, uint64_t delta_bytes,
                         uint8_t *const *dst,
                         uint64_t *bad_count, uint64_t *bad_ids, uint64_t *n_bad_ids)
{
    uint64_t N = 0;
    if (oracle_layout(n, sizes, C, NULL, NULL, NULL, &N) != 0)
        return -1;
    bad_report rep;
    memset(&rep, 0, sizeof(rep));
    for (uint64_t i = 0; i < n_dirty; i++)
        if (dirty_ids[i] >= N || (i > 0 && dirty_ids[i] <= dirty_ids[i - 1]))
            return -1;
    uint64_t s = 0, i = 0;
    FOR_EACH_CHUNK(n, sizes, C, k, c, g) {
        uint64_t len = chunk_len(sizes[k], C, c);
        if (i == n_dirty || dirty_ids[i] != g)
            continue;
        i++;
        const uint8_t *piece = NULL;
        if (!(flags[g] & ORACLE_FLAG_ZERO)) {
            if (s + round_up16(len) > delta_bytes)
                return -1;
            piece = delta + s;
            s += round_up16(len);
        }
        restore_chunk(dst[k] + c * C, len, flags[g], crc[g], piece, g, &rep);
    }
    if (bad_count) *bad_count = rep.count;
    if (n_bad_ids) *n_bad_ids = rep.n_ids;
    if (bad_ids) memcpy(bad_ids, rep.ids, rep.n_ids * sizeof(uint64_t));
    return rep.count ? 1 : 0;
}
