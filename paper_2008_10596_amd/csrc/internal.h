// internal.h -- shared declarations of libckpt's HIP kernels and host runtime.
//
// Not part of the public ABI (that is include/ckpt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ckpt {

// CRC-32C, reflected form of the Castagnoli polynomial.
constexpr uint32_t kPolyReflected = 0x82F63B78u;

// Shift-operator tables.  Every operator "feed m zero bytes through the CRC
// register" is 4 x 256 words: S[j][b] is the operator applied to the register
// value b << 8j, so applying it to v is the XOR of the four entries picked by
// v's bytes.  The chunk kernels read a chunk in rounds of 1 KiB: in one round
// lane l of a wave hashes the 16-byte piece l of the round.
constexpr int kTabWords = 1024;     // one operator, 4 x 256 words
constexpr int kTreeLevels = 6;      // cross-lane tree: m = 16 << k, k = 0..5
constexpr int kRoundBytes = 1024;   // one wave64 x 16-byte load

// The table set staged in LDS (one 1024-thread workgroup per CU):
// random-index lookups are bank-conflict free when each lane reads its own
// copy of an entry.  Byte offsets in LDS:
//   round operator (m = 1024: a lane's register one round later, for the
//   Horner combine of its per-round registers), 8 copies:
//                             (j << 13) | (b << 5) | ((lane & 7) << 2)     [0, 32 KiB)
//   2-byte chain step, 32 copies, both byte positions interleaved:
//                             32768 + ((b << 8) | (t << 7) | ((lane & 31) << 2))  [32, 96 KiB)
//   from 96 KiB, single copies: the six tree operators, then the cross-wave
//   operator (m = rounds per wave x 1 KiB).
constexpr int kRepGapBytes = 32768;
constexpr int kRepChainOff = 32768;
constexpr int kRepTreeOff = 98304;                         // bytes
constexpr int kRepWords = (kRepTreeOff / 4) + (kTreeLevels + 1) * kTabWords;   // 124 KiB

// The quad form of the hash-only pass (chunks of at most four rounds): each
// row of kQuadLanes lanes hashes its own chunk, and lane l of a row reads the
// pieces at l * 16 of every kQuadLanes * 16-byte stretch.  Its table set is
// the replicated one with the gap operator replaced by a skip: the last word
// of a piece moves the register 4 bytes and over the other lanes' pieces of
// that stretch, kQuadSkipBytes in all.
constexpr int kQuadLanes = 16;
constexpr uint32_t kQuadSkipBytes = 4 + (kQuadLanes - 1) * 16;
constexpr int kFlagZero = 1;
constexpr int kFlagDirty = 2;

// Counts the kernels read from device memory, so that one captured graph
// serves any table that fits the buffers it was captured with.
struct DevPlan {
    uint64_t n_allocs;    // rows in the allocation table
    uint64_t n_chunks;    // N, written by the layout scan
    uint64_t data_bytes;  // dense bytes, written by the layout scan
    uint64_t n_items;     // items of a restore pass (N, or the delta's id count)
    uint64_t sel_bytes;   // selection scan: total selected bytes
    uint64_t sel_count;   // selection scan: total selected ids
    unsigned long long bad_count;  // restore: chunks that failed verification
    unsigned long long tile_next;  // chunk launches: the next tile to take (zero between launches)
    unsigned long long gather_next;  // gather launches: the same for the gather's tiles
};

enum ChunkMode { kModePack = 0, kModeHash = 1, kModeRestore = 2 };

constexpr uint64_t kNoBase = ~0ull;

struct ChunkArgs {
    const DevPlan *plan;
    const uint32_t *tables;   // kRepWords words
    const uint32_t *tables_quad;   // nullable: the quad form's set
    uint32_t C;
    uint32_t waves_per_chunk;
    uint32_t nontemporal;     // 1: streaming loads/stores for the bulk data
    uint32_t pad1;
    // allocation table (n rows; off and cb have n + 1)
    const uint64_t *src;      // pack/hash: source address of each allocation
    const uint64_t *dst;      // restore: destination address of each allocation
    const uint64_t *size;
    const uint64_t *off;
    const uint64_t *cb;
    const uint32_t *map;      // chunk id -> allocation row
    // pack / hash outputs
    uint8_t *dense;           // pack: dense image
    uint32_t *crc;
    uint8_t *flags;
    const uint32_t *base_crc; // nullable
    const uint64_t *base_cb;  // nullable: the base's first chunk id for each
                              // allocation (kNoBase: no matching allocation in
                              // the base); null = the base has this table
    // restore inputs
    const uint8_t *staging;   // serialized chunks
    const uint64_t *soff;     // item -> offset in staging
    const uint32_t *want_crc;
    const uint8_t *want_flags;
    const uint64_t *ids;      // nullable: item i is chunk ids[i], else chunk i
    uint32_t zero_crc;        // CRC-32C of C zero bytes.  Restore: a full-length ZERO
                              // chunk is written as zeros and checked against it
                              // without hashing the zeros.  Pack (one wave per chunk
                              // of at most four rounds): a full-length ZERO chunk
                              // gets it as its CRC and is neither hashed nor stored
    uint32_t pad0;
    uint8_t *bad;             // per chunk, set to 1 when verification fails
    DevPlan *plan_rw;         // bad_count lives here
    // restore by segments: items [item_begin, item_end) when item_end != 0
    // (else all items of the plan); staging holds the serialized bytes from
    // offset soff_base on
    uint64_t item_begin, item_end, soff_base;
};

// Row-mode chunk launch (the serving loop): each row is a run of chunks of
// one allocation of one request, with its own addresses, so one launch can
// mix chunks of many requests, some packed and some restored.
struct StepRow {
    uint64_t src;        // pack: address of the row's first chunk; restore: staging base
    uint64_t dst;        // pack: dense-image address of the first chunk; restore: its destination
    uint64_t rem;        // bytes from the row's first chunk to the end of its allocation
    uint64_t item0;      // first item of the row in the launch
    uint64_t crc;        // uint32_t *: pack: CRC out; restore: stored CRC (first chunk)
    uint64_t flags;      // uint8_t *: pack: flags out; restore: stored flags
    uint64_t soff;       // const uint64_t *: restore: serialized offset of each chunk
    uint64_t bad;        // uint8_t *: restore: bad marks
    uint64_t bad_count;  // unsigned long long *: restore: the request's counter
    uint32_t mode;       // kModePack or kModeRestore
    uint32_t pad;
};

struct RowArgs {
    const uint32_t *tables;
    uint32_t C;
    uint32_t nontemporal;
    uint64_t n_items;
    const StepRow *rows;
    const uint32_t *map;   // item -> row
    unsigned long long *tile_ctr;   // the step plan's tile_next (zero at launch)
};

enum SelMode {
    kSelNonZero = 0,       // bytes: !ZERO chunks;            count: none
    kSelDirtyNonZero = 1,  // bytes: DIRTY && !ZERO chunks;   count: DIRTY chunks (ids out)
    kSelIdsNonZero = 2,    // items are ids[i]; bytes: !ZERO;  count: none
    kSelBad = 3            // bytes: none;                     count: bad chunks (ids out)
};

struct SelArgs {
    DevPlan *plan;
    int mode;
    uint32_t C;
    const uint64_t *size;
    const uint64_t *cb;
    const uint32_t *map;
    const uint8_t *flags;     // flags of the chunks (or bad[] for kSelBad)
    const uint64_t *ids;      // kSelIdsNonZero
    uint64_t *tile_bytes;     // per tile totals, then bases
    uint64_t *tile_count;
    uint64_t *soff;           // per item: exclusive prefix of selected bytes
    uint64_t *ids_out;        // selected ids, ascending (count side)
    uint64_t ids_cap;         // capacity of ids_out
};

constexpr int kSelThreads = 256;
constexpr int kSelPerThread = 16;
constexpr int kSelTile = kSelThreads * kSelPerThread;

struct GatherArgs {
    const DevPlan *plan;
    int mode;                 // kSelNonZero or kSelDirtyNonZero: which chunks
    int from_dense;           // 1: read the dense image; 0: read the allocations
    uint32_t C;
    const uint64_t *src;
    const uint64_t *size;
    const uint64_t *off;
    const uint64_t *cb;
    const uint32_t *map;
    const uint8_t *dense;
    const uint8_t *flags;
    const uint64_t *soff;
    uint8_t *out;             // device buffer or mapped pinned host buffer
    int out_host;             // 1: out is pinned host memory
    // by segments: chunks [g_begin, g_end) when g_end != 0 (else all chunks
    // of the plan); out holds the serialized bytes from offset soff_base on
    uint64_t g_begin, g_end, soff_base;
    uint32_t tile;            // chunks per tile (1 .. 64, a power of two); set by launch_gather
    uint32_t pad;
    unsigned long long *tile_ctr;   // the plan's gather_next; set by launch_gather
    // Several outputs straight into host memory (the drain inside the batched
    // graph), when out_addr is not null: chunk g of allocation row k belongs
    // to output o = row_out[k], whose serialized bytes start at host address
    // out_addr[o]; g's bytes go to out_addr[o] + soff[g] - soff[out_chunk0[o]]
    // (out and soff_base are unused).
    const uint64_t *out_addr;
    const uint32_t *row_out;
    const uint64_t *out_chunk0;
};

// Launch wrappers (kernels.hip).  All return the hipError_t of the launch.
hipError_t launch_layout_scan(hipStream_t s, DevPlan *plan, const uint64_t *size, uint32_t C,
                              uint64_t *off, uint64_t *cb);
// The same scan over a table in pinned host memory (`up`: a plan header,
// then n addresses, then n sizes, n from the header), which it also copies
// to plan, addr and size.  The host must not rewrite `up` until the stream
// has passed the launch.
hipError_t launch_upload_scan(hipStream_t s, const void *up, DevPlan *plan, uint64_t *addr, uint64_t *size,
                              uint32_t C, uint64_t *off, uint64_t *cb);
hipError_t launch_chunk_map(hipStream_t s, const DevPlan *plan, const uint64_t *cb, uint32_t *map,
                            int grid);
hipError_t launch_chunks(hipStream_t s, int mode, const ChunkArgs &a, int grid, int block);
hipError_t launch_rows(hipStream_t s, const RowArgs &a, int grid, int block);
hipError_t launch_select(hipStream_t s, const SelArgs &a, uint64_t max_items);
// grid: workgroups of 1024 threads (persistent; two per CU fill the chip)
hipError_t launch_gather(hipStream_t s, const GatherArgs &a, int grid);
hipError_t launch_fill_u64(hipStream_t s, uint64_t *p, uint64_t n_words, uint64_t value);
// rows: n rows of four u64 words (id, kind, address, size); writes addr[n],
// size[n] and a plan with n_allocs = n and every other count 0.
hipError_t launch_table_split(hipStream_t s, const uint64_t *rows, uint64_t n, DevPlan *plan, uint64_t *addr,
                              uint64_t *size);
hipError_t launch_pick_u64(hipStream_t s, const uint64_t *src, const uint64_t *idx, uint64_t *out,
                           uint32_t m);

// Host-side table generation (crc_tables.cpp): the set of kRepWords words
// for `rounds_per_wave` consecutive rounds per wave; its round operator moves
// the register gap_bytes forward (kRoundBytes, or kQuadSkipBytes for the quad
// form).
void build_tables_replicated(uint32_t *out, uint32_t rounds_per_wave, uint32_t gap_bytes = kRoundBytes);
// Register after feeding nbytes zero bytes (host, for tests of the tables).
uint32_t host_shift(uint32_t reg, uint64_t nbytes);

}  // namespace ckpt
