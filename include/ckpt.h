/*
 * ckpt.h -- C ABI of libckpt: drain live device allocations into a checkpoint
 * image on an AMD Instinct MI355X (gfx950), and refill them from it.
 *
 * The operation is the one CRAC (Jain & Cooperman, "CRAC: Checkpoint-Restart
 * Architecture for CUDA with Streams and UVM") performs on the GPU side of a
 * checkpoint:
 *   - the library logs the pointers returned by the allocation calls of the
 *     cudaMalloc family, not the allocator's mmap calls (Sec. 3.2, "Issue of
 *     library-allocated memory");
 *   - at checkpoint time it saves only the memory of the *active mallocs*,
 *     allocations made and not yet freed, never the allocator's arena
 *     (Sec. 3.2, "Saving the library-allocated arena"), and handles them in
 *     the order in which they were allocated (Sec. 3.1, "Log-and-replay");
 *   - device (cudaMalloc) and managed (cudaMallocManaged) regions are written
 *     out when the checkpoint is taken and put back on restart (Sec. 3.2,
 *     "restoring the CUDA library-allocated regions");
 *   - before copying, the queue of pending GPU work is drained, as CheCUDA's
 *     first step does with a device-wide synchronize (Sec. 2.2).
 * Here the caller mirrors its allocation calls with ckpt_register /
 * ckpt_unregister (the log), ckpt_checkpoint drains the live set into an
 * image, and ckpt_restore refills fresh buffers from it.
 *
 * The image format, the per-chunk CRC-32C, the ZERO/DIRTY flags, incremental
 * images, batching and serving are this library's design; the paper fixes
 * none of them.  Their exact definitions are given next to each call below.
 *
 * Conventions for every call:
 *   - Return value: CKPT_OK (0) or a negative ckpt_status.  Out-parameters
 *     are written only on success, except ckpt_restore's report, which is
 *     also written with CKPT_E_CORRUPT.
 *   - Device pointers are plain virtual addresses in the HIP device's address
 *     space (e.g. from hipMalloc, hipMallocManaged, or a PyTorch tensor's
 *     data_ptr()).  Host pointers are plain process addresses.
 *   - A stream argument is a hipStream_t passed as `void *`; NULL means the
 *     device's null stream.
 *   - Sizes are in bytes.
 *   - The caller owns all registered and destination memory; the library never
 *     frees or reallocates it.  Images belong to the caller and are freed with
 *     ckpt_image_free; a view of an image stays valid until then.  A context
 *     owns its device staging, pinned host buffers, tables and side stream.
 *   - A context is used by one thread at a time.  ckpt_server_* calls are
 *     thread-safe.
 *   - After CKPT_E_HIP, ckpt_last_hip_error() / ckpt_last_error() describe
 *     the failing HIP call (thread-local).
 */
#ifndef CKPT_H
#define CKPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ckpt_ctx ckpt_ctx;
typedef struct ckpt_image ckpt_image;
typedef struct ckpt_server ckpt_server;

/* Registration sequence number: 1, 2, 3, ... in ckpt_register order within a
 * context, never reused.  The live set is always ordered by id. */
typedef uint64_t ckpt_id;

enum ckpt_kind {
    CKPT_DEVICE = 0,   /* memory from hipMalloc (or a device tensor)      */
    CKPT_MANAGED = 1   /* memory from hipMallocManaged                      */
};

enum ckpt_mode {
    CKPT_FULL = 0,         /* every live chunk                                */
    CKPT_INCREMENTAL = 1   /* only chunks whose CRC differs from a base image */
};

enum ckpt_status {
    CKPT_OK = 0,
    CKPT_E_INVAL = -1,     /* bad argument, alignment, overlap, truncated image   */
    CKPT_E_NOTFOUND = -2,  /* unregister of a pointer that is not registered      */
    CKPT_E_NOMEM = -3,     /* device, host or pinned allocation failed            */
    CKPT_E_HIP = -4,       /* a HIP runtime call failed                          */
    CKPT_E_MISMATCH = -5,  /* image / base / destination shapes disagree         */
    CKPT_E_CORRUPT = -6,   /* restore: some chunk's CRC did not verify           */
    CKPT_E_AGAIN = -7,     /* server: request not finished yet                   */
    CKPT_E_BUDGET = -8,    /* request larger than the staging budget              */
    CKPT_E_ADDR = -9,      /* the address range asked for is not free               */
    CKPT_E_IO = -10        /* a file could not be created, written or read          */
};

/* ckpt_config.flags */
#define CKPT_STREAM_ORDERED 0x1u  /* order the checkpoint after work on the given
                                     stream only; the caller promises that no
                                     other stream writes registered memory.
                                     Default: device-wide drain first.          */
#define CKPT_KEEP_DENSE     0x2u  /* each image keeps its dense device copy
                                     (section CKPT_SEC_DENSE)                    */
#define CKPT_NO_DRAIN       0x4u  /* stop after pack + CRC: the image holds CRC,
                                     flags and the dense device copy, and no host
                                     DATA.  Without CKPT_KEEP_DENSE the dense copy
                                     is the context's staging, valid until the
                                     context's next checkpoint or restore.       */
#define CKPT_TIMING         0x8u  /* record HIP events around each phase;
                                     read them with ckpt_last_timing             */
#define CKPT_DRAIN_DIRECT   0x10u /* drain by kernel stores straight into pinned
                                     host memory instead of gather + copy engine */
#define CKPT_GRAPH          0x20u /* ckpt_checkpoint: replay a captured hipGraph of
                                     the table upload, size scan, chunk map and
                                     pack, and of the drain's select and gather
                                     into pinned host memory (full checkpoints
                                     without a base)                              */
#define CKPT_NO_GRAPH       0x40u /* ckpt_checkpoint_batch: plain launches instead
                                     of the captured graph it uses by default    */
#define CKPT_RESERVE_STAGING 0x80u /* ckpt_init allocates the whole staging_budget
                                     (which must be set) as one device block at
                                     once: the dense image at its start, a drain's
                                     or restore's segment slots after it.  Later
                                     checkpoints and restores that fit allocate no
                                     device staging, and the block takes its place
                                     before the application's later allocations. */

typedef struct ckpt_config {
    int32_t device;            /* HIP device ordinal                                  */
    uint32_t chunk_bytes;      /* C: a multiple of 16, 16 .. 2^30; 0 selects 4096     */
    uint64_t staging_budget;   /* cap on device staging bytes held by the context
                                  (dense image + compact drain buffer); 0 = no cap    */
    uint32_t flags;            /* CKPT_* flags above                                  */
    uint32_t block_threads;    /* threads per workgroup for the chunk kernels:
                                  64, 128, 256, 512 or 1024; 0 selects 1024          */
    uint32_t waves_per_chunk;  /* waves that share one chunk (1, 2, 4, 8 or 16,
                                  at most block_threads / 64); 0 selects 1            */
    uint32_t wgs_per_cu;       /* persistent workgroups per compute unit; 0 selects 1
                                  (the LDS tables fit one workgroup per CU)           */
    uint32_t lane_pieces;      /* 16-byte pieces each lane hashes per round: 1 (0
                                  selects 1; other values are CKPT_E_INVAL)           */
    uint32_t load_hint;        /* bulk loads/stores: 1 regular, 2 non-temporal;
                                  0 selects 2, except for a pack whose live bytes
                                  mostly sit in allocations whose dense image
                                  starts off a 128-byte line (many allocations of
                                  arbitrary sizes): there 1                      */
    uint32_t table_mode;       /* CRC operator tables in LDS: 2, replicated per lane
                                  (124 KiB, bank-conflict-free lookups, one workgroup
                                  per CU); 0 selects 2, other values are
                                  CKPT_E_INVAL.  block_threads 0 selects 1024         */
    uint32_t segment_mib;      /* a full checkpoint's drain (gather, then copy to the
                                  host) and a restore's refill (copy to the device,
                                  then scatter) go in segments of about this many MiB,
                                  so that the device work of one segment overlaps the
                                  host-link copy of another and at most four segments
                                  are staged on the device; 0 selects 256;
                                  0xFFFFFFFF: one pass (the whole serialized image is
                                  staged)                                              */
} ckpt_config;

/* One row of an image's allocation table (section CKPT_SEC_ALLOCS). */
typedef struct ckpt_alloc_rec {
    uint64_t id;      /* registration id                                   */
    uint32_t kind;    /* ckpt_kind                                         */
    uint32_t pad;     /* 0                                                 */
    uint64_t size;    /* bytes                                             */
    uint64_t off;     /* offset in the dense image: exclusive prefix sum of
                         sizes rounded up to 16                            */
    uint64_t cb;      /* first global chunk id: exclusive prefix sum of
                         ceil(size / C)                                    */
} ckpt_alloc_rec;

typedef struct ckpt_image_meta {
    uint32_t mode;              /* CKPT_FULL or CKPT_INCREMENTAL                    */
    uint32_t chunk_bytes;       /* C                                                */
    uint64_t n_allocs;          /* rows in CKPT_SEC_ALLOCS                          */
    uint64_t n_chunks;          /* N = sum of ceil(size / C)                        */
    uint64_t data_bytes;        /* dense image bytes = sum of roundup16(size)       */
    uint64_t serialized_bytes;  /* bytes in CKPT_SEC_DATA                           */
    uint64_t n_dirty;           /* entries in CKPT_SEC_DIRTY_IDS (incremental)      */
    uint64_t serial;            /* unique per image within the process              */
    uint64_t base_serial;       /* incremental: serial of the base; else 0          */
    uint64_t crc_digest;        /* FNV-1a over the CRC section's 64-bit words       */
    uint32_t has_dense;         /* 1 when CKPT_SEC_DENSE is available               */
    uint32_t drained;           /* 1 when CKPT_SEC_DATA is valid                    */
} ckpt_image_meta;

enum ckpt_section {
    CKPT_SEC_ALLOCS = 0,    /* host, ckpt_alloc_rec[n_allocs]                         */
    CKPT_SEC_CRC = 1,       /* host, uint32_t[N]: CRC-32C of each chunk's bytes        */
    CKPT_SEC_FLAGS = 2,     /* host, uint8_t[N]: bit0 ZERO (all bytes 0), bit1 DIRTY   */
                            /* (no base, or CRC differs from the base's); others 0      */
    CKPT_SEC_DATA = 3,      /* host (pinned), serialized bytes: full image = non-ZERO   */
                            /* chunks in ascending id; incremental = DIRTY non-ZERO     */
                            /* chunks; each chunk padded with zeros to a multiple of 16 */
    CKPT_SEC_DIRTY_IDS = 4, /* host, uint64_t[n_dirty]: ascending ids of DIRTY chunks   */
    CKPT_SEC_DENSE = 5,     /* DEVICE pointer, data_bytes: allocation k at off_k, the   */
                            /* pad of non-ZERO chunks zero; a ZERO chunk's bytes (and   */
                            /* its pad) are unspecified, read them as zeros (the pack   */
                            /* of chunks of at most 4 KiB does not store ZERO chunks)   */
                            /* (with CKPT_KEEP_DENSE or CKPT_NO_DRAIN)                  */
    CKPT_SEC_ADDRS = 6      /* host, uint64_t[n_allocs]: device address of allocation k */
                            /* when the image was taken (0 if loaded from version-1     */
                            /* serialized data); used by ckpt_restore_at                 */
};

#define CKPT_REPORT_MAX 64
typedef struct ckpt_verify_report {
    uint64_t n_bad;                 /* chunks whose CRC did not verify            */
    uint64_t n_ids;                 /* min(n_bad, CKPT_REPORT_MAX)                */
    uint64_t ids[CKPT_REPORT_MAX];  /* the smallest bad chunk ids, ascending      */
} ckpt_verify_report;

/* Per-phase times of the last checkpoint / restore on a context (needs
 * CKPT_TIMING), measured with HIP events on the streams that ran each phase. */
typedef struct ckpt_timing {
    float order_ms;       /* device-wide drain of prior work                     */
    float layout_ms;      /* descriptor upload + size scan + chunk map            */
    float pack_ms;        /* fused pack + CRC + flags (or hash-only) kernel; with a
                             replayed graph, the whole graph (upload, scan, map,
                             pack, and a drain's select and gather into host
                             memory) and layout_ms is 0                            */
    float select_ms;      /* flag scan / compaction                                */
    float gather_ms;      /* gather of selected chunks, summed over the segments    */
    float d2h_ms;         /* device-to-host copy of data + metadata: from the start
                             of the first copy to the end of the last            */
    float h2d_ms;         /* restore: host-to-device copy, first start to last end */
    float scatter_ms;     /* restore: scatter + verify kernel(s), summed over the
                             segments                                              */
    float total_ms;       /* whole call                                            */
    float pad;
    uint64_t pack_read_bytes;     /* algorithmic bytes read by the pack kernel      */
    uint64_t pack_write_bytes;    /* algorithmic bytes written by the pack kernel   */
    uint64_t link_bytes;          /* bytes over the host link                      */
} ckpt_timing;

/* --------------------------------------------------------------- context */

/* Create a context on cfg->device.  cfg may be NULL (device 0, defaults).
 * CKPT_E_INVAL: chunk_bytes not a multiple of 16 / out of range, bad
 * block_threads or waves_per_chunk.  CKPT_E_HIP: no such device. */
int ckpt_init(const ckpt_config *cfg, ckpt_ctx **out);

/* Release the context's staging, pinned buffers, streams.  NULL is a no-op.
 * Registered memory is the caller's and is not touched. */
void ckpt_destroy(ckpt_ctx *ctx);

/* Log one allocation, after the caller's own hipMalloc/hipMallocManaged
 * (mirrors the paper's log of cudaMalloc-family pointers, Sec. 3.2).
 * ptr must be 16-byte aligned; bytes may be 0; [ptr, ptr+bytes) must not
 * overlap a live registration; kind is a ckpt_kind.  *out gets the id.
 * CKPT_E_INVAL on a violation.  The memory is not read until a checkpoint. */
int ckpt_register(ckpt_ctx *ctx, void *ptr, size_t bytes, int kind, ckpt_id *out);

/* Remove the live registration that starts at ptr, before the caller frees it
 * (mirrors the logged free that ends an active malloc, Sec. 3.2).
 * CKPT_E_NOTFOUND if no live registration starts at ptr. */
int ckpt_unregister(ckpt_ctx *ctx, void *ptr);

/* Number of live registrations. */
int ckpt_live_count(const ckpt_ctx *ctx, size_t *out);

/* ------------------------------------------------------------ checkpoint */

/*
 * Drain every live registration, in id order, into a new image.
 *
 * Ordering: the image reflects all work enqueued on the device before the
 * call (device-wide synchronize first, as in the paper's Sec. 2.2), or with
 * CKPT_STREAM_ORDERED only the work enqueued on `stream` before the call.
 * The packing kernel runs on `stream`; once it ends, `stream` may run new
 * work, which does not affect the image: the drain to pinned host memory runs
 * on the context's side stream from the dense device copy.  The call returns
 * when the image is complete.
 *
 * mode CKPT_FULL: base may be NULL (every chunk DIRTY) or an image of the same
 *   chunk size (DIRTY against it).  DATA = non-ZERO chunks.
 * mode CKPT_INCREMENTAL: base is required and must have the same chunk size,
 *   else CKPT_E_MISMATCH.  DATA = DIRTY non-ZERO chunks; DIRTY_IDS = every
 *   DIRTY chunk; CRC and FLAGS are complete, so the result can be the base of
 *   the next increment.
 * The allocation table may differ from the base's (allocations made and
 * freed in between): a chunk is compared with the same chunk of the base
 * allocation with the same id, size and kind; every chunk of an allocation
 * without such a match is DIRTY.  ckpt_image_merge folds such an increment
 * into its base, and ckpt_restore does so by itself.
 * CKPT_E_BUDGET if the dense image exceeds the staging budget.
 */
int ckpt_checkpoint(ckpt_ctx *ctx, void *stream, int mode, const ckpt_image *base,
                    ckpt_image **out);

/*
 * For callers that cannot allocate memory during the call (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * device pass of ckpt_checkpoint -- size scan, chunk map and the fused pack +
 * CRC-32C + flags kernel (CKPT_FULL) or the hash-only kernel
 * (CKPT_INCREMENTAL) -- over the context's live registrations, written into
 * buffers the caller passes.  It calls no hipMalloc, hipFree or other
 * allocating routine: its descriptor tables live in one device array that the
 * library holds per device until the process ends (36 MiB: at most
 * 65536 allocations and 2^23 chunks; more is CKPT_E_BUDGET).  The results are
 * those of ckpt_checkpoint with CKPT_NO_DRAIN | CKPT_KEEP_DENSE: the dense
 * image (CKPT_SEC_DENSE's layout and contents) and the CRC and flag
 * arrays, here in device memory.  There is no serialized DATA, no dirty-id
 * list and no image object.
 *
 * base_crc: NULL (every chunk DIRTY; CKPT_FULL only), or a device array of N
 *   CRCs of a checkpoint of the same allocation table (the same sizes in the
 *   same order, e.g. the crc output of an earlier call); chunk g is DIRTY
 *   when its CRC differs from base_crc[g].  The library cannot check that the
 *   table is the same; a base of another table gives meaningless DIRTY flags.
 * dense: device, 16-byte aligned, dense_bytes >= data_bytes (CKPT_FULL; may
 *   be NULL for CKPT_INCREMENTAL, which writes no image).
 * crc, flags: device arrays of chunk_cap >= N entries (uint32 and uint8);
 *   crc 4-byte aligned.
 * n_chunks, data_bytes (host, may be NULL): receive N = sum of ceil(size / C)
 *   and sum of roundup16(size) on success and also on CKPT_E_MISMATCH, so a
 *   call with zero capacities asks for the sizes.
 * Ordering follows ckpt_checkpoint (device-wide drain first, or the stream's
 *   order with CKPT_STREAM_ORDERED).  The call returns once the work is
 *   enqueued on `stream`; the outputs are complete when the stream reaches
 *   that point.
 * Every call on one device uses that device's one array: calls whose work
 *   overlaps on one device race (the caller orders them, e.g. on one stream).
 * CKPT_E_INVAL: bad mode, CKPT_INCREMENTAL without base_crc, NULL or
 *   misaligned outputs.  CKPT_E_MISMATCH: outputs smaller than the pass
 *   needs.  CKPT_E_BUDGET: more allocations or chunks than the array holds.
 */
int ckpt_checkpoint_noalloc(ckpt_ctx *ctx, void *stream, int mode, const uint32_t *base_crc,
                            void *dense, uint64_t dense_bytes, uint32_t *crc, uint8_t *flags,
                            uint64_t chunk_cap, uint64_t *n_chunks, uint64_t *data_bytes);

/*
 * Refill n_dst destination buffers from an image, and optionally overlay an
 * incremental image (delta) on top.  dst[k] receives allocation k (id order)
 * and must be 16-byte aligned device memory of exactly the allocation's size.
 * dst_bytes[k] gives each destination's size, which must equal the
 * allocation's; dst_bytes NULL declares that every destination has exactly
 * its allocation's size (a raw device pointer's extent cannot be learned in
 * general -- a tensor may be carved out of a larger block -- so the caller's
 * word is taken).  Every chunk is written (ZERO chunks as zeros) and its CRC
 * recomputed on the device and compared with the stored one; a chunk that
 * fails is still written.  The delta's chunks are applied after the base's,
 * each verified against the delta's CRC.  Runs on `stream` and returns when
 * the destination memory is written.
 *
 * When the delta's allocation table differs from img's, the two are merged
 * first (ckpt_image_merge) and dst follows the delta's table.
 *
 * CKPT_E_MISMATCH: n_dst differs from the image's allocation count, a
 *   dst_bytes entry differs from its allocation's size (larger or smaller),
 *   or the delta's chunk size or base serial does not match img.
 * CKPT_E_INVAL: image without host DATA, misaligned dst.
 * CKPT_E_CORRUPT: some chunk failed; rep (if given) holds the number of
 *   distinct failing chunk ids and the smallest 64, ascending.
 */
int ckpt_restore(ckpt_ctx *ctx, void *stream, const ckpt_image *img, const ckpt_image *delta,
                 void *const *dst, const size_t *dst_bytes, size_t n_dst,
                 ckpt_verify_report *rep);

/* ------------------------------------------------ address-stable memory
 *
 * On restart every allocation has to come back at the device address the
 * application knew, because the application's own data holds those pointers
 * (Sec. 3.1 and Sec. 3.2, "restoring the CUDA library-allocated regions").
 * The paper gets the addresses back by replaying the logged allocation calls
 * in order against a deterministic allocator with address randomization off,
 * and names address virtualization, or a fixed-address allocation flag like
 * mmap's, as the way to drop that dependence.  HIP's virtual memory management
 * is such a mechanism: a virtual range is reserved at a requested address and
 * physical device memory is mapped into it.  These calls use it.
 *
 * Memory made by ckpt_vmm_alloc or ckpt_restore_at belongs to the context
 * (unlike memory the caller registers): it is registered as CKPT_DEVICE, is
 * released by ckpt_vmm_free or ckpt_destroy, and ckpt_unregister refuses it.
 * The caller must have finished every use of it before releasing it.
 */

/* Granularity of address-stable ranges on the context's device (bytes). */
int ckpt_vmm_granularity(ckpt_ctx *ctx, size_t *out);

/*
 * Reserve a virtual range of `bytes` rounded up to the granularity -- at
 * `addr` if it is not NULL, else where the runtime chooses -- back it with
 * device memory, make it readable and writable on the device, and register
 * [*out, *out + bytes) as CKPT_DEVICE.
 * CKPT_E_INVAL: bytes is 0, or addr is not a multiple of the granularity.
 * CKPT_E_ADDR: the range at addr is not free.  CKPT_E_NOMEM: no device memory.
 */
int ckpt_vmm_alloc(ckpt_ctx *ctx, size_t bytes, void *addr, void **out, ckpt_id *id);

/* Unregister an allocation made by ckpt_vmm_alloc or ckpt_restore_at and
 * release its range once no registration is left in it.
 * CKPT_E_NOTFOUND: ptr is not such an allocation. */
int ckpt_vmm_free(ckpt_ctx *ctx, void *ptr);

/*
 * Restore an image at the addresses it was taken from (section
 * CKPT_SEC_ADDRS), as the restart of Sec. 3.2 does, then verify every chunk as
 * ckpt_restore does (optionally overlaying an incremental image `delta`).
 * For each allocation k, in id order:
 *   - a live registration of the context with the same start, size and kind
 *     is refilled in place (rolling back memory that still exists);
 *   - otherwise the allocation is re-created: allocations sharing a
 *     granule are grouped, each group's granule-aligned range is reserved at
 *     its original address and backed with device memory, and the allocation
 *     is registered at its original address.  Its registration id is the
 *     image's id when the context has not issued that id yet (a fresh
 *     context keeps every id, so an incremental checkpoint against `img` can
 *     follow), else the next free id.
 * addrs_out (optional, n_allocs entries) receives the addresses, which equal
 * section CKPT_SEC_ADDRS on success.
 * CKPT_E_ADDR: a range is taken (by memory outside the context, or by a live
 *   registration that overlaps without matching exactly); nothing is created.
 * CKPT_E_INVAL: the image has no addresses, or a managed allocation would have
 *   to be re-created (managed memory cannot be placed at a fixed address).
 * Other errors as ckpt_restore; on any error but CKPT_E_CORRUPT the memory
 * this call created is released again.
 */
int ckpt_restore_at(ckpt_ctx *ctx, void *stream, const ckpt_image *img, const ckpt_image *delta,
                    void **addrs_out, ckpt_verify_report *rep);

/*
 * The restart path: restore the full image in file `path` (written by
 * ckpt_image_write_file, plain or compressed, or ckpt_image_serialize) at its
 * recorded addresses.  The paper's restart re-creates every allocation before
 * copying the data back (Sec. 3.2), and so does this call: it reads the
 * file's header and tables into ordinary host memory, checks them, reserves
 * and maps every address range -- before
 * it allocates any device or pinned memory of its own, so that a fresh
 * process's runtime has placed nothing there yet -- and only then loads the
 * image and refills the allocations in place, verifying every chunk.  Call
 * it before other device allocations of the process.
 * img_out (optional) receives the loaded image (the base for incremental
 * checkpoints that follow); else it is freed.  Errors as ckpt_restore_at,
 * plus CKPT_E_NOTFOUND / CKPT_E_IO for the file.
 */
int ckpt_restore_file_at(ckpt_ctx *ctx, void *stream, const char *path, void **addrs_out,
                         ckpt_verify_report *rep, ckpt_image **img_out);

/* ------------------------------------------------- automatic registration
 *
 * The paper interposes on the cudaMalloc family, so every allocation and
 * free is logged without the application's help (Sec. 3.1, "Log-and-replay";
 * Sec. 3.2, "Issue of library-allocated memory").  ckpt_hook_malloc and
 * ckpt_hook_free are that interposition for allocators that call out to a
 * pair of C functions: their signatures are the ones PyTorch's pluggable
 * allocator (torch.cuda.memory.CUDAPluggableAllocator) calls, and a caller's
 * own hipMalloc wrapper can call them too.  Each allocation on the installed
 * context's device is registered there (CKPT_DEVICE) when it is made and
 * unregistered when it is freed, so the context's live set is the active
 * allocations, in allocation order.
 *
 * One context at a time is installed, process-wide.  While a context is
 * installed, its calls and the hook functions are serialized by one lock, so
 * a checkpoint sees no half-made allocation; allocations from other threads
 * wait while it runs.  ckpt_destroy of the installed context uninstalls it;
 * memory made through the hook stays valid (address-stable memory aside,
 * which the context owns and releases).
 */
#define CKPT_HOOK_ADDRESS_STABLE 0x1u   /* allocate with ckpt_vmm_alloc, so that
                                           ckpt_restore_at can bring every
                                           allocation back at its address      */
#define CKPT_HOOK_CACHE 0x2u            /* keep freed blocks for reuse (below)   */

/* Install ctx (NULL: none) as the context the hook logs into.  Resets the
 * hook counters and releases the blocks cached for the previous context.
 * CKPT_E_INVAL: unknown flags. */
int ckpt_hook_install(ckpt_ctx *ctx, uint32_t flags);

/* Allocate `bytes` on `device` (hipMalloc, or an address-stable mapping of
 * the context with CKPT_HOOK_ADDRESS_STABLE) and register exactly `bytes`
 * there when `device` is the installed context's; other devices get plain
 * unregistered hipMalloc memory.  NULL on failure or for 0 bytes.
 *
 * Without CKPT_HOOK_CACHE `stream` is not used and the memory is usable on
 * any stream.  With it, blocks come in size classes (four per power of two,
 * at least 512 bytes; address-stable ones are granularity multiples), and a
 * freed block is kept, unregistered, for the next allocation of its class on
 * the stream it was first allocated for: that allocation follows, in stream
 * order, all work queued on that stream before the free.  As with any
 * stream-ordered caching allocator, a caller that used the memory on other
 * streams synchronizes them before freeing.  When the device runs out of
 * memory the cached blocks are released and the allocation tried again, and
 * then, if it still fails, a block of the request's own size (rounded to 2
 * MiB or the granularity) is tried; such a block is released when freed. */
void *ckpt_hook_malloc(size_t bytes, int device, void *stream);

/* Unregister memory from ckpt_hook_malloc and free it: without
 * CKPT_HOOK_CACHE after the device's queued work is done; with it into the
 * cache, at once.  bytes and stream are not used. */
void ckpt_hook_free(void *ptr, size_t bytes, int device, void *stream);

/* Registered allocations and frees since ckpt_hook_install, and allocations
 * that failed. */
int ckpt_hook_stats(uint64_t *allocs, uint64_t *frees, uint64_t *failures);

/* Blocks and bytes the cache holds now, and allocations it served since
 * ckpt_hook_install. */
int ckpt_hook_cache_stats(uint64_t *blocks, uint64_t *bytes, uint64_t *hits);

/* Release every cached block (after the device's queued work is done);
 * *released (may be NULL) = their bytes.  ckpt_restore_at and
 * ckpt_restore_file_at of the installed context do this first, so that the
 * recorded addresses are free. */
int ckpt_hook_trim(uint64_t *released);

/* ----------------------------------------------------------------- image */

/*
 * Fold an incremental image into the full image it was taken against: the
 * result is the full image (every chunk DIRTY, no base) that a checkpoint at
 * the increment's time would have given -- the increment's allocation table,
 * CRC, flags and addresses, each non-ZERO chunk's bytes from the increment
 * when DIRTY there, else from the same chunk of the base allocation with the
 * same id, size and kind.  The result carries the increment's serial (it
 * stands for the same state), so a chain base <- d1 <- d2 folds as
 * merge(merge(base, d1), d2).  Runs on the host; both images need host DATA.
 * CKPT_E_INVAL: base not full, delta not incremental, or no host DATA.
 * CKPT_E_MISMATCH: delta was not taken against base (serial, chunk size).
 * CKPT_E_CORRUPT: the delta marks a chunk clean that has no equal base chunk,
 *   or its DATA size disagrees with its flags.
 */
int ckpt_image_merge(const ckpt_image *base, const ckpt_image *delta, ckpt_image **out);

/*
 * Write the image's serialized form (the bytes ckpt_image_serialize gives) to
 * the file `path`, so that it reaches durable storage as the paper's
 * checkpoints do (DMTCP writes each process's image to a file).  The bytes go
 * out in 64 MiB blocks, staged through aligned buffers while the previous
 * block is written, with O_DIRECT unless CKPT_FILE_BUFFERED is given or the
 * file system refuses it; then fsync.  The file is written as path.partial
 * and renamed to path once complete, so path never holds a partial image.
 * *bytes (optional) receives the file size.  CKPT_E_IO on a failing file
 * operation (the partial file is removed); CKPT_E_INVAL for an image without
 * host DATA.
 */
#define CKPT_FILE_BUFFERED 0x1u   /* write through the page cache */
/* Write a compressed container instead (always through the page cache):
 * DATA in 4 MiB blocks, compressed by a pool of threads (up to 16), each
 * block either deflated at zlib's fastest level or split into byte planes of
 * 2- or 4-byte elements and Huffman-coded, whichever codes its first 64 KiB
 * smallest, and stored raw when that or the whole block does not shrink;
 * header and tables stay uncompressed.  Layout in sink.cpp.  The paper's checkpointer compresses its images with gzip by
 * default (Sec. 4.4, where it is turned off for the timings). */
#define CKPT_FILE_DEFLATE 0x2u
int ckpt_image_write_file(const ckpt_image *img, const char *path, uint32_t flags, uint64_t *bytes);

/* Read an image file written by ckpt_image_write_file (plain or compressed)
 * or any serialized image, and load it as ckpt_image_load does: header and
 * tables first, then DATA by several threads straight into the image's pinned
 * buffer (compressed blocks inflated there).  CKPT_E_NOTFOUND if the file
 * cannot be opened, CKPT_E_IO if it cannot be read, CKPT_E_INVAL for a
 * truncated or inconsistent file (a block that does not inflate to its size
 * included), and ckpt_image_load's errors for its contents. */
int ckpt_image_read_file(ckpt_ctx *ctx, const char *path, ckpt_image **out);

/* The metadata of the image in file `path` (plain or compressed) from its
 * header and tables alone, host memory only: e.g. n_allocs, to size the
 * address array of ckpt_restore_file_at.  has_dense is 0 and drained 1.
 * Errors as ckpt_image_read_file (the CRC section's digest is checked). */
int ckpt_image_file_info(const char *path, ckpt_image_meta *out);

int ckpt_image_info(const ckpt_image *img, ckpt_image_meta *out);

/* Pointer and length of one section (ckpt_section).  Host sections point into
 * the image's own buffers; CKPT_SEC_DENSE is a device pointer.  A section that
 * is absent gives *p = NULL, *bytes = 0 and CKPT_OK. */
int ckpt_image_view(const ckpt_image *img, int section, const void **p, size_t *bytes);

/* Serialize into buf (header + ALLOCS + CRC + FLAGS + DIRTY_IDS + DATA, all
 * little-endian).  *need gets the required size; with cap < need nothing is
 * written and CKPT_E_INVAL is returned (buf may be NULL to query). */
int ckpt_image_serialize(const ckpt_image *img, void *buf, size_t cap, size_t *need);

/* Parse a buffer written by ckpt_image_serialize into a new image (host
 * sections only).  CKPT_E_INVAL: bad magic/version, truncated, inconsistent
 * sizes. */
int ckpt_image_load(ckpt_ctx *ctx, const void *buf, size_t bytes, ckpt_image **out);

void ckpt_image_free(ckpt_image *img);

/* --------------------------------------------------------------- batched */

/*
 * Checkpoint (CKPT_FULL) several contexts in one pass: every context's
 * registrations are laid out in one table and packed by one persistent
 * kernel launch, replayed from a captured hipGraph (table upload from pinned
 * memory, size scan, chunk map, pack, and, unless ctxs[0] has CKPT_NO_DRAIN,
 * the drain: the select and a gather that stores each context's non-ZERO
 * chunks straight into that image's pinned host buffer; captured again only
 * when the table or the number of contexts outgrows the capacities of the
 * last capture).  The host buffers are taken before the replay with room for
 * each context's dense bytes.  With CKPT_NO_GRAPH (ctxs[0]) the kernels are
 * launched one by one and the drain goes through device staging in segments
 * and the runtime's copies.  outs[i] is the image of
 * ctxs[i], identical to what ckpt_checkpoint(ctxs[i], stream, CKPT_FULL,
 * NULL, ...) produces.  All contexts must be on one device with one chunk
 * size (else CKPT_E_INVAL); ctxs[0] provides the launch configuration,
 * staging and streams, and may not use CKPT_KEEP_DENSE or CKPT_DRAIN_DIRECT.
 * With CKPT_NO_DRAIN each image's DENSE view points into ctxs[0]'s staging.
 */
int ckpt_checkpoint_batch(ckpt_ctx *const *ctxs, size_t n, void *stream, ckpt_image **outs);

/* ---------------------------------------------------------------- serving */

/*
 * A server takes checkpoint and restore requests as they arrive and runs them
 * with continuous batching on one GPU.  Each request is a set of allocations
 * like a context's live set (checkpoint) or a set of destination buffers
 * (restore, like ckpt_restore without a delta).  Requests are admitted in
 * arrival order while fewer than max_active are admitted and the request's
 * device staging fits in what is left of staging_budget (checkpoint: dense
 * image + drain buffer + per-chunk arrays, about 2x its bytes; restore: the
 * serialized bytes + per-chunk arrays).  A checkpoint also needs pinned host
 * memory for its image: it is admitted only while the pinned bytes the library
 * has handed out (to images anywhere in the process, the caller's included),
 * plus the most that the admitted checkpoints' images can take, plus its own
 * stay within host_budget.  A checkpoint waiting for host memory lets the
 * restores behind it pass (they need none, and finishing them is what lets a
 * caller release older images); requests behind a request whose device
 * staging does not fit wait.  So a backlog queues instead of failing, and
 * images the caller keeps hold back later checkpoints until it frees them.
 * Finished checkpoints' images count too before the caller claims them: a
 * caller that waits for one held-back checkpoint while later results stay
 * unclaimed should claim results as they finish (ckpt_server_poll).  A
 * checkpoint held back for host memory for 30 s fails with CKPT_E_NOMEM.
 * The host may pin less than host_budget: a request whose preparation or
 * finish (a finished checkpoint's image included) cannot get memory keeps its
 * staging and runs that part again every few milliseconds until memory is
 * released (after 30 s it fails with CKPT_E_NOMEM); a short image buffer also
 * makes the server take the pinned bytes held at that moment as its host
 * budget.  A step whose buffers cannot grow is run again the same way.
 * Every step is one kernel launch that
 * processes up to step_bytes of each admitted request, checkpoints and
 * restores together, so requests overlap on the device; a request that
 * arrives during a step joins the next one.  Results are the same as a
 * request run alone (ckpt_checkpoint of the same allocations with CKPT_FULL
 * and no base, ids 1..n; ckpt_restore).
 * The caller keeps source/destination memory, and a restore's image, valid
 * and unmodified until the request completes.  All ckpt_server_* calls are
 * thread-safe.
 */
enum ckpt_req_op { CKPT_REQ_CHECKPOINT = 0, CKPT_REQ_RESTORE = 1 };

typedef struct ckpt_server_config {
    int32_t device;            /* HIP device ordinal                                    */
    uint32_t chunk_bytes;      /* C; 0 selects 4096                                     */
    uint64_t staging_budget;   /* device bytes for admitted requests, reserved at create;
                                  0 selects 64 GiB                                      */
    uint64_t step_bytes;       /* bytes of each admitted request per step;
                                  0 selects 256 MiB                                     */
    uint32_t max_active;       /* requests admitted at once; 0 selects 16               */
    uint32_t aux_threads;      /* workers that prepare and finish requests; 0 selects 2 */
    uint32_t block_threads;    /* 0 selects 1024                                        */
    uint32_t lane_pieces;      /* as in ckpt_config: 1 (0 selects 1)                    */
    uint64_t host_budget;      /* pinned host bytes for images (see above); 0 selects
                                  64 GiB                                                */
} ckpt_server_config;

typedef struct ckpt_request {
    uint32_t op;                /* ckpt_req_op                                          */
    uint32_t n;                 /* allocations                                          */
    void *const *ptrs;          /* checkpoint: sources; restore: destinations (device,
                                   16-byte aligned); the server copies the array       */
    const uint64_t *sizes;      /* bytes of each; restore: must equal the image's sizes */
    const uint32_t *kinds;      /* ckpt_kind of each; NULL = all CKPT_DEVICE             */
    const ckpt_image *image;    /* restore: a drained full image with n allocations     */
} ckpt_request;

typedef struct ckpt_result {
    int32_t status;             /* CKPT_OK, CKPT_E_CORRUPT (restore) or an error        */
    uint32_t op;
    ckpt_image *image;          /* checkpoint: the new image, now owned by the caller   */
    double latency_ms;          /* submit to completion: checkpoint = serialized image in
                                   pinned host memory; restore = destinations written
                                   and verified                                         */
    double queue_ms;            /* submit to admission                                  */
    uint64_t bytes;             /* algorithmic bytes: checkpoint live + dense; restore
                                   live + serialized                                    */
    uint64_t n_bad;             /* restore: chunks that failed verification             */
} ckpt_result;

typedef struct ckpt_stats {
    uint64_t submitted, completed, failed;
    uint64_t bytes;             /* live bytes of completed requests                     */
    double p50_ms, p99_ms;      /* latency percentiles (nearest rank) of completed requests */
    double mean_ms, max_ms;
    double makespan_s;          /* first submit to last completion                      */
    double gbps;                /* bytes / makespan, 1e9 B/s                            */
    uint64_t steps;             /* step launches                                        */
    uint32_t max_concurrent;    /* most requests admitted at once                       */
    uint32_t pad;
    uint64_t host_waits;        /* checkpoints held back for host memory at admission,
                                   and requests whose step waited for memory           */
    uint64_t host_peak;         /* most pinned bytes held plus reserved at an admission */
    char last_error[160];       /* message of the latest failed request ("" if none)   */
} ckpt_stats;

/* CKPT_E_INVAL: bad config; CKPT_E_NOMEM: the staging budget could not be
 * reserved. */
int ckpt_server_create(const ckpt_server_config *cfg, ckpt_server **out);

/* Queue a request; *ticket identifies it.  CKPT_E_INVAL / CKPT_E_MISMATCH on
 * a malformed request (checked here), CKPT_E_BUDGET if it can never fit the
 * staging budget or (checkpoint) the host budget. */
int ckpt_server_submit(ckpt_server *srv, const ckpt_request *req, uint64_t *ticket);

/* CKPT_E_AGAIN until the request is done; then fills *out (out may be NULL to
 * discard, which frees a checkpoint's image) and retires the ticket.
 * CKPT_E_NOTFOUND for an unknown or retired ticket. */
int ckpt_server_poll(ckpt_server *srv, uint64_t ticket, ckpt_result *out);

/* As ckpt_server_poll, but blocks until the request is done. */
int ckpt_server_wait(ckpt_server *srv, uint64_t ticket, ckpt_result *out);

int ckpt_server_stats(const ckpt_server *srv, ckpt_stats *out);
int ckpt_server_reset_stats(ckpt_server *srv);

/* Waits for admitted requests to finish, cancels queued ones, frees the
 * server and the results nobody retrieved.  NULL is a no-op. */
void ckpt_server_destroy(ckpt_server *srv);

/* --------------------------------------------------------------- timing */

int ckpt_last_timing(const ckpt_ctx *ctx, ckpt_timing *out);

/* Pinned host memory of the process-wide pool the library draws images' host
 * sections and its staging from: *live (may be NULL) = bytes handed out and
 * not yet returned (images the caller holds included), *cached (may be NULL)
 * = freed buffers kept for reuse (at most 32 GiB, given back first when a
 * pinned allocation fails).  A server's host budget counts the live bytes.
 * Host memory only; no device is touched. */
int ckpt_host_memory(uint64_t *live, uint64_t *cached);

/* ------------------------------------------------------------ diagnostics */

const char *ckpt_strerror(int status);
int ckpt_last_hip_error(void);          /* hipError_t of the last failing HIP call */
const char *ckpt_last_error(void);      /* text for the last error on this thread  */

#ifdef __cplusplus
}
#endif

#endif /* CKPT_H */
