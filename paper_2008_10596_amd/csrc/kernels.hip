// kernels.hip -- gfx950 kernels of libckpt: size scan, chunk map, fused
// pack + CRC-32C + ZERO/DIRTY flags (and its hash-only and restore/verify
// variants), selection scan, gather, and small helpers.
//
// The data path drains the memory of live allocations into an image and
// refills it (CRAC, Sec. 3.2 "Saving the library-allocated arena" and
// "restoring the CUDA library-allocated regions").  It is pure bandwidth
// work: no MFMA.  The CRC-32C per chunk is the library's own check.
//
// CRC scheme (one wave64 per chunk, or `waves_per_chunk` waves):
//   * The chunk's bytes are read in rounds of 1 KiB: in round r, lane l loads
//     the 16-byte piece r*64 + l (each load instruction covers 1 KiB of whole
//     cache lines).
//   * A chunk of len bytes is placed at the END of a window of whole rounds
//     (leading zero pieces, and zeros after len up to the next 16 bytes).
//     Leading zeros leave a zero CRC register unchanged, so the window's raw
//     CRC (zero init, no final XOR) equals that of the data followed by its
//     s = roundup16(len) - len zero pad bytes; the pad is undone at the end by
//     running the register backwards s bytes.
//   * Each lane hashes each round's piece from a zero register (two 2-byte
//     table steps per 4-byte word) and combines the rounds by Horner's rule
//     with the one-round operator (1024 - 16 bytes to the lane's next piece).
//   * A 6-level tree across lanes combines the registers: at level k the left
//     partner is moved forward 16 << k bytes and XORed with the right one;
//     only the lanes whose result is still needed do the table lookups.
//   * With several waves per chunk, each wave owns consecutive rounds and the
//     per-wave results are combined by one more operator.
//   * CRC-32C's initial value 0xFFFFFFFF is folded in by complementing the
//     first min(len, 4) data bytes before hashing (and, for len < 4, XORing
//     the part of the initial value that is still in the register), and the
//     final XOR is applied last.
//   Every "move forward m bytes" is a GF(2)-linear operator stored in LDS as
//   byte-indexed tables (crc_tables.cpp), the chain and round operators
//   replicated per lane so that the random lookups are bank-conflict free.
#include "internal.h"

namespace ckpt {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t apply_op(const uint32_t *__restrict__ t, uint32_t v)
{
    return t[v & 0xffu] ^ t[256 + ((v >> 8) & 0xffu)] ^ t[512 + ((v >> 16) & 0xffu)] ^
           t[768 + (v >> 24)];
}

// The operator tables as staged in LDS (124 KiB): per-lane copies of the
// chain and round operators, single copies of the tree and cross-wave ones.
struct Tabs {
    const uint32_t *t;   // LDS base
    uint32_t lb;         // (lane & 31) << 2, this lane's chain copy
    uint32_t lb8;        // (lane & 7) << 2, this lane's round-operator copy

    __device__ __forceinline__ uint32_t lds(uint32_t byte_off) const
    {
        return *(const uint32_t *)((const uint8_t *)t + byte_off);
    }
    // register after the 4-byte word w: two 2-byte steps
    __device__ __forceinline__ uint32_t chain(uint32_t s, uint32_t w) const
    {
        uint32_t y = s ^ w;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const uint32_t a0 = __builtin_amdgcn_perm(y, lb, 0x0c0c0400u);   // (y.byte0 << 8) | lb
            const uint32_t a1 = (y & 0xff00u) | lb;
            y = lds(kRepChainOff + a0) ^ lds(kRepChainOff + 128 + a1) ^ (y >> 16);
        }
        return y;
    }
    // the register moved one round (or, in the quad form's set, the skip) forward
    __device__ __forceinline__ uint32_t gap(uint32_t v) const
    {
        return lds(((v & 0xffu) << 5) | lb8) ^ lds(8192 + ((((v >> 8) & 0xffu) << 5) | lb8)) ^
               lds(16384 + ((((v >> 16) & 0xffu) << 5) | lb8)) ^ lds(24576 + (((v >> 24) << 5) | lb8));
    }
    __device__ __forceinline__ uint32_t tree(int k, uint32_t v) const
    {
        return apply_op(t + kRepTreeOff / 4 + k * kTabWords, v);
    }
    __device__ __forceinline__ uint32_t seg(uint32_t v) const
    {
        return apply_op(t + kRepTreeOff / 4 + kTreeLevels * kTabWords, v);
    }
};

__device__ __forceinline__ Tabs make_tabs(const uint32_t *lds_tabs, int lane)
{
    Tabs T;
    T.t = lds_tabs;
    T.lb = (uint32_t)(lane & 31) << 2;
    T.lb8 = (uint32_t)(lane & 7) << 2;
    return T;
}

__device__ __forceinline__ uint64_t round_up16(uint64_t x) { return (x + 15) & ~uint64_t(15); }

// Wave64 inclusive scan of a u64 (Hillis-Steele with shuffles).
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Bytes [0, valid) of a 16-byte piece, zeros after; never reads past valid.
__device__ __forceinline__ uint4 load_partial(const uint8_t *p, uint32_t valid)
{
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 16; i++)
        if ((uint32_t)i < valid)
            w[i >> 2] |= (uint32_t)p[i] << (8 * (i & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Writes bytes [0, valid) of a 16-byte piece only.
__device__ __forceinline__ void store_partial(uint8_t *p, uint32_t valid, uint4 v)
{
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 16; i++)
        if ((uint32_t)i < valid)
            p[i] = (uint8_t)(w[i >> 2] >> (8 * (i & 3)));
}

// Undo `s` zero pad bytes: the register one zero bit earlier is recovered
// from its top bit (set exactly when the polynomial was XORed in).
__device__ __forceinline__ uint32_t unshift_bytes(uint32_t reg, uint32_t s)
{
    for (uint32_t i = 0; i < 8 * s; i++)
        reg = (reg & 0x80000000u) ? (((reg ^ kPolyReflected) << 1) | 1u) : (reg << 1);
    return reg;
}

// Mask that complements the first min(n, 4) bytes of the first data word.
__device__ __forceinline__ uint32_t init_mask(uint32_t n)
{
    return n >= 4 ? 0xFFFFFFFFu : ((1u << (8 * n)) - 1u);
}

// CRC-32C from the window's raw register.
__device__ __forceinline__ uint32_t finish_crc(uint32_t raw, uint32_t n)
{
    uint32_t reg = unshift_bytes(raw, (uint32_t)round_up16(n) - n);
    if (n < 4)
        reg ^= 0xFFFFFFFFu >> (8 * n);
    return ~reg;
}

// ---------------------------------------------------------- K1: size scan
//
// off[k] = exclusive prefix sum of roundup16(size), cb[k] = exclusive prefix
// sum of ceil(size / C); off[n] and cb[n] get the totals, copied to the plan.
// One workgroup of 1024 threads walks the table in tiles of 1024.

// With `up` (the table in pinned host memory: a plan header, then n
// addresses, then n sizes), the kernel also copies it to the device: the
// header to `plan`, the addresses and sizes to `addr_out` and `size`, with no
// separate copies before it.  Without `up`, it reads `plan` and `size`.
template <bool FROM_HOST>
__global__ __launch_bounds__(1024) void k_layout_scan(DevPlan *plan, uint64_t *__restrict__ size,
                                                      uint32_t C, uint64_t *__restrict__ off,
                                                      uint64_t *__restrict__ cb, const uint8_t *up,
                                                      uint64_t *__restrict__ addr_out)
{
    __shared__ uint64_t s_off[16], s_cb[16];
    const DevPlan *hp = (const DevPlan *)up;
    const uint64_t n = FROM_HOST ? hp->n_allocs : plan->n_allocs;
    const uint64_t *h_addr = FROM_HOST ? (const uint64_t *)(up + sizeof(DevPlan)) : nullptr;
    const uint64_t *h_size = FROM_HOST ? h_addr + n : nullptr;
    if (FROM_HOST && threadIdx.x == 0)
        *plan = *hp;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t carry_off = 0, carry_cb = 0;
    for (uint64_t base = 0; base < n; base += 1024) {
        const uint64_t k = base + threadIdx.x;
        uint64_t sz = 0;
        if (k < n) {
            if (FROM_HOST) {
                sz = h_size[k];
                size[k] = sz;
                addr_out[k] = h_addr[k];
            } else {
                sz = size[k];
            }
        }
        const uint64_t e = round_up16(sz), c = (sz + C - 1) / C;
        const uint64_t ie = wave_incl_scan(e, lane), ic = wave_incl_scan(c, lane);
        if (lane == 63) {
            s_off[wave] = ie;
            s_cb[wave] = ic;
        }
        __syncthreads();
        uint64_t pre_off = carry_off, pre_cb = carry_cb, tot_off = 0, tot_cb = 0;
        for (int w = 0; w < 16; w++) {
            if (w < wave) {
                pre_off += s_off[w];
                pre_cb += s_cb[w];
            }
            tot_off += s_off[w];
            tot_cb += s_cb[w];
        }
        if (k < n) {
            off[k] = pre_off + ie - e;
            cb[k] = pre_cb + ic - c;
        }
        carry_off += tot_off;
        carry_cb += tot_cb;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        off[n] = carry_off;
        cb[n] = carry_cb;
        plan->data_bytes = carry_off;
        plan->n_chunks = carry_cb;
    }
}

// ------------------------------------------------------- chunk -> row map
//
// map[g] = k for every chunk g of allocation k: the descriptor table each
// workgroup of the chunk kernels stages into LDS, one load per chunk instead
// of a binary search.

__global__ void k_chunk_map(const DevPlan *plan, const uint64_t *__restrict__ cb, uint32_t *__restrict__ map)
{
    const uint64_t n = plan->n_allocs;
    const int lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t k = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); k < n; k += waves) {
        const uint64_t b = cb[k], e = cb[k + 1];
        for (uint64_t g = b + lane; g < e; g += 64)
            map[g] = (uint32_t)k;
    }
}

// -------------------------------------------- K3/K4/K8: the chunk kernels
//
// Persistent workgroups take tiles of kTile chunk items from a counter; each tile's
// descriptors are staged in LDS once, then groups of waves_per_chunk waves
// take one item each.
//   kModePack:    read the allocation, write the dense image, CRC + flags.
//   kModeHash:    read the allocation, CRC + flags (incremental checkpoints).
//   kModeRestore: read the serialized chunk from staging (or zeros for a
//                 ZERO chunk), write the destination (exactly len bytes),
//                 recompute the CRC and compare with the stored one.

constexpr int kTile = 64;

struct Desc {
    uint64_t src;   // pack/hash: source address; restore: staging address (0 for ZERO)
    uint64_t dst;   // pack: dense address; restore: destination address
    uint64_t g;     // chunk id
    uint32_t len;   // bytes in the chunk
    uint32_t zero;  // restore: the chunk is ZERO
    uint32_t want;  // the CRC to compare with (base for DIRTY, stored for restore),
                    // loaded with the descriptor so no wave waits on it at the end
    uint32_t has_base;  // pack/hash: a base chunk exists and want is its CRC
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ uint4 ld16(const void *p)
{
    if (NT) {
        const u32x4 t = __builtin_nontemporal_load((const u32x4 *)p);
        return make_uint4(t.x, t.y, t.z, t.w);
    }
    return *(const uint4 *)p;
}

template <bool NT>
__device__ __forceinline__ void st16(void *p, uint4 v)
{
    if (NT) {
        const u32x4 t = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(t, (u32x4 *)p);
    } else {
        *(uint4 *)p = v;
    }
}

template <int MODE, bool NT>
__device__ __forceinline__ uint4 load_piece(const Desc &d, uint32_t start)
{
    if (MODE == kModeRestore) {
        if (d.zero)
            return make_uint4(0u, 0u, 0u, 0u);
        return ld16<NT>((const uint8_t *)d.src + start);   // staging pieces are padded to 16
    }
    const uint8_t *p = (const uint8_t *)d.src + start;
    if (start + 16 <= d.len)
        return ld16<NT>(p);
    return load_partial(p, d.len - start);
}

template <int MODE, bool NT>
__device__ __forceinline__ void store_piece(const Desc &d, uint32_t start, uint4 v)
{
    if (MODE == kModePack) {
        st16<NT>((uint8_t *)d.dst + start, v);            // dense image keeps the zero pad
    } else if (MODE == kModeRestore) {
        uint8_t *p = (uint8_t *)d.dst + start;
        if (start + 16 <= d.len)
            st16<NT>(p, v);
        else
            store_partial(p, d.len - start, v);
    }
}

// 16-byte loads each lane keeps in flight before hashing them.
constexpr int kLoadsInFlight = 4;

// The register of the lane K places down (lane + K), for K < 16: a DPP row
// shift, with no LDS round trip.  Lanes whose source is outside their row of
// 16 get 0; the combine below reads only lanes whose source is inside.
template <int K>
__device__ __forceinline__ uint32_t dpp_down(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x100 + K, 0xF, 0xF, true);
}

// Combine the 64 lanes' registers into lane 0: at level k, lane i (a multiple
// of 2^(k+1)) moves its register past the 16 * 2^k bytes of lane i + 2^k's
// share and adds that lane's register.  Levels 0-3 stay inside rows of 16
// lanes (DPP); levels 4 and 5 cross rows (__shfl_down).  The whole wave must
// be active.
static_assert(kTreeLevels == 6, "the combine is written out for 64 lanes");

__device__ __forceinline__ uint32_t wave_combine(const Tabs &T, uint32_t acc, int lane)
{
    uint32_t right = dpp_down<1>(acc);
    if ((lane & 1) == 0)
        acc = T.tree(0, acc) ^ right;
    right = dpp_down<2>(acc);
    if ((lane & 3) == 0)
        acc = T.tree(1, acc) ^ right;
    right = dpp_down<4>(acc);
    if ((lane & 7) == 0)
        acc = T.tree(2, acc) ^ right;
    right = dpp_down<8>(acc);
    if ((lane & 15) == 0)
        acc = T.tree(3, acc) ^ right;
    right = __shfl_down(acc, 16, 64);
    if ((lane & 31) == 0)
        acc = T.tree(4, acc) ^ right;
    right = __shfl_down(acc, 32, 64);
    if (lane == 0)
        acc = T.tree(5, acc) ^ right;
    return acc;
}

// The lane's register after one 16-byte piece, chained from register c.
__device__ __forceinline__ uint32_t chain_piece(const Tabs &T, uint32_t c, const uint4 &v)
{
    c = T.chain(c, v.x);
    c = T.chain(c, v.y);
    c = T.chain(c, v.z);
    return T.chain(c, v.w);
}

constexpr int kPerRound = 64;   // 16-byte pieces per round (one per lane)

// One wave's share of a chunk: rounds [r_begin, r_end) of a window of r_win
// rounds of 1 KiB.  Returns the raw register of those rounds in lane 0 (as a
// message ending with the wave's last round) and ORs the data words into
// *orv.
template <int MODE, bool NT>
__device__ __forceinline__ uint32_t wave_rounds(const Tabs &T, const Desc &d, int lane, uint32_t r_begin,
                                                uint32_t r_end, uint32_t r_win, uint32_t *orv)
{
    constexpr int B = kLoadsInFlight;                                     // rounds per batch
    const uint32_t np = (d.len + 15) >> 4;                                // data pieces
    const uint32_t z = r_win * kPerRound - np;                            // leading zero pieces
    if (d.len == r_win * kPerRound * 16 && (MODE != kModeRestore || !d.zero)) {
        // The chunk fills the window exactly (uniform over the wave): every
        // piece is 16 bytes of data at offset (r * 64 + lane) * 16 and only
        // piece 0 carries the complemented init.
        uint32_t acc = 0, o = 0;
        for (uint32_t rb = r_begin; rb < r_end; rb += B) {
            uint4 v[B];
#pragma unroll
            for (int b = 0; b < B; b++)
                v[b] = rb + b < r_end ? ld16<NT>((const uint8_t *)d.src + ((rb + b) * kPerRound + lane) * 16)
                                      : make_uint4(0u, 0u, 0u, 0u);
            uint32_t c[B];
#pragma unroll
            for (int b = 0; b < B; b++) {
                const uint32_t r = rb + b;
                if (MODE != kModeHash && r < r_end)
                    st16<NT>((uint8_t *)d.dst + (r * kPerRound + lane) * 16, v[b]);
                o |= v[b].x | v[b].y | v[b].z | v[b].w;
                if (r == 0 && lane == 0)
                    v[b].x = ~v[b].x;
                c[b] = chain_piece(T, 0u, v[b]);
            }
#pragma unroll
            for (int b = 0; b < B; b++) {
                const uint32_t r = rb + b;
                if (r < r_end)
                    acc = (r > r_begin ? T.gap(acc) : 0u) ^ c[b];
            }
        }
        acc = wave_combine(T, acc, lane);
        *orv = o;
        return acc;
    }
    const uint32_t r0 = max(r_begin, z / kPerRound);                      // earlier rounds: all zero
    uint32_t acc = 0, o = 0;
    for (uint32_t rb = r0; rb < r_end; rb += B) {
        uint4 v[B];
#pragma unroll
        for (int b = 0; b < B; b++) {
            const int p = (int)((rb + b) * kPerRound + lane) - (int)z;
            v[b] = make_uint4(0u, 0u, 0u, 0u);
            if (rb + b < r_end && p >= 0)
                v[b] = load_piece<MODE, NT>(d, (uint32_t)p * 16);
        }
        // Each round's contribution is chained from a zero register, so the
        // rounds' lookups are independent; they are combined by Horner's rule
        // with the one-round shift.  Pieces past r_end are zero and add nothing.
        uint32_t c[B];
#pragma unroll
        for (int b = 0; b < B; b++) {
            const uint32_t r = rb + b;
            const int p = (int)(r * kPerRound + lane) - (int)z;
            if (r < r_end && p >= 0)
                store_piece<MODE, NT>(d, (uint32_t)p * 16, v[b]);
            o |= v[b].x | v[b].y | v[b].z | v[b].w;
            if (p == 0)
                v[b].x ^= init_mask(d.len);
            c[b] = chain_piece(T, 0u, v[b]);
        }
#pragma unroll
        for (int b = 0; b < B; b++) {
            const uint32_t r = rb + b;
            if (r < r_end)
                acc = (r > r0 ? T.gap(acc) : 0u) ^ c[b];
        }
    }
    acc = wave_combine(T, acc, lane);
    *orv = o;
    return acc;
}

// Chunks of at most one batch of rounds (r_win <= kLoadsInFlight, one wave
// per chunk): the same steps as wave_rounds, split into the loads and the
// rest, so that a wave can have the next chunk's loads in flight while it
// hashes, combines and finishes the current one.
template <int MODE, bool NT>
__device__ __forceinline__ void small_loads(const Desc &d, int lane, uint32_t r_win, uint4 (&v)[kLoadsInFlight])
{
    const uint32_t np = (d.len + 15) >> 4;
    const uint32_t z = r_win * kPerRound - np;
    if (d.len == r_win * kPerRound * 16 && (MODE != kModeRestore || !d.zero)) {
        // the chunk fills the window exactly (uniform over the wave): every
        // piece is 16 bytes of data
#pragma unroll
        for (int b = 0; b < kLoadsInFlight; b++)
            v[b] = (uint32_t)b < r_win ? ld16<NT>((const uint8_t *)d.src + ((uint32_t)b * kPerRound + lane) * 16)
                                       : make_uint4(0u, 0u, 0u, 0u);
        return;
    }
    const uint32_t r0 = z / kPerRound;
#pragma unroll
    for (int b = 0; b < kLoadsInFlight; b++) {
        const int p = (int)((r0 + b) * kPerRound + lane) - (int)z;
        v[b] = make_uint4(0u, 0u, 0u, 0u);
        if (r0 + b < r_win && p >= 0)
            v[b] = load_piece<MODE, NT>(d, (uint32_t)p * 16);
    }
}

// store: write the chunk's pieces (pack); a ZERO chunk's pieces are not
// stored, since the dense image leaves ZERO chunks unwritten.
template <int MODE, bool NT>
__device__ __forceinline__ uint32_t small_rest(const Tabs &T, const Desc &d, int lane, uint32_t r_win,
                                               uint4 (&v)[kLoadsInFlight], uint32_t *orv, bool store)
{
    constexpr int B = kLoadsInFlight;
    const uint32_t np = (d.len + 15) >> 4;
    const uint32_t z = r_win * kPerRound - np;
    if (d.len == r_win * kPerRound * 16) {
        // The chunk fills the window exactly (uniform over the wave): every
        // piece is 16 bytes of data, and only lane 0's first piece carries the
        // complemented init (the chunk is at least 16 bytes long).
        uint32_t acc = 0, o = 0, c[B];
#pragma unroll
        for (int b = 0; b < B; b++) {
            const uint32_t off = ((uint32_t)b * kPerRound + lane) * 16;
            if (MODE != kModeHash && store && (uint32_t)b < r_win)
                st16<NT>((uint8_t *)d.dst + off, v[b]);
            o |= v[b].x | v[b].y | v[b].z | v[b].w;
            if (b == 0 && lane == 0)
                v[b].x = ~v[b].x;
            c[b] = chain_piece(T, 0u, v[b]);
        }
#pragma unroll
        for (int b = 0; b < B; b++)
            if ((uint32_t)b < r_win)
                acc = (b > 0 ? T.gap(acc) : 0u) ^ c[b];
        acc = wave_combine(T, acc, lane);
        *orv = o;
        return acc;
    }
    const uint32_t r0 = z / kPerRound;
    uint32_t acc = 0, o = 0, c[B];
    // independent per-round chains, then Horner's rule (as in wave_rounds)
#pragma unroll
    for (int b = 0; b < B; b++) {
        const uint32_t r = r0 + b;
        const int p = (int)(r * kPerRound + lane) - (int)z;
        if (r < r_win && p >= 0 && store)
            store_piece<MODE, NT>(d, (uint32_t)p * 16, v[b]);
        o |= v[b].x | v[b].y | v[b].z | v[b].w;
        if (p == 0)
            v[b].x ^= init_mask(d.len);
        c[b] = chain_piece(T, 0u, v[b]);
    }
#pragma unroll
    for (int b = 0; b < B; b++)
        if (r0 + b < r_win)
            acc = (b > 0 ? T.gap(acc) : 0u) ^ c[b];
    acc = wave_combine(T, acc, lane);
    *orv = o;
    return acc;
}

// Restore of a full-length ZERO chunk: its bytes are zeros, so its CRC is the
// CRC of C zero bytes, known beforehand; the wave stores the zeros and the
// stored CRC is compared with that value, with no table lookups.
template <bool NT>
__device__ __forceinline__ void restore_zero_chunk(const ChunkArgs &a, const Desc &d, int lane)
{
    const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t p = (uint32_t)lane * 16; p < d.len; p += 64 * 16)
        st16<NT>((uint8_t *)d.dst + p, zero);
    if (lane == 0 && a.zero_crc != d.want) {
        a.bad[d.g] = 1;
        atomicAdd(&a.plan_rw->bad_count, 1ull);
    }
}

// Pack / hash of a full-length ZERO chunk: its CRC is that of C zero bytes,
// known beforehand, and the dense image leaves it unwritten.
__device__ __forceinline__ void record_zero_chunk(const ChunkArgs &a, const Desc &d)
{
    uint8_t f = kFlagZero;
    if (!d.has_base || d.want != a.zero_crc)
        f |= kFlagDirty;
    a.crc[d.g] = a.zero_crc;
    a.flags[d.g] = f;
}

template <int MODE>
__device__ __forceinline__ void finish_chunk(const ChunkArgs &a, const Desc &d, uint32_t raw, bool nonzero)
{
    const uint32_t crc = finish_crc(raw, d.len);
    if (MODE == kModeRestore) {
        if (crc != d.want) {
            a.bad[d.g] = 1;
            atomicAdd(&a.plan_rw->bad_count, 1ull);
        }
    } else {
        uint8_t f = nonzero ? 0 : kFlagZero;
        if (!d.has_base || d.want != crc)
            f |= kFlagDirty;
        a.crc[d.g] = crc;
        a.flags[d.g] = f;
    }
}

// One chunk of the one-wave form, its loads in v: a full-length ZERO chunk
// of a restore is written as zeros; in a pack or hash, ZERO is known once the
// loads are in, so a ZERO chunk is not stored and a full-length one not
// hashed; every other chunk is hashed (and stored) and finished.
template <int MODE, bool NT>
__device__ __forceinline__ void small_chunk(const ChunkArgs &a, const Tabs &T, const Desc &d, int lane,
                                            uint32_t r_win, uint32_t C, uint4 (&v)[kLoadsInFlight])
{
    if (MODE == kModeRestore && d.zero && d.len == C) {   // uniform over the wave
        restore_zero_chunk<NT>(a, d, lane);
        return;
    }
    bool store = true;
    if (MODE != kModeRestore) {
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < kLoadsInFlight; b++)
            o |= v[b].x | v[b].y | v[b].z | v[b].w;
        store = __ballot(o != 0) != 0;   // uniform over the wave
        if (!store && d.len == C) {
            if (lane == 0)
                record_zero_chunk(a, d);
            return;
        }
    }
    uint32_t orv = 0;
    const uint32_t raw = small_rest<MODE, NT>(T, d, lane, r_win, v, &orv, store);
    const bool nonzero = __ballot(orv != 0) != 0;
    if (lane == 0)
        finish_chunk<MODE>(a, d, raw, nonzero);
}

// The descriptor of item i (chunk g = i, or ids[i] in a delta restore).
template <int MODE>
__device__ __forceinline__ Desc make_desc(const ChunkArgs &a, uint64_t i, uint32_t C)
{
    if (MODE == kModeRestore)
        i += a.item_begin;
    const uint64_t g = (MODE == kModeRestore && a.ids) ? a.ids[i] : i;
    const uint32_t k = a.map[g];
    const uint64_t start = (g - a.cb[k]) * C;
    const uint64_t rest = a.size[k] - start;
    Desc d;
    d.g = g;
    d.len = (uint32_t)(rest < C ? rest : C);
    d.has_base = 0;
    if (MODE == kModeRestore) {
        d.zero = a.want_flags[g] & kFlagZero;
        d.want = a.want_crc[g];
        d.src = d.zero ? 0 : (uint64_t)(a.staging + (a.soff[i] - a.soff_base));
        d.dst = a.dst[k] + start;
    } else {
        d.zero = 0;
        // the base chunk: the same id when the base has this table, else the
        // same chunk of the base allocation with this allocation's id
        uint64_t bg = g;
        d.has_base = a.base_crc != nullptr;
        if (a.base_cb) {
            const uint64_t b0 = a.base_cb[k];
            d.has_base = b0 != kNoBase;
            bg = b0 + (g - a.cb[k]);
        }
        d.want = d.has_base ? a.base_crc[bg] : 0;
        d.src = a.src[k] + start;
        d.dst = (MODE == kModePack) ? (uint64_t)(a.dense + a.off[k] + start) : 0;
    }
    return d;
}

// --------------------------------------------- quad form (hash only, C <= 4 KiB)
//
// Each row of 16 lanes hashes a chunk of its own, four chunks per wave.  A
// chunk of len bytes sits at the end of a window of r_win rounds of 1 KiB as
// in the one-wave form.  The window is cut into stretches of 256 bytes, one
// 16-byte piece per lane: lane l of the row reads piece l of every stretch,
// so each load instruction covers 256 contiguous bytes per row.  The lane
// chains its pieces in order into one register; the last word of a piece
// (but the last piece's) uses the skip operator, which also moves the
// register over the other 15 lanes' pieces of the stretch, so no separate
// round operator is needed.  The row's 16 registers are then combined inside
// the row with the tree operators for 16, 32, 64 and 128 bytes.  The
// cross-lane tree, the flag test and the finish are shared by four chunks,
// which is what this form saves over one wave per chunk.
constexpr int kQuadRows = 64 / kQuadLanes;        // chunks per wave
constexpr int kQuadPieces = 4;                    // 16-byte pieces per lane per round
constexpr int kQuadRoundPieces = kQuadLanes * kQuadPieces;
constexpr int kQuadMaxRounds = 4;
static_assert(kQuadRoundPieces * 16 == kRoundBytes, "a row round is one wave round long");
static_assert(kQuadRows == 4, "the row flags are 16-bit fields of the wave ballot");

// descriptor tile of the quad form: four chunks per wave and four quads per
// wave of a 1024-thread workgroup between two barriers
constexpr int kQuadTile = 256;

// Loads of round b of a row's window (b < r_win): piece j of the lane is
// window piece (4 b + j) * 16 + lr.
template <bool NT>
__device__ __forceinline__ void quad_loads(const Desc &d, bool valid, bool exact, int lr, uint32_t r_win, uint32_t b,
                                           uint4 (&v)[kQuadPieces])
{
    const uint32_t first = b * kQuadRoundPieces + lr;   // window piece of v[0]
    if (exact) {   // every row's chunk fills its window: whole pieces, no offset
#pragma unroll
        for (int j = 0; j < kQuadPieces; j++)
            v[j] = ld16<NT>((const uint8_t *)d.src + (first + j * kQuadLanes) * 16);
        return;
    }
    const int z = valid ? (int)(r_win * kQuadRoundPieces) - (int)((d.len + 15) >> 4) : 0;
#pragma unroll
    for (int j = 0; j < kQuadPieces; j++) {
        const int p = (int)(first + j * kQuadLanes) - z;
        v[j] = make_uint4(0u, 0u, 0u, 0u);
        if (valid && p >= 0)
            v[j] = load_piece<kModeHash, NT>(d, (uint32_t)p * 16);
    }
}

// Chains round b's pieces into the lane's register (T is the quad table set:
// its gap operator is the skip) and ORs their data words into *o.
__device__ __forceinline__ void quad_hash(const Tabs &T, const Desc &d, bool valid, bool exact, int lr,
                                          uint32_t r_win, uint32_t b, uint4 (&v)[kQuadPieces], uint32_t *acc,
                                          uint32_t *o)
{
    const uint32_t first = b * kQuadRoundPieces + lr;
    const int z = (valid && !exact) ? (int)(r_win * kQuadRoundPieces) - (int)((d.len + 15) >> 4) : 0;
    const bool last_round = b + 1 == r_win;   // uniform over the wave
    uint32_t r = *acc;
#pragma unroll
    for (int j = 0; j < kQuadPieces; j++) {
        *o |= v[j].x | v[j].y | v[j].z | v[j].w;
        // the first data byte's piece carries the complemented init (zero
        // pieces before it leave the register at zero)
        if (exact) {
            if (first + j * kQuadLanes == 0)
                v[j].x = ~v[j].x;
        } else if (valid && (int)(first + j * kQuadLanes) == z) {
            v[j].x ^= init_mask(d.len);
        }
        r = T.chain(r, v[j].x);
        r = T.chain(r, v[j].y);
        r = T.chain(r, v[j].z);
        if (j == kQuadPieces - 1 && last_round)
            r = T.chain(r, v[j].w);   // the window ends with this stretch
        else
            r = T.gap(r ^ v[j].w);    // 4 bytes, then the other lanes' pieces
    }
    *acc = r;
}

// The row's 16 registers combined into the row's lane 0 (DPP row shifts):
// at level k, lane i moves its register past the 16 << k bytes of lane
// i + 2^k's pieces and adds that lane's register.
__device__ __forceinline__ uint32_t quad_combine(const Tabs &T, uint32_t acc, int lane)
{
    uint32_t right = dpp_down<1>(acc);
    if ((lane & 1) == 0)
        acc = T.tree(0, acc) ^ right;
    right = dpp_down<2>(acc);
    if ((lane & 3) == 0)
        acc = T.tree(1, acc) ^ right;
    right = dpp_down<4>(acc);
    if ((lane & 7) == 0)
        acc = T.tree(2, acc) ^ right;
    right = dpp_down<8>(acc);
    if ((lane & 15) == 0)
        acc = T.tree(3, acc) ^ right;
    return acc;
}

// Tile counters: every taker (a workgroup of a chunk launch, a wave of a
// gather) takes tiles until its first miss (a value of at least n_tiles), so
// a launch makes n_tiles + takers takes.  The taker whose miss is the last
// take of the launch sets the counter back to zero for the next launch on the
// same plan (such launches are stream-ordered, and the host writes every plan
// with zero counters).
__device__ __forceinline__ uint64_t take_tile(unsigned long long *ctr)
{
    return atomicAdd(ctr, 1ull);
}

__device__ __forceinline__ void tiles_done(unsigned long long *ctr, uint64_t miss, uint64_t n_tiles, uint64_t takers)
{
    if (miss == n_tiles + takers - 1)
        atomicExch(ctr, 0ull);
}

// FORM: kFormWave (one or more waves per chunk), kFormSmall (every chunk is
// one batch of rounds and one wave hashes it; the wave keeps the next chunk's
// loads in flight while it finishes the current one) or kFormQuad (above).
// The host picks kFormSmall and kFormQuad only where they apply.
constexpr int kFormWave = 0;
constexpr int kFormSmall = 1;
constexpr int kFormQuad = 2;

template <int MODE, bool NT, int FORM = kFormWave>
__global__ __launch_bounds__(1024) void k_chunks(ChunkArgs a)
{
    __shared__ uint32_t tabs[kRepWords];
    // two descriptor tiles: the first wave loads the next tile's descriptors
    // while the workgroup works on the current one
    constexpr int kDescTile = FORM == kFormQuad ? kQuadTile : kTile;
    __shared__ Desc desc[2][kDescTile];
    __shared__ uint32_t s_part[16];
    __shared__ uint32_t s_nz[16];

    for (int i = threadIdx.x; i < kRepWords; i += blockDim.x)
        tabs[i] = a.tables[i];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const Tabs T = make_tabs(tabs, lane);
    const int nwaves = blockDim.x >> 6;
    const int W = a.waves_per_chunk;
    const int groups = nwaves / W, group = wave / W, wig = wave % W;
    const uint32_t C = a.C;
    const uint32_t r_full = (C + kRoundBytes - 1) / kRoundBytes;
    const uint32_t rw = (r_full + W - 1) / W;            // rounds per wave
    const uint32_t r_win = rw * W;
    const uint64_t M = (MODE != kModeRestore) ? a.plan->n_chunks
                       : a.item_end ? a.item_end - a.item_begin : a.plan->n_items;

    // The items go in tiles that the workgroups take in order from a counter
    // in the plan, one tile ahead (thread 0 takes the tile after the next
    // while the workgroup works on the current one), so the grid sweeps the
    // memory in order and a workgroup whose tiles are cheap (ZERO chunks,
    // read only) takes more of them.
    // A tile holds at most kDescTile chunks and, for large chunks, about
    // 1 MiB (but at least one chunk per group of waves), so that a launch
    // has many tiles per workgroup and its last tiles end close together.
    int tile = kDescTile < (int)blockDim.x ? kDescTile : (int)blockDim.x;
    if (FORM == kFormWave) {
        const int by_bytes = (int)((1u << 20) / C);
        const int want = by_bytes > groups ? by_bytes : groups;
        tile = want < tile ? want : tile;
    }
    const uint64_t n_tiles = (M + tile - 1) / tile;
    const bool stager = (int)threadIdx.x < tile;
    __shared__ uint64_t s_tile[2];
    if (threadIdx.x == 0) {
        const uint64_t c = take_tile(&a.plan_rw->tile_next);
        uint64_t n = n_tiles;
        if (c < n_tiles)
            n = take_tile(&a.plan_rw->tile_next);
        if (c >= n_tiles)
            tiles_done(&a.plan_rw->tile_next, c, n_tiles, gridDim.x);
        else if (n >= n_tiles)
            tiles_done(&a.plan_rw->tile_next, n, n_tiles, gridDim.x);
        s_tile[0] = c;
        s_tile[1] = n;
    }
    __syncthreads();
    uint64_t cur = s_tile[0], nxt = s_tile[1];   // the tile worked on, the tile staged meanwhile
    if (cur < n_tiles && stager && cur * tile + threadIdx.x < M)
        desc[0][threadIdx.x] = make_desc<MODE>(a, cur * tile + threadIdx.x, C);
    int buf = 0;
    for (uint32_t it = 0; cur < n_tiles; it++, buf ^= 1) {
        __syncthreads();   // tables, this tile's descriptors and the last take are in LDS
        if (it > 0)
            nxt = s_tile[(it + 1) & 1];   // taken during the previous iteration
        uint64_t taken = n_tiles;
        if (threadIdx.x == 0 && nxt < n_tiles)
            taken = take_tile(&a.plan_rw->tile_next);   // its value is first needed at the end of the tile
        const uint64_t g0 = cur * tile, hi = g0 + tile < M ? g0 + tile : M;
        const uint64_t n0 = nxt * tile, n1 = nxt < n_tiles ? (n0 + tile < M ? n0 + tile : M) : n0;
        Desc nd;
        if (stager && n0 + threadIdx.x < n1)
            nd = make_desc<MODE>(a, n0 + threadIdx.x, C);   // loads in flight during the tile
        const int cnt = (int)(hi - g0);   // uniform over the workgroup, at most tile
        if constexpr (FORM == kFormQuad) {
            static_assert(MODE == kModeHash, "the quad form only hashes");
            // This wave's quads of the tile, round by round: the next round's
            // loads (of this quad, or the first of the next) are in flight
            // while the current round is hashed.
            const int q = lane / kQuadLanes, lr = lane & (kQuadLanes - 1);
            const int stride = kQuadRows * nwaves, first = kQuadRows * wave;
            const int nq = first < cnt ? (cnt - first + stride - 1) / stride : 0;   // uniform over the wave
            Desc dn;
            bool vn = false, en = false;
            uint4 cur[kQuadPieces], nxt[kQuadPieces];
            if (nq > 0) {
                vn = first + q < cnt;
                if (vn)
                    dn = desc[buf][first + q];
                en = __ballot(!vn || dn.len != r_win * kRoundBytes) == 0;
                quad_loads<NT>(dn, vn, en, lr, r_win, 0, nxt);
            }
            for (int k = 0; k < nq; k++) {
                const Desc dc = dn;
                const bool vc = vn, ec = en;
                uint32_t acc = 0, orv = 0;
                for (uint32_t b = 0; b < r_win; b++) {
#pragma unroll
                    for (int j = 0; j < kQuadPieces; j++)
                        cur[j] = nxt[j];
                    if (b + 1 < r_win) {
                        quad_loads<NT>(dc, vc, ec, lr, r_win, b + 1, nxt);
                    } else if (k + 1 < nq) {
                        const int t = first + (k + 1) * stride + q;
                        vn = t < cnt;
                        if (vn)
                            dn = desc[buf][t];
                        en = __ballot(!vn || dn.len != r_win * kRoundBytes) == 0;
                        quad_loads<NT>(dn, vn, en, lr, r_win, 0, nxt);
                    }
                    quad_hash(T, dc, vc, ec, lr, r_win, b, cur, &acc, &orv);
                }
                const uint32_t raw = quad_combine(T, acc, lane);
                const uint64_t nz = __ballot(orv != 0);
                if (vc && lr == 0)
                    finish_chunk<MODE>(a, dc, raw, ((nz >> (q * kQuadLanes)) & 0xFFFFull) != 0);
            }
        } else if constexpr (FORM == kFormSmall) {
            // Two register buffers in rotation: while the wave hashes and
            // stores one chunk, the next chunk's loads are in flight.  The
            // loop is unrolled by two so that no buffer is ever copied into
            // the other (a copy would wait for its loads).
            uint4 v0[kLoadsInFlight], v1[kLoadsInFlight];
            const Desc *td = desc[buf];
            if (group < cnt)
                small_loads<MODE, NT>(td[group], lane, r_win, v0);
            for (int t = group; t < cnt; t += 2 * groups) {   // uniform over the wave
                if (t + groups < cnt)
                    small_loads<MODE, NT>(td[t + groups], lane, r_win, v1);
                small_chunk<MODE, NT>(a, T, td[t], lane, r_win, C, v0);
                if (t + groups >= cnt)
                    break;
                if (t + 2 * groups < cnt)
                    small_loads<MODE, NT>(td[t + 2 * groups], lane, r_win, v0);
                small_chunk<MODE, NT>(a, T, td[t + groups], lane, r_win, C, v1);
            }
        } else {
        for (int slot = 0; slot < cnt; slot += groups) {
            const int t = slot + group;
            const bool valid = t < cnt;
            uint32_t raw = 0, orv = 0;
            Desc d;
            if (valid) {
                d = desc[buf][t];
                if (MODE == kModeRestore && W == 1 && d.zero && d.len == C) {   // uniform over the wave
                    restore_zero_chunk<NT>(a, d, lane);
                    continue;
                }
                raw = wave_rounds<MODE, NT>(T, d, lane, wig * rw, (wig + 1) * rw, r_win, &orv);
            }
            const bool nonzero = __ballot(orv != 0) != 0;
            if (W == 1) {
                if (valid && lane == 0)
                    finish_chunk<MODE>(a, d, raw, nonzero);
            } else {
                if (lane == 0) {
                    s_part[wave] = raw;
                    s_nz[wave] = nonzero;
                }
                __syncthreads();
                if (valid && wig == 0 && lane == 0) {
                    uint32_t acc = s_part[wave];
                    bool nz = s_nz[wave];
                    for (int w = 1; w < W; w++) {
                        acc = T.seg(acc) ^ s_part[wave + w];
                        nz = nz || s_nz[wave + w];
                    }
                    finish_chunk<MODE>(a, d, acc, nz);
                }
                __syncthreads();
            }
        }
        }
        if (stager && n0 + threadIdx.x < n1)
            desc[buf ^ 1][threadIdx.x] = nd;   // the other tile was consumed before the last barrier
        if (threadIdx.x == 0 && nxt < n_tiles) {
            s_tile[it & 1] = taken;   // read after the next barrier
            if (taken >= n_tiles)
                tiles_done(&a.plan_rw->tile_next, taken, n_tiles, gridDim.x);
        }
        cur = nxt;
    }
}

// ------------------------------------------------- row mode (serving loop)
//
// Same per-chunk work as k_chunks (one wave per chunk), but each item's
// addresses come from its row, and each row says whether its chunks are
// packed or restored; the branch is uniform across a wave.

struct RowDesc {
    Desc d;
    uint64_t crc, flags, bad, bad_count;
    uint32_t mode, pad;
};

__device__ __forceinline__ RowDesc make_row_desc(const RowArgs &a, uint64_t i, uint32_t C)
{
    const StepRow &row = a.rows[a.map[i]];
    const uint64_t c = i - row.item0;
    const uint64_t start = c * C;
    const uint64_t rest = row.rem - start;
    RowDesc r;
    r.d.g = i;
    r.d.len = (uint32_t)(rest < C ? rest : C);
    r.d.has_base = 0;
    r.mode = row.mode;
    r.pad = 0;
    r.crc = row.crc + 4 * c;
    r.flags = row.flags + c;
    r.bad = row.bad + c;
    r.bad_count = row.bad_count;
    if (row.mode == kModeRestore) {
        r.d.zero = *(const uint8_t *)r.flags & kFlagZero;
        r.d.want = *(const uint32_t *)r.crc;
        r.d.src = r.d.zero ? 0 : row.src + ((const uint64_t *)row.soff)[c];
    } else {
        r.d.zero = 0;
        r.d.want = 0;
        r.d.src = row.src + start;
    }
    r.d.dst = row.dst + start;
    return r;
}

template <bool NT>
__global__ __launch_bounds__(1024) void k_rows(RowArgs a)
{
    __shared__ uint32_t tabs[kRepWords];
    __shared__ RowDesc desc[2][kTile];

    for (int i = threadIdx.x; i < kRepWords; i += blockDim.x)
        tabs[i] = a.tables[i];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const Tabs T = make_tabs(tabs, lane);
    const int nwaves = blockDim.x >> 6;
    const uint32_t C = a.C;
    const uint32_t r_win = (C + kRoundBytes - 1) / kRoundBytes;
    const uint64_t M = a.n_items;

    // Tiles taken from the step's counter, one ahead, and double-buffered
    // descriptors, as in k_chunks.
    const uint64_t n_tiles = (M + kTile - 1) / kTile;
    const bool stager = threadIdx.x < kTile;
    __shared__ uint64_t s_tile[2];
    if (threadIdx.x == 0) {
        const uint64_t c = take_tile(a.tile_ctr);
        uint64_t n = n_tiles;
        if (c < n_tiles)
            n = take_tile(a.tile_ctr);
        if (c >= n_tiles)
            tiles_done(a.tile_ctr, c, n_tiles, gridDim.x);
        else if (n >= n_tiles)
            tiles_done(a.tile_ctr, n, n_tiles, gridDim.x);
        s_tile[0] = c;
        s_tile[1] = n;
    }
    __syncthreads();
    uint64_t cur = s_tile[0], nxt = s_tile[1];
    if (cur < n_tiles && stager && cur * kTile + threadIdx.x < M)
        desc[0][threadIdx.x] = make_row_desc(a, cur * kTile + threadIdx.x, C);
    int buf = 0;
    for (uint32_t it = 0; cur < n_tiles; it++, buf ^= 1) {
        __syncthreads();
        if (it > 0)
            nxt = s_tile[(it + 1) & 1];
        uint64_t taken = n_tiles;
        if (threadIdx.x == 0 && nxt < n_tiles)
            taken = take_tile(a.tile_ctr);
        const uint64_t g0 = cur * kTile, hi = g0 + kTile < M ? g0 + kTile : M;
        const uint64_t n0 = nxt * kTile, n1 = nxt < n_tiles ? (n0 + kTile < M ? n0 + kTile : M) : n0;
        RowDesc nd;
        if (stager && n0 + threadIdx.x < n1)
            nd = make_row_desc(a, n0 + threadIdx.x, C);
        const int cnt = (int)(hi - g0);
        for (int t = wave; t < cnt; t += nwaves) {
            const RowDesc rd = desc[buf][t];
            uint32_t raw, orv;
            if (rd.mode == kModeRestore)
                raw = wave_rounds<kModeRestore, NT>(T, rd.d, lane, 0, r_win, r_win, &orv);
            else
                raw = wave_rounds<kModePack, NT>(T, rd.d, lane, 0, r_win, r_win, &orv);
            const bool nonzero = __ballot(orv != 0) != 0;
            if (lane == 0) {
                const uint32_t crc = finish_crc(raw, rd.d.len);
                if (rd.mode == kModeRestore) {
                    if (crc != rd.d.want) {
                        *(uint8_t *)rd.bad = 1;
                        atomicAdd((unsigned long long *)rd.bad_count, 1ull);
                    }
                } else {
                    *(uint32_t *)rd.crc = crc;
                    *(uint8_t *)rd.flags = (nonzero ? 0 : kFlagZero) | kFlagDirty;
                }
            }
        }
        if (stager && n0 + threadIdx.x < n1)
            desc[buf ^ 1][threadIdx.x] = nd;
        if (threadIdx.x == 0 && nxt < n_tiles) {
            s_tile[it & 1] = taken;
            if (taken >= n_tiles)
                tiles_done(a.tile_ctr, taken, n_tiles, gridDim.x);
        }
        cur = nxt;
    }
}

// ------------------------------------------------------ K5: selection scan
//
// Reduce-then-scan over items in tiles of kSelTile: each thread owns
// kSelPerThread consecutive items.  Per item: `bytes` (roundup16 of the
// chunk's length when the chunk is selected) and `count` (1 when its id goes
// to the id list).  soff[i] gets the exclusive prefix of bytes; ids_out gets
// the counted ids in ascending order.

__device__ __forceinline__ uint64_t sel_items(const SelArgs &a)
{
    return a.mode == kSelIdsNonZero ? a.plan->n_items : a.plan->n_chunks;
}

__device__ __forceinline__ void sel_item(const SelArgs &a, uint64_t i, uint64_t *bytes, uint32_t *count,
                                         uint64_t *gout)
{
    const uint64_t g = a.mode == kSelIdsNonZero ? a.ids[i] : i;
    const uint8_t f = a.flags[g];
    bool take_bytes = false;
    uint32_t c = 0;
    switch (a.mode) {
    case kSelNonZero:
    case kSelIdsNonZero:
        take_bytes = !(f & kFlagZero);
        break;
    case kSelDirtyNonZero:
        take_bytes = (f & kFlagDirty) && !(f & kFlagZero);
        c = (f & kFlagDirty) ? 1 : 0;
        break;
    default:   // kSelBad: flags holds the bad marks
        c = f ? 1 : 0;
        break;
    }
    uint64_t b = 0;
    if (take_bytes) {
        const uint32_t k = a.map[g];
        const uint64_t rest = a.size[k] - (g - a.cb[k]) * a.C;
        b = round_up16(rest < a.C ? rest : a.C);
    }
    *bytes = b;
    *count = c;
    *gout = g;
}

// Block-wide exclusive scan of (bytes, count) pairs; returns the block totals.
__device__ __forceinline__ void block_excl_scan(uint64_t &b, uint64_t &c, uint64_t *tot_b, uint64_t *tot_c)
{
    __shared__ uint64_t sb[16], sc[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint64_t ib = wave_incl_scan(b, lane), ic = wave_incl_scan(c, lane);
    if (lane == 63) {
        sb[wave] = ib;
        sc[wave] = ic;
    }
    __syncthreads();
    uint64_t pb = 0, pc = 0, tb = 0, tc = 0;
    for (int w = 0; w < nw; w++) {
        if (w < wave) {
            pb += sb[w];
            pc += sc[w];
        }
        tb += sb[w];
        tc += sc[w];
    }
    __syncthreads();
    b = pb + ib - b;
    c = pc + ic - c;
    *tot_b = tb;
    *tot_c = tc;
}

__global__ __launch_bounds__(kSelThreads) void k_sel_reduce(SelArgs a)
{
    const uint64_t M = sel_items(a);
    const uint64_t base = (uint64_t)blockIdx.x * kSelTile + (uint64_t)threadIdx.x * kSelPerThread;
    uint64_t b = 0, c = 0;
    if ((uint64_t)blockIdx.x * kSelTile < M) {
        for (int j = 0; j < kSelPerThread; j++) {
            const uint64_t i = base + j;
            if (i < M) {
                uint64_t ib, g;
                uint32_t ic;
                sel_item(a, i, &ib, &ic, &g);
                b += ib;
                c += ic;
            }
        }
    }
    uint64_t tb, tc;
    block_excl_scan(b, c, &tb, &tc);
    if (threadIdx.x == 0) {
        a.tile_bytes[blockIdx.x] = tb;
        a.tile_count[blockIdx.x] = tc;
    }
}

__global__ __launch_bounds__(1024) void k_sel_scan(SelArgs a)
{
    const uint64_t M = sel_items(a);
    const uint64_t tiles = (M + kSelTile - 1) / kSelTile;
    uint64_t carry_b = 0, carry_c = 0;
    for (uint64_t base = 0; base < tiles; base += 1024) {
        const uint64_t t = base + threadIdx.x;
        uint64_t b = t < tiles ? a.tile_bytes[t] : 0, c = t < tiles ? a.tile_count[t] : 0;
        uint64_t tb, tc;
        block_excl_scan(b, c, &tb, &tc);
        if (t < tiles) {
            a.tile_bytes[t] = carry_b + b;
            a.tile_count[t] = carry_c + c;
        }
        carry_b += tb;
        carry_c += tc;
    }
    if (threadIdx.x == 0) {
        a.plan->sel_bytes = carry_b;
        a.plan->sel_count = carry_c;
    }
}

__global__ __launch_bounds__(kSelThreads) void k_sel_down(SelArgs a)
{
    const uint64_t M = sel_items(a);
    if ((uint64_t)blockIdx.x * kSelTile >= M)
        return;
    const uint64_t base = (uint64_t)blockIdx.x * kSelTile + (uint64_t)threadIdx.x * kSelPerThread;
    uint64_t ib[kSelPerThread], ig[kSelPerThread];
    uint32_t ic[kSelPerThread];
    uint64_t b = 0, c = 0;
    for (int j = 0; j < kSelPerThread; j++) {
        const uint64_t i = base + j;
        ib[j] = 0;
        ic[j] = 0;
        ig[j] = 0;
        if (i < M)
            sel_item(a, i, &ib[j], &ic[j], &ig[j]);
        b += ib[j];
        c += ic[j];
    }
    uint64_t tb, tc;
    block_excl_scan(b, c, &tb, &tc);
    b += a.tile_bytes[blockIdx.x];
    c += a.tile_count[blockIdx.x];
    for (int j = 0; j < kSelPerThread; j++) {
        const uint64_t i = base + j;
        if (i < M) {
            if (a.soff)
                a.soff[i] = b;
            if (ic[j] && a.ids_out && c < a.ids_cap)
                a.ids_out[c] = ig[j];
        }
        b += ib[j];
        c += ic[j];
    }
}

// --------------------------------------------------------------- K6: gather
//
// Copies each selected chunk (roundup16(len) bytes) to out + soff[g], from the
// dense image or straight from the allocation (zero pad written, never read);
// or, for several outputs in host memory, into each output's own buffer.
// A workgroup takes tiles of 16 * `tile` consecutive chunks (`tile` up to 64,
// fewer when a launch covers few chunks, so that every wave of the grid has
// work); wave w of the workgroup takes chunks w, w + 16, ... of the tile, and
// its lane l fetches the descriptor of the l-th of them, so the descriptor
// loads are in flight together.  The wave then copies its selected chunks one
// after the other (their addresses read from the owning lane), each lane
// issuing up to kGatherLoads 16-byte loads before its first store.

constexpr int kGatherLoads = 8;

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int j)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

template <bool NT_ST>
__device__ __forceinline__ void gather_copy(const uint8_t *s, uint8_t *d, uint32_t n, bool whole, int lane)
{
    const uint32_t np = (n + 15) >> 4;
    for (uint32_t p0 = 0; p0 < np; p0 += 64 * kGatherLoads) {
        uint4 v[kGatherLoads];
#pragma unroll
        for (int u = 0; u < kGatherLoads; u++) {
            const uint32_t p = p0 + u * 64 + lane;
            v[u] = make_uint4(0u, 0u, 0u, 0u);
            if (p < np) {
                const uint32_t o = 16 * p;
                // the dense image's pad is zero and may be read; an allocation's tail may not
                v[u] = (whole || o + 16 <= n) ? ld16<true>(s + o) : load_partial(s + o, n - o);
            }
        }
#pragma unroll
        for (int u = 0; u < kGatherLoads; u++) {
            const uint32_t p = p0 + u * 64 + lane;
            if (p < np)
                st16<NT_ST>(d + 16 * p, v[u]);
        }
    }
}

template <bool NT_ST>
__global__ __launch_bounds__(1024) void k_gather(GatherArgs a)
{
    __shared__ uint64_t s_t[2];
    const uint64_t N = a.g_end ? a.g_end : a.plan->n_chunks;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t tile = a.tile;                       // chunks per wave per tile
    const uint64_t span = (uint64_t)tile * nw;          // chunks per tile
    const uint64_t n_tiles = N > a.g_begin ? (N - a.g_begin + span - 1) / span : 0;
    // Workgroup b's first tile is tile b; the rest are taken in order from the
    // plan's counter by thread 0, so that a workgroup whose tiles hold few
    // selected chunks takes more of them.  The waves of a workgroup share its
    // tile chunk by chunk (wave w: chunks w, w + nw, ...), so that together
    // they stream through one window of memory.
    const uint64_t n_dyn = n_tiles > gridDim.x ? n_tiles - gridDim.x : 0;
    for (uint32_t it = 0;; it++) {
        if (threadIdx.x == 0) {
            uint64_t t = n_tiles;
            if (it == 0) {
                t = blockIdx.x;
            } else if (n_dyn) {
                const uint64_t v = take_tile(a.tile_ctr);
                if (v >= n_dyn)
                    tiles_done(a.tile_ctr, v, n_dyn, gridDim.x);
                t = gridDim.x + v;
            }
            s_t[it & 1] = t;   // the other slot may still be read
        }
        __syncthreads();
        const uint64_t cur = s_t[it & 1];
        if (cur >= n_tiles)
            break;
        const uint64_t g = a.g_begin + cur * span + (uint64_t)lane * nw + wave;
        bool take = false;
        uint64_t src = 0, dst = 0;
        uint32_t len = 0;
        if ((uint32_t)lane < tile && g < N) {
            const uint8_t f = a.flags[g];
            const uint32_t k = a.map[g];
            const uint64_t so = a.soff[g];
            take = a.mode == kSelNonZero ? !(f & kFlagZero) : ((f & kFlagDirty) && !(f & kFlagZero));
            if (take) {
                const uint64_t start = (g - a.cb[k]) * a.C;
                const uint64_t rest = a.size[k] - start;
                len = (uint32_t)(rest < a.C ? rest : a.C);
                src = a.from_dense ? (uint64_t)(a.dense + a.off[k] + start) : a.src[k] + start;
                if (a.out_addr) {
                    const uint32_t o = a.row_out[k];
                    dst = a.out_addr[o] + (so - a.soff[a.out_chunk0[o]]);
                } else {
                    dst = (uint64_t)(a.out + (so - a.soff_base));
                }
            }
        }
        uint64_t m = __ballot(take);
        while (m) {
            const int j = __builtin_ctzll(m);   // uniform over the wave
            m &= m - 1;
            gather_copy<NT_ST>((const uint8_t *)readlane_u64(src, j), (uint8_t *)readlane_u64(dst, j),
                               (uint32_t)__builtin_amdgcn_readlane((int)len, j), a.from_dense != 0, lane);
        }
    }
}

// ------------------------------------------------------------------ helpers

__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// The allocation table as the host keeps it (rows of four words: id, kind,
// address, size) split into the address and size arrays the scan and the
// chunk kernels read; the first thread also writes a fresh plan for n rows.
__global__ void k_table_split(const uint64_t *__restrict__ rows, uint64_t n, DevPlan *plan,
                              uint64_t *__restrict__ addr, uint64_t *__restrict__ size)
{
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) {
        DevPlan p = {};
        p.n_allocs = n;
        *plan = p;
    }
    for (uint64_t k = i0; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
        addr[k] = rows[4 * k + 2];
        size[k] = rows[4 * k + 3];
    }
}

__global__ void k_pick_u64(const uint64_t *src, const uint64_t *idx, uint64_t *out, uint32_t m)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m)
        out[i] = src[idx[i]];
}

// ----------------------------------------------------------- launch wrappers

hipError_t launch_layout_scan(hipStream_t s, DevPlan *plan, const uint64_t *size, uint32_t C, uint64_t *off,
                              uint64_t *cb)
{
    hipLaunchKernelGGL(k_layout_scan<false>, dim3(1), dim3(1024), 0, s, plan, const_cast<uint64_t *>(size), C, off,
                       cb, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_upload_scan(hipStream_t s, const void *up, DevPlan *plan, uint64_t *addr, uint64_t *size,
                              uint32_t C, uint64_t *off, uint64_t *cb)
{
    hipLaunchKernelGGL(k_layout_scan<true>, dim3(1), dim3(1024), 0, s, plan, size, C, off, cb, (const uint8_t *)up,
                       addr);
    return hipGetLastError();
}

hipError_t launch_chunk_map(hipStream_t s, const DevPlan *plan, const uint64_t *cb, uint32_t *map, int grid)
{
    hipLaunchKernelGGL(k_chunk_map, dim3(grid), dim3(256), 0, s, plan, cb, map);
    return hipGetLastError();
}

template <int MODE>
static void launch_chunks_m(hipStream_t s, const ChunkArgs &a, int grid, int block)
{
    const uint32_t rounds = (a.C + kRoundBytes - 1) / kRoundBytes;
    // hash-only chunks of at most 4 KiB: four chunks per wave
    if (MODE == kModeHash && a.tables_quad && a.waves_per_chunk == 1 && rounds <= kQuadMaxRounds) {
        ChunkArgs q = a;
        q.tables = a.tables_quad;
        if (a.nontemporal)
            hipLaunchKernelGGL((k_chunks<kModeHash, true, kFormQuad>), dim3(grid), dim3(block), 0, s, q);
        else
            hipLaunchKernelGGL((k_chunks<kModeHash, false, kFormQuad>), dim3(grid), dim3(block), 0, s, q);
        return;
    }
    // one wave per chunk and one batch of rounds per chunk: the pipelined form
    const bool small = a.waves_per_chunk == 1 && rounds <= kLoadsInFlight;
    if (small) {
        if (a.nontemporal)
            hipLaunchKernelGGL((k_chunks<MODE, true, kFormSmall>), dim3(grid), dim3(block), 0, s, a);
        else
            hipLaunchKernelGGL((k_chunks<MODE, false, kFormSmall>), dim3(grid), dim3(block), 0, s, a);
    } else if (a.nontemporal) {
        hipLaunchKernelGGL((k_chunks<MODE, true>), dim3(grid), dim3(block), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_chunks<MODE, false>), dim3(grid), dim3(block), 0, s, a);
    }
}

hipError_t launch_chunks(hipStream_t s, int mode, const ChunkArgs &a, int grid, int block)
{
    switch (mode) {
    case kModePack: launch_chunks_m<kModePack>(s, a, grid, block); break;
    case kModeHash: launch_chunks_m<kModeHash>(s, a, grid, block); break;
    default: launch_chunks_m<kModeRestore>(s, a, grid, block); break;
    }
    return hipGetLastError();
}

hipError_t launch_rows(hipStream_t s, const RowArgs &a, int grid, int block)
{
    if (a.nontemporal)
        hipLaunchKernelGGL((k_rows<true>), dim3(grid), dim3(block), 0, s, a);
    else
        hipLaunchKernelGGL((k_rows<false>), dim3(grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_select(hipStream_t s, const SelArgs &a, uint64_t max_items)
{
    const uint64_t tiles = (max_items + kSelTile - 1) / kSelTile;
    const unsigned grid = (unsigned)(tiles ? tiles : 1);
    hipLaunchKernelGGL(k_sel_reduce, dim3(grid), dim3(kSelThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(1024), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sel_down, dim3(grid), dim3(kSelThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gather(hipStream_t s, const GatherArgs &a_in, int grid)
{
    GatherArgs a = a_in;
    a.tile_ctr = (unsigned long long *)((uintptr_t)a.plan + offsetof(DevPlan, gather_next));
    // a launch over a chunk range gives every wave of the grid at least one
    // tile; without a range (all chunks of the plan) the tile is 64
    a.tile = 64;
    if (a.g_end) {
        const uint64_t per_wave = (a.g_end - a.g_begin) / ((uint64_t)grid * 16);
        while (a.tile > 1 && a.tile > per_wave)
            a.tile >>= 1;
    }
    // stores into pinned host memory (the direct drain) keep the default policy
    if (a.out_host)
        hipLaunchKernelGGL(k_gather<false>, dim3(grid), dim3(1024), 0, s, a);
    else
        hipLaunchKernelGGL(k_gather<true>, dim3(grid), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_u64(hipStream_t s, uint64_t *p, uint64_t n_words, uint64_t value)
{
    if (n_words == 0)
        return hipSuccess;
    uint64_t blocks = (n_words + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, n_words, value);
    return hipGetLastError();
}

hipError_t launch_table_split(hipStream_t s, const uint64_t *rows, uint64_t n, DevPlan *plan, uint64_t *addr,
                              uint64_t *size)
{
    uint64_t blocks = (n + 255) / 256;
    blocks = blocks < 1 ? 1 : blocks > 1024 ? 1024 : blocks;
    hipLaunchKernelGGL(k_table_split, dim3((unsigned)blocks), dim3(256), 0, s, rows, n, plan, addr, size);
    return hipGetLastError();
}

hipError_t launch_pick_u64(hipStream_t s, const uint64_t *src, const uint64_t *idx, uint64_t *out, uint32_t m)
{
    if (m == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pick_u64, dim3((m + 255) / 256), dim3(256), 0, s, src, idx, out, m);
    return hipGetLastError();
}

}  // namespace ckpt
