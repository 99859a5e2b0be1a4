// probe.hip -- plain HBM read, write and copy kernels for measurement only
// (libckpt_probe.so, loaded by bench.py): they give the ceilings that the
// drain/refill kernels of libckpt are compared with.  None of them is on the
// checkpoint path.
//
// Each static kernel sweeps one buffer with a grid of persistent workgroups: in
// iteration i, wave w of W handles the U * 1 KiB at ((i * W + w) * U) KiB, lane
// l the 16-byte pieces l, l + 64, ..., so the whole grid moves through memory
// one window of W * U KiB at a time.  U loads are issued before any of them is
// used (read: OR-reduced; copy: stored).  NT selects non-temporal loads and
// stores.  Sizes must be multiples of 16 bytes; the tail of a window is
// guarded.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ u32x4 ld(const u32x4 *p)
{
    if (NT)
        return __builtin_nontemporal_load(p);
    return *p;
}

template <bool NT>
__device__ __forceinline__ void st(u32x4 *p, u32x4 v)
{
    if (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int U, bool NT>
__global__ __launch_bounds__(1024) void k_read(const u32x4 *__restrict__ src, uint64_t n16, uint32_t *__restrict__ sink)
{
    const uint64_t lane = threadIdx.x & 63;
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t W = (uint64_t)gridDim.x * (blockDim.x >> 6);
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (uint64_t base = w * 64 * U; base < n16; base += W * 64 * U) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t p = base + u * 64 + lane;
            v[u] = p < n16 ? ld<NT>(src + p) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < U; u++)
            acc |= v[u];
    }
    const uint32_t r = acc.x | acc.y | acc.z | acc.w;
    if (r == 0x9E3779B9u)   // practically never: keeps the loads without a store per thread
        sink[0] = r;
}

template <int U, bool NT>
__global__ __launch_bounds__(1024) void k_write(u32x4 *__restrict__ dst, uint64_t n16, uint32_t value)
{
    const uint64_t lane = threadIdx.x & 63;
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t W = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const u32x4 v = {value, value, value, value};
    for (uint64_t base = w * 64 * U; base < n16; base += W * 64 * U) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t p = base + u * 64 + lane;
            if (p < n16)
                st<NT>(dst + p, v);
        }
    }
}

template <int U, bool NT>
__global__ __launch_bounds__(1024) void k_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, uint64_t n16)
{
    const uint64_t lane = threadIdx.x & 63;
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t W = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t base = w * 64 * U; base < n16; base += W * 64 * U) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t p = base + u * 64 + lane;
            v[u] = p < n16 ? ld<NT>(src + p) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t p = base + u * 64 + lane;
            if (p < n16)
                st<NT>(dst + p, v[u]);
        }
    }
}

// A copy whose loads and stores take separate hints (NL: loads, NS: stores).
template <int U, bool NL, bool NS>
__global__ __launch_bounds__(1024) void k_copy2(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, uint64_t n16)
{
    const uint64_t lane = threadIdx.x & 63;
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t W = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t base = w * 64 * U; base < n16; base += W * 64 * U) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t p = base + u * 64 + lane;
            v[u] = p < n16 ? ld<NL>(src + p) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t p = base + u * 64 + lane;
            if (p < n16)
                st<NS>(dst + p, v[u]);
        }
    }
}

// The same three kernels as the chunk kernels of libckpt schedule their work:
// each workgroup takes tiles of 256 KiB in order from a counter (thread 0
// takes, the workgroup reads the value from LDS), and its waves take the
// tile's blocks of 64 * U pieces in turn (KIND 0 read, 1 write, 2 copy; both
// hints alike).  Every workgroup takes until its first miss (a value of at
// least n_tiles); the workgroup whose miss is the launch's last take sets the
// counter back to zero for the next launch.
__device__ unsigned long long g_tile;
constexpr uint64_t kTile16 = 16384;   // 16-byte pieces per tile

template <int KIND, int U, bool NT>
__global__ __launch_bounds__(1024) void k_dyn(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, uint64_t n16,
                                              uint32_t *__restrict__ sink)
{
    __shared__ uint64_t s_t;
    const uint64_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint64_t n_tiles = (n16 + kTile16 - 1) / kTile16;
    u32x4 acc = {0u, 0u, 0u, 0u};
    const u32x4 zero = {0u, 0u, 0u, 0u};
    for (;;) {
        if (threadIdx.x == 0) {
            const uint64_t t = atomicAdd(&g_tile, 1ull);
            if (t == n_tiles + gridDim.x - 1)
                atomicExch(&g_tile, 0ull);
            s_t = t;
        }
        __syncthreads();
        const uint64_t t = s_t;
        __syncthreads();   // every wave has read s_t before it is written again
        if (t >= n_tiles)
            break;
        const uint64_t end = (t + 1) * kTile16 < n16 ? (t + 1) * kTile16 : n16;
        for (uint64_t base = t * kTile16 + wave * 64 * U; base < end; base += nw * 64 * U) {
            u32x4 v[U];
            if (KIND != 1) {
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const uint64_t p = base + u * 64 + lane;
                    v[u] = p < end ? ld<NT>(src + p) : zero;
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const uint64_t p = base + u * 64 + lane;
                if (KIND == 0)
                    acc |= v[u];
                else if (p < end)
                    st<NT>(dst + p, KIND == 1 ? zero : v[u]);
            }
        }
    }
    if (KIND == 0) {
        const uint32_t r = acc.x | acc.y | acc.z | acc.w;
        if (r == 0x9E3779B9u)   // practically never: keeps the loads without a store per thread
            sink[0] = r;
    }
}

template <int U, bool NT>
void launch(int kind, const void *src, void *dst, uint64_t n16, int grid, int block, hipStream_t s)
{
    if (kind == 0)
        hipLaunchKernelGGL((k_read<U, NT>), dim3(grid), dim3(block), 0, s, (const u32x4 *)src, n16, (uint32_t *)dst);
    else if (kind == 1)
        hipLaunchKernelGGL((k_write<U, NT>), dim3(grid), dim3(block), 0, s, (u32x4 *)dst, n16, 0u);
    else if (kind == 2)
        hipLaunchKernelGGL((k_copy<U, NT>), dim3(grid), dim3(block), 0, s, (const u32x4 *)src, (u32x4 *)dst, n16);
    else if (kind == 3)   // non-temporal loads only when NT, regular stores
        hipLaunchKernelGGL((k_copy2<U, NT, false>), dim3(grid), dim3(block), 0, s, (const u32x4 *)src, (u32x4 *)dst,
                           n16);
    else if (kind == 4)   // regular loads, non-temporal stores only when NT
        hipLaunchKernelGGL((k_copy2<U, false, NT>), dim3(grid), dim3(block), 0, s, (const u32x4 *)src, (u32x4 *)dst,
                           n16);
    else if (kind == 5)
        hipLaunchKernelGGL((k_dyn<0, U, NT>), dim3(grid), dim3(block), 0, s, (const u32x4 *)src, nullptr, n16,
                           (uint32_t *)dst);
    else if (kind == 6)
        hipLaunchKernelGGL((k_dyn<1, U, NT>), dim3(grid), dim3(block), 0, s, nullptr, (u32x4 *)dst, n16, nullptr);
    else
        hipLaunchKernelGGL((k_dyn<2, U, NT>), dim3(grid), dim3(block), 0, s, (const u32x4 *)src, (u32x4 *)dst, n16,
                           nullptr);
}

}  // namespace

// kind: 0 read (dst: a 4-byte sink), 1 write, 2 copy, 3 copy with only the
// loads non-temporal (when nt), 4 copy with only the stores non-temporal
// (when nt); 5, 6, 7: read, write and copy taking tiles from a counter.
// Launches of kinds 5-7 must not overlap (they share one counter).  bytes: a multiple of
// 16.  loads: 1, 2, 4, 8 or 16 pieces per lane per iteration; nt: 0/1.
// Returns 0, or -1 for bad arguments, or the hipError_t of the launch.
extern "C" int probe_launch(int kind, const void *src, void *dst, uint64_t bytes, int loads, int nt, int grid,
                            int block, void *stream)
{
    if (kind < 0 || kind > 7 || bytes % 16 || grid <= 0 || (block != 256 && block != 512 && block != 1024))
        return -1;
    if ((kind != 1 && kind != 6 && !src) || !dst)
        return -1;
    const uint64_t n16 = bytes / 16;
    hipStream_t s = (hipStream_t)stream;
#define CASE(U)                                                                          \
    case U:                                                                              \
        if (nt)                                                                          \
            launch<U, true>(kind, src, dst, n16, grid, block, s);                        \
        else                                                                             \
            launch<U, false>(kind, src, dst, n16, grid, block, s);                       \
        break;
    switch (loads) {
        CASE(1)
        CASE(2)
        CASE(4)
        CASE(8)
        CASE(16)
    default:
        return -1;
    }
#undef CASE
    return (int)hipGetLastError();
}
