"""Automatic registration of every PyTorch device allocation.

CRAC logs each allocation and free by interposing on the cudaMalloc family
(Sec. 3.1, "Log-and-replay"; Sec. 3.2, "Issue of library-allocated memory").
`install(ctx)` does the same for PyTorch: it points torch's device allocator
at libckpt's ckpt_hook_malloc / ckpt_hook_free (through torch's pluggable
allocator), and each allocation is registered in `ctx` as it is made and
unregistered as it is freed.  With `address_stable=True` the memory comes from
ckpt_vmm_alloc, so `ctx.restore_at(image)` -- in this process or a fresh one --
brings every allocation back at its address.

torch accepts a new allocator only before the process's first device
allocation, so install() must run first.  The pluggable allocator does not
cache: every tensor allocation reaches the hook, which is what makes the log
exact.  Without `cache` each one costs a hipMalloc (or a mapping) and each
free a wait for the device; with `cache=True` freed blocks are kept for
reuse on their stream, as torch's own caching allocator does, and the log
stays exact (a cached block is unregistered until it is handed out again).
"""
import ctypes

import torch

from . import ckpt as K


def install(ctx, address_stable=False, cache=False):
    """Log torch's device allocations into ctx; returns the allocator object."""
    flags = (K.CKPT_HOOK_ADDRESS_STABLE if address_stable else 0) | (K.CKPT_HOOK_CACHE if cache else 0)
    K._check(K.lib().ckpt_hook_install(ctx.handle, flags), "ckpt_hook_install")
    alloc = torch.cuda.memory.CUDAPluggableAllocator(K.LIB_PATH, "ckpt_hook_malloc", "ckpt_hook_free")
    torch.cuda.memory.change_current_allocator(alloc)
    return alloc


def stats():
    """{"allocs", "frees", "failures"} since install()."""
    v = [ctypes.c_uint64() for _ in range(3)]
    K._check(K.lib().ckpt_hook_stats(*[ctypes.byref(x) for x in v]), "ckpt_hook_stats")
    return {"allocs": v[0].value, "frees": v[1].value, "failures": v[2].value}


def cache_stats():
    """{"blocks", "bytes", "hits"} of the block cache."""
    v = [ctypes.c_uint64() for _ in range(3)]
    K._check(K.lib().ckpt_hook_cache_stats(*[ctypes.byref(x) for x in v]), "ckpt_hook_cache_stats")
    return {"blocks": v[0].value, "bytes": v[1].value, "hits": v[2].value}


def trim():
    """Release every cached block; returns their bytes.  torch.cuda.empty_cache()
    does not reach the hook's cache (torch's pluggable allocator passes only
    allocations and frees), so this is the way to hand the memory back."""
    n = ctypes.c_uint64()
    K._check(K.lib().ckpt_hook_trim(ctypes.byref(n)), "ckpt_hook_trim")
    return n.value
