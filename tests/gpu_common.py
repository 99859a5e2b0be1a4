"""Helpers shared by the GPU tests: device inputs, host copies for the oracle,
and section-by-section comparison of a library image with the oracle's."""
import numpy as np
import torch

import synth
from oracle import oracle as O
from paper_2008_10596_amd import ckpt as K

FLAG_ZERO, FLAG_DIRTY = 1, 2


_hip = None


def d2h(ptr, nbytes):
    """Copy device memory at a raw address into a new numpy array (hipMemcpy
    through the HIP runtime torch already loaded)."""
    import ctypes
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so.7")
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    out = np.empty(nbytes, np.uint8)
    if nbytes:
        rc = _hip.hipMemcpy(out.ctypes.data, ptr, nbytes, 2)   # hipMemcpyDeviceToHost
        assert rc == 0, "hipMemcpy failed: %d" % rc
    return out


def log(msg):
    print(msg, flush=True)


def host(t):
    return t.detach().cpu().numpy().copy()


def device_bytes(arr):
    """A fresh device uint8 tensor holding numpy bytes."""
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.uint8)).to("cuda")


def random_allocs(sizes, seed, zero=()):
    out = []
    for k, s in enumerate(sizes):
        t = torch.empty(int(s), dtype=torch.uint8, device="cuda")
        if k in zero:
            t.zero_()
        else:
            synth.fill_random_(t, seed * 7919 + k)
        out.append(t)
    return out


def register_all(ctx, tensors, kinds=None):
    return [ctx.register(t, kind=(kinds[k] if kinds else K.CKPT_DEVICE)) for k, t in enumerate(tensors)]


def r16(x):
    return (x + 15) // 16 * 16


def dense_defined(sizes, C, flags):
    """Mask of the dense image's defined bytes: every byte except those of
    ZERO chunks and, for a ZERO tail chunk, its pad (the pack may leave ZERO
    chunks unwritten; their bytes read as zeros by the flags)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    off, cb, data_bytes, N = O.layout(sizes, C)
    keep = np.ones(int(data_bytes), bool)
    z = np.flatnonzero(np.asarray(flags) & FLAG_ZERO)
    if z.size:
        cb = np.asarray(cb, np.int64)
        off = np.asarray(off, np.int64)
        # the allocation of each chunk: the last k with cb[k] <= g (size-0
        # allocations share their successor's cb and come before it)
        k = np.searchsorted(cb, z, side="right") - 1
        start = (z - cb[k]) * C
        end = np.minimum(start + C, sizes[k])
        end = np.where(end == sizes[k], (end + 15) // 16 * 16, end)   # a tail keeps its pad
        for lo, hi in zip(off[k] + start, off[k] + end):
            keep[lo:hi] = False
    return keep


def assert_dense(got, want, sizes, C, flags):
    """The dense image equals the oracle's on every defined byte."""
    got, want = np.asarray(got), np.asarray(want)
    assert got.size == want.size
    keep = dense_defined(sizes, C, flags)
    diff = np.flatnonzero((got != want) & keep)
    assert diff.size == 0, "dense image differs at bytes %s" % diff[:10]


def check_full(img, ref, tensors, C, ids=None):
    """Bit-exact: allocation table, CRC, FLAGS, serialized DATA."""
    info = img.info()
    sizes = [t.numel() for t in tensors]
    off, cb, data_bytes, N = O.layout(sizes, C)
    assert info["chunk_bytes"] == C
    assert info["n_allocs"] == len(tensors)
    assert info["n_chunks"] == N == ref["n_chunks"]
    assert info["data_bytes"] == data_bytes
    al = img.allocs
    assert list(al["size"]) == sizes
    assert list(al["off"]) == [int(x) for x in off]
    assert list(al["cb"]) == [int(x) for x in cb]
    if ids is not None:
        assert list(al["id"]) == list(ids)
    crc, flags = img.crc, img.flags
    bad = np.flatnonzero(crc != ref["crc"])
    assert bad.size == 0, "CRC differs at chunks %s" % bad[:10]
    bad = np.flatnonzero(flags != ref["flags"])
    assert bad.size == 0, "FLAGS differ at chunks %s: got %s want %s" % (bad[:10], flags[bad[:10]], ref["flags"][bad[:10]])
    assert info["serialized_bytes"] == ref["serialized_bytes"]
    data = img.data
    if ref["serialized"] is not None:
        diff = np.flatnonzero(data != ref["serialized"])
        assert diff.size == 0, "DATA differs at bytes %s" % diff[:10]


def check_restored(dsts, srcs):
    for k, (d, s) in enumerate(zip(dsts, srcs)):
        assert torch.equal(d, s), "allocation %d differs after restore" % k


def _hipapi():
    import ctypes
    global _hip
    if _hip is None:
        d2h(0, 0)
    return _hip


def managed_alloc(nbytes):
    """hipMallocManaged (global attach); returns the address."""
    import ctypes
    hip = _hipapi()
    hip.hipMallocManaged.restype = ctypes.c_int
    hip.hipMallocManaged.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.c_uint]
    p = ctypes.c_void_p()
    rc = hip.hipMallocManaged(ctypes.byref(p), max(nbytes, 1), 1)   # hipMemAttachGlobal
    assert rc == 0, "hipMallocManaged failed: %d" % rc
    return p.value


def managed_free(ptr):
    import ctypes
    hip = _hipapi()
    hip.hipFree.restype = ctypes.c_int
    hip.hipFree.argtypes = [ctypes.c_void_p]
    assert hip.hipFree(ptr) == 0


def h2d(ptr, arr):
    import ctypes
    hip = _hipapi()
    a = np.ascontiguousarray(arr, dtype=np.uint8)
    if a.size:
        rc = hip.hipMemcpy(ptr, a.ctypes.data, a.size, 1)   # hipMemcpyHostToDevice
        assert rc == 0, "hipMemcpy failed: %d" % rc


def prefetch_to_host(ptr, nbytes):
    """Move managed pages host-side (hipCpuDeviceId); returns False when the
    device does not support it."""
    import ctypes
    hip = _hipapi()
    hip.hipMemPrefetchAsync.restype = ctypes.c_int
    hip.hipMemPrefetchAsync.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    hip.hipDeviceSynchronize.restype = ctypes.c_int
    rc = hip.hipMemPrefetchAsync(ptr, nbytes, -1, None)
    hip.hipDeviceSynchronize()
    return rc == 0


def hip_malloc(nbytes):
    """Plain hipMalloc; returns the address."""
    import ctypes
    hip = _hipapi()
    hip.hipMalloc.restype = ctypes.c_int
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    p = ctypes.c_void_p()
    rc = hip.hipMalloc(ctypes.byref(p), max(nbytes, 1))
    assert rc == 0, "hipMalloc failed: %d" % rc
    return p.value


def hip_free(ptr):
    managed_free(ptr)
