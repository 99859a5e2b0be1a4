"""ctypes binding of libckpt (include/ckpt.h): argument marshalling only.

Every step of the data path runs in the library's HIP kernels; this module
only converts Python values (ints, torch tensors, streams) to the C ABI and
back.  The raw entry points keep their C names (ckpt_init, ckpt_register,
...); Context / Image / checkpoint_batch are thin conveniences over them.

torch is imported first on purpose: it loads its HIP runtime
(libamdhip64.so.7), and libckpt.so then binds to that same runtime, so torch
tensors and streams are valid in the library.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library shares)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libckpt.so")

# ---- constants (mirror include/ckpt.h) -----------------------------------
CKPT_DEVICE, CKPT_MANAGED = 0, 1
CKPT_FULL, CKPT_INCREMENTAL = 0, 1
CKPT_OK = 0
CKPT_E_INVAL, CKPT_E_NOTFOUND, CKPT_E_NOMEM, CKPT_E_HIP = -1, -2, -3, -4
CKPT_E_MISMATCH, CKPT_E_CORRUPT, CKPT_E_AGAIN, CKPT_E_BUDGET = -5, -6, -7, -8
CKPT_E_ADDR, CKPT_E_IO = -9, -10
CKPT_FILE_BUFFERED = 0x1
CKPT_FILE_DEFLATE = 0x2
CKPT_STREAM_ORDERED = 0x1
CKPT_KEEP_DENSE = 0x2
CKPT_NO_DRAIN = 0x4
CKPT_TIMING = 0x8
CKPT_DRAIN_DIRECT = 0x10
CKPT_GRAPH = 0x20
CKPT_NO_GRAPH = 0x40
CKPT_RESERVE_STAGING = 0x80
CKPT_HOOK_ADDRESS_STABLE = 0x1
CKPT_HOOK_CACHE = 0x2
CKPT_SEC_ALLOCS, CKPT_SEC_CRC, CKPT_SEC_FLAGS, CKPT_SEC_DATA, CKPT_SEC_DIRTY_IDS, CKPT_SEC_DENSE = range(6)
CKPT_SEC_ADDRS = 6
CKPT_REPORT_MAX = 64
CKPT_REQ_CHECKPOINT, CKPT_REQ_RESTORE = 0, 1

STATUS_NAMES = {0: "CKPT_OK", -1: "CKPT_E_INVAL", -2: "CKPT_E_NOTFOUND", -3: "CKPT_E_NOMEM",
                -4: "CKPT_E_HIP", -5: "CKPT_E_MISMATCH", -6: "CKPT_E_CORRUPT", -7: "CKPT_E_AGAIN",
                -8: "CKPT_E_BUDGET", -9: "CKPT_E_ADDR", -10: "CKPT_E_IO"}


class ckpt_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("chunk_bytes", ctypes.c_uint32),
                ("staging_budget", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("block_threads", ctypes.c_uint32), ("waves_per_chunk", ctypes.c_uint32),
                ("wgs_per_cu", ctypes.c_uint32), ("lane_pieces", ctypes.c_uint32),
                ("load_hint", ctypes.c_uint32), ("table_mode", ctypes.c_uint32),
                ("segment_mib", ctypes.c_uint32)]


class ckpt_alloc_rec(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("kind", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("size", ctypes.c_uint64), ("off", ctypes.c_uint64), ("cb", ctypes.c_uint64)]


ALLOC_DTYPE = np.dtype([("id", "<u8"), ("kind", "<u4"), ("pad", "<u4"), ("size", "<u8"),
                        ("off", "<u8"), ("cb", "<u8")])


class ckpt_image_meta(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("chunk_bytes", ctypes.c_uint32),
                ("n_allocs", ctypes.c_uint64), ("n_chunks", ctypes.c_uint64),
                ("data_bytes", ctypes.c_uint64), ("serialized_bytes", ctypes.c_uint64),
                ("n_dirty", ctypes.c_uint64), ("serial", ctypes.c_uint64),
                ("base_serial", ctypes.c_uint64), ("crc_digest", ctypes.c_uint64),
                ("has_dense", ctypes.c_uint32), ("drained", ctypes.c_uint32)]


class ckpt_verify_report(ctypes.Structure):
    _fields_ = [("n_bad", ctypes.c_uint64), ("n_ids", ctypes.c_uint64),
                ("ids", ctypes.c_uint64 * CKPT_REPORT_MAX)]


class ckpt_timing(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("order_ms", "layout_ms", "pack_ms", "select_ms",
                                                "gather_ms", "d2h_ms", "h2d_ms", "scatter_ms",
                                                "total_ms", "pad")] + \
               [("pack_read_bytes", ctypes.c_uint64), ("pack_write_bytes", ctypes.c_uint64),
                ("link_bytes", ctypes.c_uint64)]


class ckpt_server_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("chunk_bytes", ctypes.c_uint32),
                ("staging_budget", ctypes.c_uint64), ("step_bytes", ctypes.c_uint64),
                ("max_active", ctypes.c_uint32), ("aux_threads", ctypes.c_uint32),
                ("block_threads", ctypes.c_uint32), ("lane_pieces", ctypes.c_uint32),
                ("host_budget", ctypes.c_uint64)]


class ckpt_request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("n", ctypes.c_uint32),
                ("ptrs", ctypes.POINTER(ctypes.c_void_p)), ("sizes", ctypes.POINTER(ctypes.c_uint64)),
                ("kinds", ctypes.POINTER(ctypes.c_uint32)), ("image", ctypes.c_void_p)]


class ckpt_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("op", ctypes.c_uint32), ("image", ctypes.c_void_p),
                ("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double),
                ("bytes", ctypes.c_uint64), ("n_bad", ctypes.c_uint64)]


class ckpt_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("bytes", ctypes.c_uint64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("makespan_s", ctypes.c_double), ("gbps", ctypes.c_double),
                ("steps", ctypes.c_uint64), ("max_concurrent", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("host_waits", ctypes.c_uint64), ("host_peak", ctypes.c_uint64),
                ("last_error", ctypes.c_char * 160)]


_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)

# (name, restype, argtypes) of every entry point in include/ckpt.h
SIGNATURES = [
    ("ckpt_init", ctypes.c_int, [ctypes.POINTER(ckpt_config), ctypes.POINTER(_vp)]),
    ("ckpt_destroy", None, [_vp]),
    ("ckpt_register", ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]),
    ("ckpt_unregister", ctypes.c_int, [_vp, _vp]),
    ("ckpt_live_count", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    ("ckpt_checkpoint", ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    ("ckpt_checkpoint_noalloc", ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, ctypes.c_uint64, _vp, _vp,
                                                ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64),
                                                ctypes.POINTER(ctypes.c_uint64)]),
    ("ckpt_restore", ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.c_size_t, ctypes.POINTER(ckpt_verify_report)]),
    ("ckpt_image_info", ctypes.c_int, [_vp, ctypes.POINTER(ckpt_image_meta)]),
    ("ckpt_image_view", ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_size_t)]),
    ("ckpt_image_serialize", ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    ("ckpt_image_load", ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    ("ckpt_image_free", None, [_vp]),
    ("ckpt_image_merge", ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp)]),
    ("ckpt_image_write_file", ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]),
    ("ckpt_image_read_file", ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.POINTER(_vp)]),
    ("ckpt_image_file_info", ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ckpt_image_meta)]),
    ("ckpt_checkpoint_batch", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    ("ckpt_vmm_granularity", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    ("ckpt_vmm_alloc", ctypes.c_int, [_vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_uint64)]),
    ("ckpt_vmm_free", ctypes.c_int, [_vp, _vp]),
    ("ckpt_restore_at", ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.POINTER(_vp), ctypes.POINTER(ckpt_verify_report)]),
    ("ckpt_hook_install", ctypes.c_int, [_vp, ctypes.c_uint32]),
    ("ckpt_hook_malloc", _vp, [ctypes.c_size_t, ctypes.c_int, _vp]),
    ("ckpt_hook_free", None, [_vp, ctypes.c_size_t, ctypes.c_int, _vp]),
    ("ckpt_hook_stats", ctypes.c_int, [ctypes.POINTER(ctypes.c_uint64)] * 3),
    ("ckpt_hook_cache_stats", ctypes.c_int, [ctypes.POINTER(ctypes.c_uint64)] * 3),
    ("ckpt_hook_trim", ctypes.c_int, [ctypes.POINTER(ctypes.c_uint64)]),
    ("ckpt_restore_file_at", ctypes.c_int, [_vp, _vp, ctypes.c_char_p, ctypes.POINTER(_vp),
                                             ctypes.POINTER(ckpt_verify_report), ctypes.POINTER(_vp)]),
    ("ckpt_last_timing", ctypes.c_int, [_vp, ctypes.POINTER(ckpt_timing)]),
    ("ckpt_host_memory", ctypes.c_int, [ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
    ("ckpt_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("ckpt_last_hip_error", ctypes.c_int, []),
    ("ckpt_last_error", ctypes.c_char_p, []),
    ("ckpt_server_create", ctypes.c_int, [ctypes.POINTER(ckpt_server_config), ctypes.POINTER(_vp)]),
    ("ckpt_server_submit", ctypes.c_int, [_vp, ctypes.POINTER(ckpt_request), ctypes.POINTER(ctypes.c_uint64)]),
    ("ckpt_server_poll", ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(ckpt_result)]),
    ("ckpt_server_wait", ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(ckpt_result)]),
    ("ckpt_server_stats", ctypes.c_int, [_vp, ctypes.POINTER(ckpt_stats)]),
    ("ckpt_server_reset_stats", ctypes.c_int, [_vp]),
    ("ckpt_server_destroy", None, [_vp]),
]

_lib = None


def lib():
    """The loaded libckpt.so.  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libckpt.so is not built (%s); run `python -m paper_2008_10596_amd.build`"
                               % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class CkptError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = lib().ckpt_last_error()
        self.detail = msg.decode() if msg else ""
        super().__init__("%s: %s (%s) %s" % (where, STATUS_NAMES.get(status, status),
                                             lib().ckpt_strerror(status).decode(), self.detail))


def _check(rc, where):
    if rc != CKPT_OK:
        raise CkptError(rc, where)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream   # torch.cuda.Stream


def _ptr(x):
    if isinstance(x, torch.Tensor):
        return x.data_ptr()
    return int(x)


def _nbytes(x):
    return x.numel() * x.element_size()


def _np_view(p, nbytes, dtype):
    """Zero-copy numpy view of host memory owned by the library."""
    dt = np.dtype(dtype)
    if not p or nbytes == 0:
        return np.zeros(0, dt)
    buf = (ctypes.c_uint8 * nbytes).from_address(p)
    return np.frombuffer(buf, dtype=dt)


# ---- images ---------------------------------------------------------------

class Image:
    """Owns one ckpt_image; frees it on close() / garbage collection."""

    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle:
            lib().ckpt_image_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        m = ckpt_image_meta()
        _check(lib().ckpt_image_info(self.handle, ctypes.byref(m)), "ckpt_image_info")
        return {f: getattr(m, f) for f, _ in ckpt_image_meta._fields_}

    def view(self, section):
        p, n = _vp(), ctypes.c_size_t()
        _check(lib().ckpt_image_view(self.handle, section, ctypes.byref(p), ctypes.byref(n)), "ckpt_image_view")
        return p.value or 0, n.value

    def _arr(self, section, dtype):
        p, n = self.view(section)
        return _np_view(p, n, dtype)

    # numpy views (valid while the image is open)
    @property
    def allocs(self):
        return self._arr(CKPT_SEC_ALLOCS, ALLOC_DTYPE)

    @property
    def crc(self):
        return self._arr(CKPT_SEC_CRC, np.uint32)

    @property
    def flags(self):
        return self._arr(CKPT_SEC_FLAGS, np.uint8)

    @property
    def data(self):
        return self._arr(CKPT_SEC_DATA, np.uint8)

    @property
    def dirty_ids(self):
        return self._arr(CKPT_SEC_DIRTY_IDS, np.uint64)

    @property
    def addrs(self):
        return self._arr(CKPT_SEC_ADDRS, np.uint64)

    @property
    def dense_ptr(self):
        return self.view(CKPT_SEC_DENSE)

    def serialize(self):
        need = ctypes.c_size_t()
        _check(lib().ckpt_image_serialize(self.handle, None, 0, ctypes.byref(need)), "ckpt_image_serialize")
        buf = (ctypes.c_uint8 * need.value)()
        _check(lib().ckpt_image_serialize(self.handle, buf, need.value, ctypes.byref(need)),
               "ckpt_image_serialize")
        return bytes(buf)

    def write_file(self, path, buffered=False, deflate=False):
        """Write the serialized image to path (O_DIRECT unless buffered; with
        deflate, the compressed container); returns the file size."""
        n = ctypes.c_uint64()
        flags = (CKPT_FILE_BUFFERED if buffered else 0) | (CKPT_FILE_DEFLATE if deflate else 0)
        _check(lib().ckpt_image_write_file(self.handle, os.fsencode(path), flags, ctypes.byref(n)),
               "ckpt_image_write_file")
        return n.value

    @staticmethod
    def read_file(path, ctx=None):
        out = _vp()
        _check(lib().ckpt_image_read_file(ctx.handle if ctx else None, os.fsencode(path), ctypes.byref(out)),
               "ckpt_image_read_file")
        return Image(out.value)

    @staticmethod
    def load(buf, ctx=None):
        b = (ctypes.c_uint8 * len(buf)).from_buffer_copy(buf)
        out = _vp()
        _check(lib().ckpt_image_load(ctx.handle if ctx else None, b, len(buf), ctypes.byref(out)),
               "ckpt_image_load")
        return Image(out.value)


# ---- contexts ---------------------------------------------------------------

class Context:
    def __init__(self, device=0, chunk_bytes=4096, staging_budget=0, flags=0, block_threads=0,
                 waves_per_chunk=0, wgs_per_cu=0, lane_pieces=0, load_hint=0, table_mode=0, segment_mib=0):
        cfg = ckpt_config(device, chunk_bytes, staging_budget, flags, block_threads, waves_per_chunk,
                          wgs_per_cu, lane_pieces, load_hint, table_mode, segment_mib)
        h = _vp()
        _check(lib().ckpt_init(ctypes.byref(cfg), ctypes.byref(h)), "ckpt_init")
        self.handle = h.value
        self.chunk_bytes = chunk_bytes or 4096

    def close(self):
        if self.handle:
            lib().ckpt_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def register(self, ptr, nbytes=None, kind=CKPT_DEVICE):
        if nbytes is None:
            nbytes = _nbytes(ptr)
        out = ctypes.c_uint64()
        _check(lib().ckpt_register(self.handle, _ptr(ptr), nbytes, kind, ctypes.byref(out)), "ckpt_register")
        return out.value

    def unregister(self, ptr):
        _check(lib().ckpt_unregister(self.handle, _ptr(ptr)), "ckpt_unregister")

    def live_count(self):
        n = ctypes.c_size_t()
        _check(lib().ckpt_live_count(self.handle, ctypes.byref(n)), "ckpt_live_count")
        return n.value

    def checkpoint(self, stream=None, mode=CKPT_FULL, base=None):
        out = _vp()
        _check(lib().ckpt_checkpoint(self.handle, _stream_handle(stream), mode,
                                     base.handle if base else None, ctypes.byref(out)), "ckpt_checkpoint")
        return Image(out.value)

    def noalloc_sizes(self):
        """(N, data_bytes) of the live set, from ckpt_checkpoint_noalloc with
        zero capacities (CKPT_E_MISMATCH reports them).  When the live set has
        no chunks, that call is an empty pass of its own."""
        n, d = ctypes.c_uint64(), ctypes.c_uint64()
        rc = lib().ckpt_checkpoint_noalloc(self.handle, None, CKPT_FULL, None, None, 0, None, None, 0,
                                           ctypes.byref(n), ctypes.byref(d))
        if rc not in (CKPT_OK, CKPT_E_MISMATCH):
            raise CkptError(rc, "ckpt_checkpoint_noalloc")
        return n.value, d.value

    def checkpoint_noalloc(self, crc, flags, dense=None, base_crc=None, mode=CKPT_FULL, stream=None,
                           dense_bytes=None, chunk_cap=None):
        """The allocation-free device pass into caller buffers (tensors or
        device addresses): dense image, CRC and flag arrays.  Enqueued on
        `stream`; returns (N, data_bytes).  Capacities default to the
        tensors' sizes."""
        n, d = ctypes.c_uint64(), ctypes.c_uint64()
        if dense_bytes is None:
            dense_bytes = _nbytes(dense) if isinstance(dense, torch.Tensor) else 0
        if chunk_cap is None:
            chunk_cap = min(_nbytes(crc) // 4, _nbytes(flags)) if isinstance(crc, torch.Tensor) else 0
        _check(lib().ckpt_checkpoint_noalloc(self.handle, _stream_handle(stream), mode,
                                             _ptr(base_crc) if base_crc is not None else None,
                                             _ptr(dense) if dense is not None else None, dense_bytes,
                                             _ptr(crc), _ptr(flags), chunk_cap, ctypes.byref(n), ctypes.byref(d)),
               "ckpt_checkpoint_noalloc")
        return n.value, d.value

    def restore(self, image, dsts, delta=None, stream=None, dst_bytes=None, raise_on_corrupt=False):
        """Refill dsts (tensors or device addresses) from image (+ delta).
        Returns (status, report dict); raises on every status but OK/CORRUPT."""
        n = len(dsts)
        ptrs = (_vp * max(n, 1))(*[_ptr(d) for d in dsts])
        if dst_bytes is None and all(isinstance(d, torch.Tensor) for d in dsts):
            dst_bytes = [_nbytes(d) for d in dsts]
        sizes = (ctypes.c_size_t * max(n, 1))(*dst_bytes) if dst_bytes is not None else None
        rep = ckpt_verify_report()
        rc = lib().ckpt_restore(self.handle, _stream_handle(stream), image.handle,
                                delta.handle if delta else None, ptrs, sizes, n, ctypes.byref(rep))
        if rc not in (CKPT_OK, CKPT_E_CORRUPT) or (rc == CKPT_E_CORRUPT and raise_on_corrupt):
            raise CkptError(rc, "ckpt_restore")
        return rc, {"n_bad": rep.n_bad, "ids": [rep.ids[i] for i in range(rep.n_ids)]}

    def vmm_granularity(self):
        g = ctypes.c_size_t()
        _check(lib().ckpt_vmm_granularity(self.handle, ctypes.byref(g)), "ckpt_vmm_granularity")
        return g.value

    def vmm_alloc(self, nbytes, addr=0):
        """Address-stable device memory of the context: returns (address, id)."""
        p, i = _vp(), ctypes.c_uint64()
        _check(lib().ckpt_vmm_alloc(self.handle, nbytes, addr or None, ctypes.byref(p), ctypes.byref(i)),
               "ckpt_vmm_alloc")
        return p.value, i.value

    def vmm_free(self, ptr):
        _check(lib().ckpt_vmm_free(self.handle, _ptr(ptr)), "ckpt_vmm_free")

    def restore_at(self, image, delta=None, stream=None, raise_on_corrupt=False):
        """Restore image at its recorded addresses (re-creating what is gone).
        Returns (status, report dict, addresses)."""
        n = image.info()["n_allocs"]
        out = (_vp * max(n, 1))()
        rep = ckpt_verify_report()
        rc = lib().ckpt_restore_at(self.handle, _stream_handle(stream), image.handle,
                                   delta.handle if delta else None, out, ctypes.byref(rep))
        if rc not in (CKPT_OK, CKPT_E_CORRUPT) or (rc == CKPT_E_CORRUPT and raise_on_corrupt):
            raise CkptError(rc, "ckpt_restore_at")
        return rc, {"n_bad": rep.n_bad, "ids": [rep.ids[i] for i in range(rep.n_ids)]}, \
            [out[k] or 0 for k in range(n)]

    def restore_file_at(self, path, n_allocs=None, stream=None, raise_on_corrupt=False):
        """The restart path: restore the image file at its recorded addresses,
        reserving them before any other device memory of this call.  Returns
        (status, report dict, addresses, Image)."""
        if n_allocs is None:
            n_allocs = file_info(path)["n_allocs"]
        out = (_vp * max(n_allocs, 1))()
        rep = ckpt_verify_report()
        img = _vp()
        rc = lib().ckpt_restore_file_at(self.handle, _stream_handle(stream), os.fsencode(path), out,
                                        ctypes.byref(rep), ctypes.byref(img))
        if rc not in (CKPT_OK, CKPT_E_CORRUPT) or (rc == CKPT_E_CORRUPT and raise_on_corrupt):
            raise CkptError(rc, "ckpt_restore_file_at")
        return rc, {"n_bad": rep.n_bad, "ids": [rep.ids[i] for i in range(rep.n_ids)]}, \
            [out[k] or 0 for k in range(n_allocs)], Image(img.value)

    def timing(self):
        t = ckpt_timing()
        _check(lib().ckpt_last_timing(self.handle, ctypes.byref(t)), "ckpt_last_timing")
        return {f: getattr(t, f) for f, _ in ckpt_timing._fields_ if f != "pad"}


def file_info(path):
    """Metadata of the image in a file (plain or compressed), from its header
    and tables alone."""
    m = ckpt_image_meta()
    _check(lib().ckpt_image_file_info(os.fsencode(path), ctypes.byref(m)), "ckpt_image_file_info")
    return {f: getattr(m, f) for f, _ in ckpt_image_meta._fields_}


def merge(base, *deltas):
    """Fold a chain of incremental images (each taken against the previous
    one, the first against base) into one full image."""
    img = base
    for d in deltas:
        out = _vp()
        _check(lib().ckpt_image_merge(img.handle, d.handle, ctypes.byref(out)), "ckpt_image_merge")
        if img is not base:
            img.close()
        img = Image(out.value)
    return img


def host_memory():
    """(live, cached) pinned bytes of the library's pool (ckpt_host_memory)."""
    live, cached = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().ckpt_host_memory(ctypes.byref(live), ctypes.byref(cached)), "ckpt_host_memory")
    return live.value, cached.value


def checkpoint_batch(ctxs, stream=None):
    n = len(ctxs)
    hs = (_vp * n)(*[c.handle for c in ctxs])
    outs = (_vp * n)()
    _check(lib().ckpt_checkpoint_batch(hs, n, _stream_handle(stream), outs), "ckpt_checkpoint_batch")
    return [Image(outs[i]) for i in range(n)]


# ---- serving -----------------------------------------------------------------

class Server:
    """Continuous-batching server (ckpt_server_*)."""

    def __init__(self, device=0, chunk_bytes=4096, staging_budget=0, step_bytes=0, max_active=0,
                 aux_threads=0, block_threads=0, lane_pieces=0, host_budget=0):
        cfg = ckpt_server_config(device, chunk_bytes, staging_budget, step_bytes, max_active, aux_threads,
                                 block_threads, lane_pieces, host_budget)
        h = _vp()
        _check(lib().ckpt_server_create(ctypes.byref(cfg), ctypes.byref(h)), "ckpt_server_create")
        self.handle = h.value

    def close(self):
        if self.handle:
            lib().ckpt_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, op, bufs, image=None, sizes=None, kinds=None):
        """bufs: tensors or device addresses; returns a ticket."""
        n = len(bufs)
        ptrs = (_vp * max(n, 1))(*[_ptr(b) for b in bufs])
        if sizes is None:
            sizes = [_nbytes(b) for b in bufs]
        sz = (ctypes.c_uint64 * max(n, 1))(*sizes)
        kd = (ctypes.c_uint32 * max(n, 1))(*kinds) if kinds is not None else None
        req = ckpt_request(op, n, ptrs, sz, kd, image.handle if image else None)
        t = ctypes.c_uint64()
        _check(lib().ckpt_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)), "ckpt_server_submit")
        return t.value

    def _result(self, res):
        out = {f: getattr(res, f) for f, _ in ckpt_result._fields_}
        out["image"] = Image(res.image) if res.image else None
        return out

    def poll(self, ticket):
        res = ckpt_result()
        rc = lib().ckpt_server_poll(self.handle, ticket, ctypes.byref(res))
        if rc == CKPT_E_AGAIN:
            return None
        _check(rc, "ckpt_server_poll")
        return self._result(res)

    def wait(self, ticket):
        res = ckpt_result()
        _check(lib().ckpt_server_wait(self.handle, ticket, ctypes.byref(res)), "ckpt_server_wait")
        return self._result(res)

    def stats(self):
        st = ckpt_stats()
        _check(lib().ckpt_server_stats(self.handle, ctypes.byref(st)), "ckpt_server_stats")
        out = {f: getattr(st, f) for f, _ in ckpt_stats._fields_ if f != "pad"}
        out["last_error"] = out["last_error"].decode(errors="replace")
        return out

    def reset_stats(self):
        _check(lib().ckpt_server_reset_stats(self.handle), "ckpt_server_reset_stats")
