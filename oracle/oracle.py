"""ctypes wrapper around the C oracle (ckpt_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  The product package never
imports it, and the oracle shares no code with the HIP path.

Every function takes host numpy arrays and returns host numpy arrays; see
ckpt_oracle.c for the rules each one follows and the passages of the paper
they restate.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ckpt_oracle.c")
# A test may point this at another build of the oracle source (the mutation
# tests do, to show that the pins catch planted mistakes).
LIB = os.environ.get("CKPT_ORACLE_LIB") or os.path.join(HERE, "libckpt_oracle.so")

FLAG_ZERO = 1
FLAG_DIRTY = 2
MAX_REPORT = 64

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u8pp = ctypes.POINTER(_u8p)


def build(out=LIB, src=SRC, extra=()):
    """Compile the oracle with gcc (plain -O2, no SIMD intrinsics)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-pthread", *extra, "-o", out, src]
    subprocess.run(cmd, check=True)
    return out


def load(path=LIB):
    """Load (building first if absent) and declare the oracle's C functions."""
    if not os.path.exists(path):
        build(path)
    lib = ctypes.CDLL(path)
    lib.oracle_crc32c.restype = ctypes.c_uint32
    lib.oracle_crc32c.argtypes = [_u8p, ctypes.c_size_t]
    lib.oracle_crc32c_bitwise.restype = ctypes.c_uint32
    lib.oracle_crc32c_bitwise.argtypes = [_u8p, ctypes.c_size_t]
    lib.oracle_crc32c_table.restype = None
    lib.oracle_crc32c_table.argtypes = [_u32p]
    lib.oracle_layout.restype = ctypes.c_int
    lib.oracle_layout.argtypes = [ctypes.c_size_t, _u64p, ctypes.c_uint64, _u64p, _u64p, _u64p, _u64p]
    lib.oracle_checkpoint.restype = ctypes.c_int
    lib.oracle_checkpoint.argtypes = [ctypes.c_size_t, _u8pp, _u64p, ctypes.c_uint64, _u32p,
                                      ctypes.c_int, _u8p, _u32p, _u8p, _u8p, _u64p]
    lib.oracle_delta.restype = ctypes.c_int
    lib.oracle_delta.argtypes = [ctypes.c_size_t, _u8pp, _u64p, ctypes.c_uint64, _u32p,
                                 ctypes.c_int, _u32p, _u8p, _u64p, _u64p, _u8p, _u64p]
    lib.oracle_restore.restype = ctypes.c_int
    lib.oracle_restore.argtypes = [ctypes.c_size_t, _u64p, ctypes.c_uint64, _u32p, _u8p,
                                   _u8p, ctypes.c_uint64, _u8pp, _u64p, _u64p, _u64p]
    lib.oracle_restore_delta.restype = ctypes.c_int
    lib.oracle_restore_delta.argtypes = [ctypes.c_size_t, _u64p, ctypes.c_uint64, _u32p, _u8p,
                                         _u64p, ctypes.c_uint64, _u8p, ctypes.c_uint64, _u8pp,
                                         _u64p, _u64p, _u64p]
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _bytes(a):
    a = np.ascontiguousarray(np.frombuffer(bytes(a), np.uint8) if isinstance(a, (bytes, bytearray)) else a)
    assert a.dtype == np.uint8
    return a


def _garbage(n, dtype):
    """Output buffer pre-filled with a non-zero pattern, so that a byte the
    oracle forgets to write shows up in the tests instead of reading as 0."""
    return np.full(max(n, 1), 0xA5, dtype)


def _ptr_array(arrs):
    ptrs = (_u8p * max(1, len(arrs)))()
    for i, a in enumerate(arrs):
        ptrs[i] = a.ctypes.data_as(_u8p)
    return ptrs


def crc32c(data):
    a = _bytes(data)
    return int(lib().oracle_crc32c(_p(a, _u8p), a.size))


def crc32c_bitwise_c(data):
    a = _bytes(data)
    return int(lib().oracle_crc32c_bitwise(_p(a, _u8p), a.size))


def crc32c_table():
    t = np.zeros(256, np.uint32)
    lib().oracle_crc32c_table(_p(t, _u32p))
    return t


def layout(sizes, C):
    """(off[n], cb[n], data_bytes, N) for the dense layout and chunk grid."""
    sizes = np.ascontiguousarray(sizes, dtype=np.uint64)
    n = sizes.size
    off = np.zeros(max(n, 1), np.uint64)
    cb = np.zeros(max(n, 1), np.uint64)
    db = np.zeros(1, np.uint64)
    N = np.zeros(1, np.uint64)
    rc = lib().oracle_layout(n, _p(sizes, _u64p), C, _p(off, _u64p), _p(cb, _u64p),
                             _p(db, _u64p), _p(N, _u64p))
    if rc != 0:
        raise ValueError("chunk size must be a positive multiple of 16")
    return off[:n], cb[:n], int(db[0]), int(N[0])


def checkpoint(allocs, C, base_crc=None, threads=1, dense=True, serialized=True):
    """Full checkpoint of host copies `allocs` (list of uint8 arrays)."""
    allocs = [_bytes(a) for a in allocs]
    sizes = np.array([a.size for a in allocs], np.uint64)
    _, _, data_bytes, N = layout(sizes, C)
    crc = _garbage(N, np.uint32)
    flags = _garbage(N, np.uint8)
    dn = _garbage(data_bytes, np.uint8) if dense else None
    ser = _garbage(data_bytes, np.uint8) if serialized else None
    ser_bytes = np.zeros(1, np.uint64)
    if base_crc is not None:
        base_crc = np.ascontiguousarray(base_crc, dtype=np.uint32)
        assert base_crc.size == N
    rc = lib().oracle_checkpoint(len(allocs), _ptr_array(allocs), _p(sizes, _u64p), C,
                                 _p(base_crc, _u32p), threads, _p(dn, _u8p), _p(crc, _u32p),
                                 _p(flags, _u8p), _p(ser, _u8p), _p(ser_bytes, _u64p))
    if rc != 0:
        raise RuntimeError("oracle_checkpoint failed: %d" % rc)
    sb = int(ser_bytes[0])
    return {
        "crc": crc[:N], "flags": flags[:N],
        "dense": dn[:data_bytes] if dense else None,
        "serialized": ser[:sb] if serialized else None,
        "serialized_bytes": sb, "data_bytes": data_bytes, "n_chunks": N,
    }


def delta(allocs, C, base_crc, threads=1):
    """Incremental checkpoint of `allocs` against base_crc."""
    allocs = [_bytes(a) for a in allocs]
    sizes = np.array([a.size for a in allocs], np.uint64)
    _, _, data_bytes, N = layout(sizes, C)
    base_crc = np.ascontiguousarray(base_crc, dtype=np.uint32)
    assert base_crc.size == N
    crc = _garbage(N, np.uint32)
    flags = _garbage(N, np.uint8)
    ids = _garbage(N, np.uint64)
    nd = np.zeros(1, np.uint64)
    out = _garbage(data_bytes, np.uint8)
    ob = np.zeros(1, np.uint64)
    rc = lib().oracle_delta(len(allocs), _ptr_array(allocs), _p(sizes, _u64p), C,
                            _p(base_crc, _u32p), threads, _p(crc, _u32p), _p(flags, _u8p),
                            _p(ids, _u64p), _p(nd, _u64p), _p(out, _u8p), _p(ob, _u64p))
    if rc != 0:
        raise RuntimeError("oracle_delta failed: %d" % rc)
    return {"crc": crc[:N], "flags": flags[:N], "dirty_ids": ids[:int(nd[0])],
            "delta": out[:int(ob[0])]}


def restore(sizes, C, crc, flags, ser):
    """Full restore into fresh host buffers; returns (bufs, bad_count, bad_ids)."""
    sizes = np.ascontiguousarray(sizes, dtype=np.uint64)
    bufs = [np.full(int(s), 0xA5, np.uint8) for s in sizes]   # not zero: restore must write
    crc = np.ascontiguousarray(crc, dtype=np.uint32)
    flags = np.ascontiguousarray(flags, dtype=np.uint8)
    ser_len = len(ser)
    ser = _bytes(ser) if ser_len else np.zeros(1, np.uint8)
    cnt, ids, nids = np.zeros(1, np.uint64), np.zeros(MAX_REPORT, np.uint64), np.zeros(1, np.uint64)
    rc = lib().oracle_restore(sizes.size, _p(sizes, _u64p), C, _p(crc, _u32p), _p(flags, _u8p),
                              _p(ser, _u8p), ser_len,
                              _ptr_array(bufs), _p(cnt, _u64p), _p(ids, _u64p), _p(nids, _u64p))
    if rc < 0:
        raise ValueError("serialized data too short for the flags")
    return bufs, int(cnt[0]), ids[:int(nids[0])]


def restore_delta(bufs, sizes, C, crc, flags, dirty_ids, delta_data):
    """Overlay a delta onto already-restored host buffers; (bad_count, bad_ids)."""
    sizes = np.ascontiguousarray(sizes, dtype=np.uint64)
    crc = np.ascontiguousarray(crc, dtype=np.uint32)
    flags = np.ascontiguousarray(flags, dtype=np.uint8)
    ids_in = np.ascontiguousarray(dirty_ids, dtype=np.uint64)
    n_ids = ids_in.size
    if n_ids == 0:
        ids_in = np.zeros(1, np.uint64)
    dd = _bytes(delta_data) if len(delta_data) else np.zeros(1, np.uint8)
    cnt, ids, nids = np.zeros(1, np.uint64), np.zeros(MAX_REPORT, np.uint64), np.zeros(1, np.uint64)
    rc = lib().oracle_restore_delta(sizes.size, _p(sizes, _u64p), C, _p(crc, _u32p),
                                    _p(flags, _u8p), _p(ids_in, _u64p), n_ids, _p(dd, _u8p), len(delta_data), _ptr_array(bufs),
                                    _p(cnt, _u64p), _p(ids, _u64p), _p(nids, _u64p))
    if rc < 0:
        raise ValueError("delta ids or data inconsistent with the flags")
    return int(cnt[0]), ids[:int(nids[0])]


def delta_by_id(allocs, ids, kinds, C, base_ids, base_kinds, base_sizes, base_crc):
    """Incremental checkpoint of `allocs` (registration ids `ids`, kinds
    `kinds`) against a base whose allocation table may differ.

    The paper fixes no incremental scheme; the reading here: a chunk is
    compared with the same chunk of the base allocation that has the same
    registration id, size and kind, and every chunk of an allocation without
    such a base allocation is DIRTY.  Allocations of the base that are gone
    play no part.  CRC and ZERO come from the full checkpoint; DIRTY, the
    dirty ids and the delta data follow chunk by chunk (plain loops: small
    inputs only)."""
    allocs = [_bytes(a) for a in allocs]
    sizes = [int(a.size) for a in allocs]
    full = checkpoint(allocs, C, dense=False, serialized=False)
    _, cb, _, N = layout(sizes, C)
    _, bcb, _, _ = layout([int(s) for s in base_sizes], C)
    base_crc = np.ascontiguousarray(base_crc, dtype=np.uint32)
    base_row = {int(i): j for j, i in enumerate(base_ids)}
    flags = (full["flags"] & FLAG_ZERO).astype(np.uint8)
    out = []
    for k, a in enumerate(allocs):
        j = base_row.get(int(ids[k]))
        match = (j is not None and int(base_sizes[j]) == sizes[k] and int(base_kinds[j]) == int(kinds[k]))
        for c in range((sizes[k] + C - 1) // C):
            g = int(cb[k]) + c
            if match and full["crc"][g] == base_crc[int(bcb[j]) + c]:
                continue
            flags[g] |= FLAG_DIRTY
            if not flags[g] & FLAG_ZERO:
                piece = a[c * C:min(sizes[k], (c + 1) * C)]
                out.append(piece)
                out.append(np.zeros((-piece.size) % 16, np.uint8))
    data = np.concatenate(out) if out else np.zeros(0, np.uint8)
    return {"crc": full["crc"], "flags": flags, "dirty_ids": np.nonzero(flags & FLAG_DIRTY)[0].astype(np.uint64),
            "delta": data}
