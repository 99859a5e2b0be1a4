"""Image files are untrusted input: damaged plain files and compressed
containers must be refused with a status, never crash the process.  Runs on
the CPU: a file whose header and tables pass is refused later, when the
pinned buffer for its DATA cannot be had without a device."""
import ctypes
import struct
import zlib

import numpy as np
import pytest

from oracle import oracle as O

MASK = (1 << 64) - 1


def _digest(crc_bytes):
    """FNV-1a over the CRC section's little-endian 64-bit words (the last
    one zero-padded): the image header's check of that section."""
    h = 0xcbf29ce484222325
    for i in range(0, len(crc_bytes), 8):
        w = int.from_bytes(crc_bytes[i:i + 8].ljust(8, b"\0"), "little")
        h = ((h ^ w) * 0x100000001b3) & MASK
    return h


def image_bytes(sizes, C=4096, seed=1):
    """A serialized full image (version 2) of random allocations, built from
    the documented layout with the oracle's CRC."""
    rng = np.random.default_rng(seed)
    allocs = [rng.integers(0, 256, s, dtype=np.uint8) for s in sizes]
    ref = O.checkpoint(allocs, C)
    crc, flags, data = ref["crc"], ref["flags"], ref["serialized"]
    n, N = len(sizes), len(crc)
    rows, off, cb = b"", 0, 0
    for k, s in enumerate(sizes):
        rows += struct.pack("<QIIQQQ", k + 1, 0, 0, s, off, cb)
        off += (s + 15) // 16 * 16
        cb += -(-s // C)
    hdr = b"CKPTIMG1" + struct.pack("<IIII", 2, 0, C, 16)
    hdr += struct.pack("<8Q", n, N, off, len(data), 0, 7, 0, _digest(crc.tobytes()))
    addrs = b"".join(struct.pack("<Q", 0x7000_0000_0000 + 0x100000 * k) for k in range(n))
    flags_b = flags.tobytes() + bytes((-N) % 8)
    return hdr + rows + addrs + crc.tobytes() + flags_b + data.tobytes(), len(data)


def container(img, data_bytes, block=4096):
    """The compressed container around a serialized image: DATA in blocks,
    alternately deflated and stored raw."""
    head, data = img[:len(img) - data_bytes], img[len(img) - data_bytes:]
    blocks, table = b"", []
    for i in range(0, len(data), block):
        piece = data[i:i + block]
        z = zlib.compress(piece, 1)
        if (i // block) % 2 == 0 and len(z) < len(piece):
            table.append(len(z))
            blocks += z
        else:
            table.append((1 << 63) | len(piece))
            blocks += piece
    out = b"CKPTZIP1" + struct.pack("<II", 1, block) + struct.pack("<QQQ", len(head), len(data), len(table))
    return out + b"".join(struct.pack("<Q", t) for t in table) + head + blocks


@pytest.fixture(scope="module")
def lib():
    from paper_2008_10596_amd import ckpt
    return ckpt


def _statuses(ck, path):
    out = ctypes.c_void_p()
    m = ck.ckpt_image_meta()
    a = ck.lib().ckpt_image_read_file(None, str(path).encode(), ctypes.byref(out))
    b = ck.lib().ckpt_image_file_info(str(path).encode(), ctypes.byref(m))
    if a == ck.CKPT_OK:   # only where a device gives the pinned buffer
        ck.lib().ckpt_image_free(out)
    return a, b


def test_valid_files_parse(lib, tmp_path):
    """The hand-built files pass every check that needs no device."""
    img, nd = image_bytes([5000, 1, 4096, 70000])
    for name, blob in (("plain", img), ("zip", container(img, nd))):
        p = tmp_path / name
        p.write_bytes(blob)
        m = lib.ckpt_image_meta()
        assert lib.lib().ckpt_image_file_info(str(p).encode(), ctypes.byref(m)) == lib.CKPT_OK, name
        assert (m.n_allocs, m.serialized_bytes, m.serial) == (4, nd, 7)


@pytest.mark.parametrize("kind", ["plain", "zip"])
def test_damaged_files_are_refused(lib, tmp_path, kind):
    img, nd = image_bytes([5000, 1, 4096, 70000, 33])
    base = img if kind == "plain" else container(img, nd)
    head_len = len(base) - (nd if kind == "plain" else 0)
    rng = np.random.default_rng(7 if kind == "plain" else 8)
    p = tmp_path / "f.img"
    # with no device a file that passes its checks fails for want of pinned memory
    allowed = {lib.CKPT_OK, lib.CKPT_E_INVAL, lib.CKPT_E_NOMEM, lib.CKPT_E_HIP, lib.CKPT_E_IO}
    seen = set()
    for trial in range(300):
        b = bytearray(base)
        what = trial % 4
        if what == 0:      # flip bytes in the header and tables
            for _ in range(int(rng.integers(1, 4))):
                i = int(rng.integers(0, min(head_len, len(b))))
                b[i] ^= int(rng.integers(1, 256))
        elif what == 1:    # cut the file
            b = b[:int(rng.integers(0, len(b)))]
        elif what == 2:    # extend it
            b += bytes(rng.integers(0, 256, int(rng.integers(1, 64)), dtype=np.uint8))
        else:              # overwrite one 8-byte field with an extreme value
            i = int(rng.integers(0, max(1, min(head_len, len(b)) - 8)))
            extremes = (0, 1, MASK, 1 << 62, 1 << 63, 0xFFFFFFFF)
            b[i:i + 8] = struct.pack("<Q", extremes[int(rng.integers(0, len(extremes)))])
        p.write_bytes(bytes(b))
        a, f = _statuses(lib, p)
        assert a in allowed and f in allowed, (trial, a, f)
        seen.add(a)
    assert lib.CKPT_E_INVAL in seen
