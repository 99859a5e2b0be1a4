"""Images to files and back: the file holds exactly the serialized bytes, a
read image equals the written one section by section, and restoring from it
gives the original memory."""
import os
import zlib

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2008_10596_amd import ckpt as K
from tests.gpu_common import check_restored, host, log, random_allocs

pytestmark = pytest.mark.gpu

C = 4096


@pytest.mark.parametrize("buffered", [False, True])
@pytest.mark.parametrize("sizes", [[5000, 3 * C, 1, 0], [150 << 20, 40 << 20, 777]])
def test_write_read_file_roundtrip(tmp_path, sizes, buffered):
    log("sink sizes=%s buffered=%s" % (sizes, buffered))
    tensors = random_allocs(sizes, seed=31, zero=(1,))
    ctx = K.Context(chunk_bytes=C)
    for t in tensors:
        ctx.register(t)
    img = ctx.checkpoint()
    path = str(tmp_path / "img.ckpt")
    n = img.write_file(path, buffered=buffered)
    blob = img.serialize()
    assert n == len(blob) == os.path.getsize(path)
    assert not os.path.exists(path + ".partial")
    with open(path, "rb") as f:
        assert f.read() == blob
    back = K.Image.read_file(path, ctx)
    for key in ("allocs", "crc", "flags", "data", "addrs"):
        assert np.array_equal(getattr(back, key), getattr(img, key)), key
    if sum(sizes) < (1 << 20):
        ref = O.checkpoint([host(t) for t in tensors], C)
        assert np.array_equal(back.crc, ref["crc"]) and np.array_equal(back.data, ref["serialized"])
    dsts = [torch.empty_like(t) for t in tensors]
    rc, _ = ctx.restore(back, dsts)
    assert rc == K.CKPT_OK
    check_restored(dsts, tensors)
    for im in (img, back):
        im.close()
    ctx.close()


def test_file_errors(tmp_path):
    tensors = random_allocs([3 * C], seed=32)
    ctx = K.Context(chunk_bytes=C)
    ctx.register(tensors[0])
    img = ctx.checkpoint()
    with pytest.raises(K.CkptError) as e:
        img.write_file(str(tmp_path / "no" / "such" / "dir" / "x.ckpt"))
    assert e.value.status == K.CKPT_E_IO
    with pytest.raises(K.CkptError) as e:
        K.Image.read_file(str(tmp_path / "missing.ckpt"), ctx)
    assert e.value.status == K.CKPT_E_NOTFOUND
    # a truncated file is refused by the loader
    path = str(tmp_path / "t.ckpt")
    img.write_file(path)
    with open(path, "r+b") as f:
        f.truncate(os.path.getsize(path) - 1)
    with pytest.raises(K.CkptError) as e:
        K.Image.read_file(path, ctx)
    assert e.value.status == K.CKPT_E_INVAL
    # an image kept on the device only has nothing to write
    nd = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN)
    nd.register(tensors[0])
    dimg = nd.checkpoint()
    with pytest.raises(K.CkptError) as e:
        dimg.write_file(str(tmp_path / "d.ckpt"))
    assert e.value.status == K.CKPT_E_INVAL
    for im in (img, dimg):
        im.close()
    nd.close()
    ctx.close()


def join_planes(piece, w):
    """Inverse of the byte-plane split: plane j holds byte j of every w-byte
    element; trailing bytes follow as they are."""
    m = len(piece) // w
    a = np.frombuffer(piece, np.uint8)
    return a[:w * m].reshape(w, m).T.reshape(-1).tobytes() + piece[w * m:]


def read_container(path):
    """The compressed container read with Python's zlib, following the
    documented layout: returns (head + DATA, (raw, element width) per block)."""
    with open(path, "rb") as f:
        b = f.read()
    assert b[:8] == b"CKPTZIP1"
    version, block = int.from_bytes(b[8:12], "little"), int.from_bytes(b[12:16], "little")
    head_bytes, data_bytes, nb = (int.from_bytes(b[16 + 8 * i:24 + 8 * i], "little") for i in range(3))
    assert version == 1 and nb == -(-data_bytes // block)
    table = [int.from_bytes(b[40 + 8 * i:48 + 8 * i], "little") for i in range(nb)]
    pos = 40 + 8 * nb
    out = bytearray(b[pos:pos + head_bytes])
    pos += head_bytes
    raws = []
    for i, t in enumerate(table):
        raw, code, n = bool(t >> 63), (t >> 61) & 3, t & ((1 << 61) - 1)
        w = (1, 2, 4)[code]
        chunk = b[pos:pos + n]
        piece = chunk if raw else zlib.decompress(chunk)
        assert len(piece) == min(block, data_bytes - i * block)
        out += join_planes(piece, w) if w > 1 else piece
        raws.append((raw, w))
        pos += n
    assert pos == len(b)
    return bytes(out), raws


def compressible_allocs(sizes, seed, dtype=torch.bfloat16):
    """Values drawn from N(0, 1) in dtype (model-weight-like bytes), as uint8 views."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    w = torch.empty(0, dtype=dtype).element_size()
    out = []
    for s in sizes:
        t = torch.randn((s + w - 1) // w, generator=g, device="cuda").to(dtype)
        out.append(t.view(torch.uint8)[:s].clone())
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("kind", ["random", "bf16", "f32"])
def test_deflate_container_roundtrip(tmp_path, kind):
    """The compressed file holds the serialized image block by block (checked
    with an independent zlib reader), reads back section by section, and
    restores the original memory.  Random data stays raw; bf16 data shrinks."""
    sizes = [9 << 20, 3 << 20, 5000, 1, 0, 4096]
    log("deflate container kind=%s" % kind)
    if kind == "random":
        tensors = random_allocs(sizes, seed=33, zero=(1,))
    else:
        tensors = compressible_allocs(sizes, seed=34, dtype=torch.bfloat16 if kind == "bf16" else torch.float32)
    ctx = K.Context(chunk_bytes=C)
    for t in tensors:
        ctx.register(t)
    img = ctx.checkpoint()
    path = str(tmp_path / "img.ckptz")
    n = img.write_file(path, deflate=True)
    assert n == os.path.getsize(path) and not os.path.exists(path + ".partial")
    blob, forms = read_container(path)
    assert blob == img.serialize()
    ser = img.info()["serialized_bytes"]
    assert len(forms) == -(-ser // (4 << 20)) and len(forms) >= 3
    if kind == "random":
        assert all(raw for raw, _ in forms)
    else:
        # 2- or 4-byte values: that many byte planes, entropy-coded
        width = 2 if kind == "bf16" else 4
        assert all(not raw and w == width for raw, w in forms[:-1]) and n < 0.9 * len(blob)
    back = K.Image.read_file(path, ctx)
    for key in ("allocs", "crc", "flags", "data", "addrs"):
        assert np.array_equal(getattr(back, key), getattr(img, key)), key
    ref = O.checkpoint([host(t) for t in tensors], C)
    assert np.array_equal(back.crc, ref["crc"]) and np.array_equal(back.data, ref["serialized"])
    dsts = [torch.empty_like(t) for t in tensors]
    rc, _ = ctx.restore(back, dsts)
    assert rc == K.CKPT_OK
    check_restored(dsts, tensors)
    for im in (img, back):
        im.close()
    ctx.close()


def test_deflate_container_damage_is_refused(tmp_path):
    tensors = compressible_allocs([6 << 20], seed=35)
    ctx = K.Context(chunk_bytes=C)
    ctx.register(tensors[0])
    img = ctx.checkpoint()
    path = str(tmp_path / "img.ckptz")
    n = img.write_file(path, deflate=True)
    # a flipped byte in the middle of the last compressed block
    with open(path, "r+b") as f:
        f.seek(n - 100)
        x = f.read(1)
        f.seek(n - 100)
        f.write(bytes([x[0] ^ 0x40]))
    with pytest.raises(K.CkptError) as e:
        K.Image.read_file(path, ctx)
    assert e.value.status == K.CKPT_E_INVAL
    # and a file cut short
    img.write_file(path, deflate=True)
    with open(path, "r+b") as f:
        f.truncate(n - 1)
    with pytest.raises(K.CkptError) as e:
        K.Image.read_file(path, ctx)
    assert e.value.status == K.CKPT_E_INVAL
    img.close()
    ctx.close()
