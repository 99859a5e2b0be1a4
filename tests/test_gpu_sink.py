"""Images to files and back: the file holds exactly the serialized bytes, a
read image equals the written one section by section, and restoring from it
gives the original memory."""
import os

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
