"""Child process of the restart test (run as `python -m tests.restart_child`).

  save PATH [deflate]
                make address-stable allocations with seeded contents in a
                fresh process, checkpoint them, write the serialized image to
                PATH (the compressed container with "deflate") and print the
                addresses and ids as JSON;
  restore PATH  in another fresh process, restore the image file at the
                addresses it was taken from (ranges reserved first), check the
                bytes there, take an incremental checkpoint against the loaded
                image, and print the results as JSON.

Each side regenerates the contents from the same seed, so no data passes
between the processes except the image file.
"""
import json
import sys

import numpy as np

from paper_2008_10596_amd import ckpt as K
from tests.gpu_common import d2h, h2d

C = 4096
SIZES = [1 << 20, 5000, 3 * 4096 + 17, 64, 2 << 20]
ZERO = (3,)
SEED = 12701


def contents():
    rng = np.random.default_rng(SEED)
    out = []
    for k, s in enumerate(SIZES):
        a = rng.integers(0, 256, s, dtype=np.uint8)
        if k in ZERO:
            a[:] = 0
        out.append(a)
    return out


def save(path, deflate=False):
    data = contents()
    ctx = K.Context(chunk_bytes=C)
    addrs, ids = [], []
    for a in data:
        p, i = ctx.vmm_alloc(a.size)
        h2d(p, a)
        addrs.append(p)
        ids.append(i)
    img = ctx.checkpoint()
    img.write_file(path, deflate=deflate)
    print(json.dumps({"addrs": addrs, "ids": ids}), flush=True)


def restore(path):
    data = contents()
    ctx = K.Context(chunk_bytes=C)
    # the restart path: the address ranges come first, before any other
    # device or pinned memory of this process
    rc, rep, addrs, img = ctx.restore_file_at(path)
    same = [bool(np.array_equal(d2h(p, a.size), a)) for p, a in zip(addrs, data)]
    ids = [int(x) for x in img.allocs["id"]]
    # the restored context keeps the image's ids, so it can continue incrementally
    delta = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=img)
    clean = [int(x) for x in delta.dirty_ids]
    h2d(addrs[0] + 2 * C, np.full(10, 7, np.uint8))
    delta2 = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=img)
    dirty = [int(x) for x in delta2.dirty_ids]
    print(json.dumps({"rc": rc, "n_bad": rep["n_bad"], "addrs": addrs, "same": same, "ids": ids,
                      "clean": clean, "dirty": dirty}), flush=True)


if __name__ == "__main__":
    if sys.argv[1] == "save":
        save(sys.argv[2], deflate=len(sys.argv) > 3 and sys.argv[3] == "deflate")
    else:
        restore(sys.argv[2])
