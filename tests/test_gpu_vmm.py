"""Address-stable memory and restore at the original addresses.

The paper restores every allocation at the address the application saw
(Sec. 3.1, Sec. 3.2 "restoring the CUDA library-allocated regions"); here HIP
virtual memory management reserves those addresses explicitly.  The images are
checked against the oracle like any other (the address section aside), the
restored bytes against the bytes written, and the restart across two fresh
processes against the contents regenerated from the seed.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2008_10596_amd import ckpt as K
from tests.gpu_common import d2h, h2d, hip_free, hip_malloc, log, managed_alloc, managed_free

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C = 4096


def seeded(sizes, seed, zero=()):
    rng = np.random.default_rng(seed)
    out = []
    for k, s in enumerate(sizes):
        a = rng.integers(0, 256, s, dtype=np.uint8)
        if k in zero:
            a[:] = 0
        out.append(a)
    return out


def check_image(img, data):
    ref = O.checkpoint(data, C)
    assert np.array_equal(img.crc, ref["crc"])
    assert np.array_equal(img.flags, ref["flags"])
    assert np.array_equal(img.data, ref["serialized"])


def test_vmm_alloc_and_free():
    ctx = K.Context(chunk_bytes=C)
    g = ctx.vmm_granularity()
    assert g >= 4096 and g & (g - 1) == 0
    sizes = [1, 4096, 5000, 3 * g + 17]
    ptrs = []
    for s in sizes:
        p, i = ctx.vmm_alloc(s)
        assert p % g == 0
        ptrs.append(p)
    assert ctx.live_count() == len(sizes)
    data = seeded(sizes, 1)
    for p, a in zip(ptrs, data):
        h2d(p, a)
    for p, a in zip(ptrs, data):
        assert np.array_equal(d2h(p, a.size), a)
    # the context owns this memory: unregister refuses it
    with pytest.raises(K.CkptError) as e:
        ctx.unregister(ptrs[0])
    assert e.value.status == K.CKPT_E_INVAL
    # a taken address, a misaligned one, zero bytes
    with pytest.raises(K.CkptError) as e:
        ctx.vmm_alloc(100, addr=ptrs[1])
    assert e.value.status == K.CKPT_E_ADDR
    with pytest.raises(K.CkptError) as e:
        ctx.vmm_alloc(100, addr=ptrs[1] + 16)
    assert e.value.status == K.CKPT_E_INVAL
    with pytest.raises(K.CkptError) as e:
        ctx.vmm_alloc(0)
    assert e.value.status == K.CKPT_E_INVAL
    # free, then take the same address again on request
    ctx.vmm_free(ptrs[2])
    with pytest.raises(K.CkptError) as e:
        ctx.vmm_free(ptrs[2])
    assert e.value.status == K.CKPT_E_NOTFOUND
    p, _ = ctx.vmm_alloc(sizes[2], addr=ptrs[2])
    assert p == ptrs[2]
    assert ctx.live_count() == len(sizes)
    ctx.close()   # releases the rest


def test_restore_at_recreates_freed_allocations():
    sizes = [1 << 20, 5000, 3 * 4096 + 17, 64, 0, 123457]
    data = seeded(sizes, 2, zero=(3,))
    ctx = K.Context(chunk_bytes=C)
    ptrs = []
    for a in data:
        if a.size == 0:
            ptrs.append(0)
            ctx.register(0, 0)
            continue
        p, _ = ctx.vmm_alloc(a.size)
        h2d(p, a)
        ptrs.append(p)
    img = ctx.checkpoint()
    check_image(img, data)
    assert list(img.addrs) == ptrs
    ids_before = [int(x) for x in img.allocs["id"]]
    for p in ptrs:
        if p:
            ctx.vmm_free(p)
        else:
            ctx.unregister(0)
    assert ctx.live_count() == 0
    rc, rep, addrs = ctx.restore_at(img)
    assert rc == K.CKPT_OK and rep["n_bad"] == 0
    assert addrs == ptrs
    for p, a in zip(addrs, data):
        assert np.array_equal(d2h(p, a.size), a)
    assert ctx.live_count() == len(sizes)
    # this context issued those ids already: the re-created ones get new ids
    again = ctx.checkpoint()
    assert all(int(x) > max(ids_before) for x in again.allocs["id"])
    assert np.array_equal(again.crc, img.crc) and np.array_equal(again.data, img.data)
    assert list(again.addrs) == ptrs
    for p in ptrs:
        if p:
            ctx.vmm_free(p)
    ctx.close()


def test_restore_at_shared_granules_and_hipmalloc_memory():
    """Allocations from hipMalloc, several inside one granule, re-created after
    hipFree at the same addresses (the paper's restart, without replay)."""
    big = hip_malloc(8 << 20)
    # sub-ranges of one hipMalloc block stand for an allocator's sub-allocations
    offs = [0, 256, 4096 + 512, (1 << 20) + 16, (4 << 20) + 4096]
    sizes = [200, 4000, 7000, 1 << 20, 3 << 20]
    data = seeded(sizes, 3, zero=(2,))
    ctx = K.Context(chunk_bytes=C)
    for o, a in zip(offs, data):
        h2d(big + o, a)
        ctx.register(big + o, a.size)
    img = ctx.checkpoint()
    check_image(img, data)
    for o in offs:
        ctx.unregister(big + o)
    hip_free(big)
    rc, rep, addrs = ctx.restore_at(img)
    assert rc == K.CKPT_OK and rep["n_bad"] == 0
    assert addrs == [big + o for o in offs]
    for p, a in zip(addrs, data):
        assert np.array_equal(d2h(p, a.size), a)
    for p in addrs:
        ctx.vmm_free(p)
    ctx.close()


def test_restore_at_in_place_rolls_back_live_memory():
    """Live registrations with the recorded start, size and kind are refilled
    where they are, caller memory (torch tensors) included."""
    t = [torch.empty(s, dtype=torch.uint8, device="cuda") for s in (70000, 4096, 33)]
    data = seeded([x.numel() for x in t], 4)
    ctx = K.Context(chunk_bytes=C)
    for x, a in zip(t, data):
        x.copy_(torch.from_numpy(a))
        ctx.register(x)
    vp, _ = ctx.vmm_alloc(10000)
    vdata = seeded([10000], 5)[0]
    h2d(vp, vdata)
    img = ctx.checkpoint()
    check_image(img, data + [vdata])
    for x in t:
        x.fill_(0x11)
    h2d(vp, np.full(10000, 0x22, np.uint8))
    torch.cuda.synchronize()
    live = ctx.live_count()
    rc, rep, addrs = ctx.restore_at(img)
    assert rc == K.CKPT_OK
    assert addrs == [x.data_ptr() for x in t] + [vp]
    assert ctx.live_count() == live
    for x, a in zip(t, data):
        assert np.array_equal(x.cpu().numpy(), a)
    assert np.array_equal(d2h(vp, 10000), vdata)
    ctx.vmm_free(vp)
    ctx.close()


def test_restore_at_refuses_taken_ranges_and_managed_memory():
    ctx = K.Context(chunk_bytes=C)
    x = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    x.fill_(3)
    ctx.register(x)
    img = ctx.checkpoint()
    # the memory still exists outside the context: its range cannot be reserved
    ctx.unregister(x)
    live = ctx.live_count()
    with pytest.raises(K.CkptError) as e:
        ctx.restore_at(img)
    assert e.value.status == K.CKPT_E_ADDR
    assert ctx.live_count() == live
    # a live registration overlapping without matching exactly
    ctx.register(x.data_ptr() + 4096, 4096)
    with pytest.raises(K.CkptError) as e:
        ctx.restore_at(img)
    assert e.value.status == K.CKPT_E_ADDR
    ctx.unregister(x.data_ptr() + 4096)
    img.close()
    # managed memory cannot be re-created at a fixed address
    m = managed_alloc(8192)
    ctx.register(m, 8192, kind=K.CKPT_MANAGED)
    img = ctx.checkpoint()
    ctx.unregister(m)
    with pytest.raises(K.CkptError) as e:
        ctx.restore_at(img)
    assert e.value.status == K.CKPT_E_INVAL
    # but refilled in place while it is registered
    ctx.register(m, 8192, kind=K.CKPT_MANAGED)
    rc, _, addrs = ctx.restore_at(img)
    assert rc == K.CKPT_OK and addrs == [m]
    ctx.unregister(m)
    managed_free(m)
    # an image without addresses (version-1 data)
    blob = bytearray(img.serialize())
    v1 = bytearray(blob[:88 + 40] + blob[88 + 48:])
    v1[8:12] = (1).to_bytes(4, "little")
    old = K.Image.load(bytes(v1), ctx)
    with pytest.raises(K.CkptError) as e:
        ctx.restore_at(old)
    assert e.value.status == K.CKPT_E_INVAL
    ctx.close()
    del x


def test_restore_at_with_delta_and_corruption():
    sizes = [9 * 4096 + 5, 4096]
    data = seeded(sizes, 6)
    ctx = K.Context(chunk_bytes=C)
    ptrs = []
    for a in data:
        p, _ = ctx.vmm_alloc(a.size)
        h2d(p, a)
        ptrs.append(p)
    base = ctx.checkpoint()
    new = [a.copy() for a in data]
    new[0][3 * 4096:3 * 4096 + 100] = 9
    new[1][:] = 0
    for p, a in zip(ptrs, new):
        h2d(p, a)
    delta = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    ref = O.delta(new, C, base.crc)
    assert np.array_equal(delta.dirty_ids.astype(np.int64), ref["dirty_ids"])
    for p in ptrs:
        ctx.vmm_free(p)
    rc, rep, addrs = ctx.restore_at(base, delta=delta)
    assert rc == K.CKPT_OK and addrs == ptrs
    for p, a in zip(addrs, new):
        assert np.array_equal(d2h(p, a.size), a)
    # a flipped data byte is reported, and the memory is kept
    blob = bytearray(base.serialize())
    blob[-1] ^= 0x40
    bad = K.Image.load(bytes(blob), ctx)
    for p in addrs:
        ctx.vmm_free(p)
    rc, rep, addrs = ctx.restore_at(bad)
    assert rc == K.CKPT_E_CORRUPT and rep["n_bad"] == 1
    assert addrs == ptrs and ctx.live_count() == 2
    for p in addrs:
        ctx.vmm_free(p)
    ctx.close()


def test_restore_file_at(tmp_path):
    sizes = [3 * 4096 + 5, 70000, 16]
    data = seeded(sizes, 7, zero=(2,))
    ctx = K.Context(chunk_bytes=C)
    ptrs = []
    for a in data:
        p, _ = ctx.vmm_alloc(a.size)
        h2d(p, a)
        ptrs.append(p)
    img = ctx.checkpoint()
    path = str(tmp_path / "a.ckpt")
    img.write_file(path)
    for p in ptrs:
        ctx.vmm_free(p)
    rc, rep, addrs, back = ctx.restore_file_at(path)
    assert rc == K.CKPT_OK and rep["n_bad"] == 0 and addrs == ptrs
    for p, a in zip(addrs, data):
        assert np.array_equal(d2h(p, a.size), a)
    assert np.array_equal(back.crc, img.crc) and np.array_equal(back.data, img.data)
    # while the allocations live, the same call refills them in place
    h2d(ptrs[1], np.zeros(70000, np.uint8))
    rc, _, addrs2, back2 = ctx.restore_file_at(path)
    assert rc == K.CKPT_OK and addrs2 == ptrs and ctx.live_count() == 3
    assert np.array_equal(d2h(ptrs[1], 70000), data[1])
    with pytest.raises(K.CkptError) as e:
        ctx.restore_file_at(str(tmp_path / "missing.ckpt"), n_allocs=3)
    assert e.value.status == K.CKPT_E_NOTFOUND
    for p in ptrs:
        ctx.vmm_free(p)
    for im in (img, back, back2):
        im.close()
    ctx.close()


@pytest.mark.parametrize("deflate", [False, True])
def test_restart_in_a_fresh_process_at_the_same_addresses(tmp_path, deflate):
    """Save in one fresh process, restore in another: every allocation comes
    back at its address, with its id, and an incremental checkpoint against
    the loaded image follows.  The file is plain or the compressed container."""
    path = str(tmp_path / "image.ckpt")
    env = dict(os.environ)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")

    def child(*args):
        log("child: %s" % " ".join(args))
        r = subprocess.run([sys.executable, "-m", "tests.restart_child", *args], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    a = child("save", path, *(["deflate"] if deflate else []))
    b = child("restore", path)
    assert b["rc"] == K.CKPT_OK and b["n_bad"] == 0
    assert b["addrs"] == a["addrs"]
    assert b["ids"] == a["ids"]
    assert all(b["same"])
    assert b["clean"] == []
    assert b["dirty"] == [2]   # the chunk rewritten after the restore
    # and the saved image is the oracle's
    from tests.restart_child import contents  # noqa: E402
    img = K.Image.read_file(path)
    check_image(img, contents())
    img.close()


def _child(module, *args):
    env = dict(os.environ)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    log("child %s: %s" % (module, " ".join(args)))
    r = subprocess.run([sys.executable, "-m", module, *args], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def _check_logged(out):
    assert out["failures"] == 0
    assert out["live_count"] == out["n_live"] == out["stats_live"]
    assert out["order"], "live set not in allocation order"
    assert out["crc"] and out["flags"] and out["data"]


def test_hook_logs_every_torch_allocation():
    """torch's allocations reach the hook: the live set is the live tensors,
    in allocation order, and the checkpoint is the oracle's."""
    out = _child("tests.hook_child", "log")
    _check_logged(out)
    assert out["after_free"] == 0


def test_hook_address_stable_restart(tmp_path):
    path = str(tmp_path / "torch.ckpt")
    a = _child("tests.hook_child", "save", path)
    _check_logged(a)
    b = _child("tests.hook_child", "restore", path)
    assert b["rc"] == K.CKPT_OK and b["n_bad"] == 0
    assert b["addrs"] == a["addrs"]
    assert b["sha"] == a["sha"]


@pytest.mark.parametrize("mode", ["plain", "stable"])
def test_hook_cache_keeps_the_log_exact(mode):
    """With the block cache, the live set is still exactly the live tensors
    (registered with their own sizes, whatever the block's class), a freed
    block is handed out again, and trim() empties the cache."""
    out = _child("tests.hook_child", "cache", mode)
    _check_logged(out)
    assert out["cached_after_frees"] >= 1
    assert out["reused"] and out["hit"]
    _check_logged(out["after_reuse"])
    assert out["other_stream_fresh"] and out["same_stream_reused"]
    if mode == "stable":
        # the restore at the recorded addresses gives the cached block back first
        assert out["restore_rc"] == K.CKPT_OK and out["restore_bad"] == 0
        assert out["restore_addrs"] and out["restore_sha"]
        assert out["cached_after_restore"] == 0
    else:
        assert out["cached_before_trim"] >= 1 and out["trimmed"] > 0
    assert out["cached_after_trim"] == 0
    # stable: the allocation re-created by the restore belongs to the context
    assert out["live_at_end"] == (1 if mode == "stable" else 0)


def test_hook_cache_address_stable_restart(tmp_path):
    path = str(tmp_path / "torch_cache.ckpt")
    a = _child("tests.hook_child", "save_cache", path)
    _check_logged(a)
    b = _child("tests.hook_child", "restore", path)
    assert b["rc"] == K.CKPT_OK and b["n_bad"] == 0
    assert b["addrs"] == a["addrs"]
    assert b["sha"] == a["sha"]


def test_hook_cache_under_memory_pressure():
    """A cached block gives way to an allocation that does not fit beside it;
    a request that fits only at its own size is served at that size and not
    cached.  Nothing fails."""
    out = _child("tests.hook_child", "oom")
    log("memory pressure: %s" % out)
    assert out["cached_a"] == 1
    assert out["after_b"] == {"cached": 0, "live": 1}
    assert out["trimmed_b"]
    if out["exact_case"]:
        assert out["after_d"] == {"cached": 0, "live": 1}
    assert out["end"] == {"cached": 0, "live": 0}
    assert out["failures"] == 0
