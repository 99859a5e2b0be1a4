"""Incremental checkpoints across allocation-set changes, chained increments
and merging, against the oracle.

Between two checkpoints the application frees and allocates (the paper's
applications allocate much and free little, but some churn).  The increment is
compared with the oracle's id-keyed increment; folding it into its base must
give exactly the full checkpoint of the current state (the plain definition);
restoring base + increment must give the current bytes.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2008_10596_amd import ckpt as K
from tests.gpu_common import d2h, h2d, host, random_allocs

pytestmark = pytest.mark.gpu

C = 4096


def oracle_delta(tensors, ids, base):
    al = base.allocs
    return O.delta_by_id([host(t) for t in tensors], ids, [0] * len(ids), C, base_ids=list(al["id"]),
                         base_kinds=list(al["kind"]), base_sizes=list(al["size"]), base_crc=base.crc)


def check_delta(delta, ref):
    assert np.array_equal(delta.crc, ref["crc"])
    assert np.array_equal(delta.flags, ref["flags"])
    assert np.array_equal(delta.dirty_ids.astype(np.int64), ref["dirty_ids"].astype(np.int64))
    assert np.array_equal(delta.data, ref["delta"])


def check_same_image(a, b):
    for key in ("allocs", "crc", "flags", "data", "addrs"):
        assert np.array_equal(getattr(a, key), getattr(b, key)), key


def churn(ctx, live, seed):
    """Free the second allocation, edit the first, allocate two new ones (one
    all-zero); returns the new live list of (id, tensor)."""
    (i0, t0), (i1, t1) = live[0], live[1]
    ctx.unregister(t1)
    e = min(t0.numel() - 9, 3 * C + 3)
    t0[e:e + 6] += 1
    rest = live[2:]
    new = random_allocs([3 * C + 100, 2 * C], seed=seed, zero=(1,))
    out = [(i0, t0)] + rest
    for t in new:
        out.append((ctx.register(t), t))
    torch.cuda.synchronize()
    return out


def test_increment_after_frees_and_allocations():
    tensors = random_allocs([9 * C + 5, 4 * C, 123457, C], seed=21, zero=(3,))
    ctx = K.Context(chunk_bytes=C)
    live = [(ctx.register(t), t) for t in tensors]
    base = ctx.checkpoint()
    live = churn(ctx, live, seed=22)
    ids = [i for i, _ in live]
    ts = [t for _, t in live]
    delta = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    ref = oracle_delta(ts, ids, base)
    check_delta(delta, ref)
    assert list(delta.allocs["id"]) == ids
    assert delta.info()["base_serial"] == base.info()["serial"]
    # a full checkpoint against the same base marks the same chunks DIRTY
    full_vs_base = ctx.checkpoint(mode=K.CKPT_FULL, base=base)
    assert np.array_equal(full_vs_base.flags, ref["flags"])
    # merged = the full checkpoint now = the oracle's
    merged = K.merge(base, delta)
    now = ctx.checkpoint()
    check_same_image(merged, now)
    full = O.checkpoint([host(t) for t in ts], C)
    assert np.array_equal(merged.crc, full["crc"]) and np.array_equal(merged.flags, full["flags"])
    assert np.array_equal(merged.data, full["serialized"])
    assert merged.info()["mode"] == K.CKPT_FULL and merged.info()["serial"] == delta.info()["serial"]
    # restore base + increment into buffers of the new table
    dsts = [torch.empty_like(t) for t in ts]
    rc, rep = ctx.restore(base, dsts, delta=delta)
    assert rc == K.CKPT_OK, rep
    for a, b in zip(dsts, ts):
        assert torch.equal(a, b)
    # the old table's destination count is refused
    with pytest.raises(K.CkptError) as e:
        ctx.restore(base, [torch.empty_like(t) for t in tensors], delta=delta)
    assert e.value.status == K.CKPT_E_MISMATCH
    for im in (base, delta, full_vs_base, merged, now):
        im.close()
    ctx.close()


def test_chain_of_increments_folds_into_the_current_image():
    tensors = random_allocs([5 * C, 3 * C + 1, 70000], seed=23)
    ctx = K.Context(chunk_bytes=C)
    live = [(ctx.register(t), t) for t in tensors]
    base = ctx.checkpoint()
    live = churn(ctx, live, seed=24)
    d1 = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    # second step: same table, an edit only
    live[-2][1][7:20] = 3
    torch.cuda.synchronize()
    d2 = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=d1)
    ref2 = oracle_delta([t for _, t in live], [i for i, _ in live], d1)
    check_delta(d2, ref2)
    # third step: another table change
    live = churn(ctx, live, seed=25)
    d3 = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=d2)
    ref3 = oracle_delta([t for _, t in live], [i for i, _ in live], d2)
    check_delta(d3, ref3)
    merged = K.merge(base, d1, d2, d3)
    now = ctx.checkpoint()
    check_same_image(merged, now)
    # restore the chain's last step on top of the merge of the first two
    m12 = K.merge(base, d1, d2)
    dsts = [torch.empty_like(t) for _, t in live]
    rc, _ = ctx.restore(m12, dsts, delta=d3)
    assert rc == K.CKPT_OK
    for a, (_, b) in zip(dsts, live):
        assert torch.equal(a, b)
    # merging out of order is refused
    with pytest.raises(K.CkptError) as e:
        K.merge(base, d2)
    assert e.value.status == K.CKPT_E_MISMATCH
    for im in (base, d1, d2, d3, merged, now, m12):
        im.close()
    ctx.close()


def test_merge_refuses_inconsistent_images():
    tensors = random_allocs([3 * C], seed=26)
    ctx = K.Context(chunk_bytes=C)
    for t in tensors:
        ctx.register(t)
    base = ctx.checkpoint()
    tensors[0][10] += 1
    delta = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    with pytest.raises(K.CkptError) as e:
        K.merge(delta, delta)
    assert e.value.status == K.CKPT_E_INVAL
    # an increment whose serialized DATA was cut disagrees with its flags
    blob = delta.serialize()
    n_data = delta.info()["serialized_bytes"]
    assert n_data > 0
    cut = bytearray(blob[:-16])
    # patch the header's serialized-bytes field (fourth 64-bit header word)
    cut[24 + 3 * 8:24 + 4 * 8] = (n_data - 16).to_bytes(8, "little")
    short = K.Image.load(bytes(cut), ctx)
    with pytest.raises(K.CkptError) as e:
        K.merge(base, short)
    assert e.value.status == K.CKPT_E_CORRUPT
    # another chunk size is refused at checkpoint time
    c2 = K.Context(chunk_bytes=2 * C)
    c2.register(tensors[0])
    with pytest.raises(K.CkptError) as e:
        c2.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    assert e.value.status == K.CKPT_E_MISMATCH
    for im in (base, delta, short):
        im.close()
    c2.close()
    ctx.close()


def test_restore_at_follows_the_increments_table():
    """Address-stable memory: after frees and new allocations, base +
    increment come back at the increment's addresses."""
    ctx = K.Context(chunk_bytes=C)
    rng = np.random.default_rng(27)
    sizes = [6 * C + 7, 2 * C, 5000]
    data = [rng.integers(0, 256, s, dtype=np.uint8) for s in sizes]
    ptrs = []
    for a in data:
        p, _ = ctx.vmm_alloc(a.size)
        h2d(p, a)
        ptrs.append(p)
    base = ctx.checkpoint()
    ctx.vmm_free(ptrs[1])
    data[0][C:C + 50] = 0
    h2d(ptrs[0], data[0])
    p3, _ = ctx.vmm_alloc(3 * C)
    d3 = rng.integers(0, 256, 3 * C, dtype=np.uint8)
    h2d(p3, d3)
    delta = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    want = [(ptrs[0], data[0]), (ptrs[2], data[2]), (p3, d3)]
    for p in (ptrs[0], ptrs[2], p3):
        ctx.vmm_free(p)
    rc, rep, addrs = ctx.restore_at(base, delta=delta)
    assert rc == K.CKPT_OK and rep["n_bad"] == 0
    assert addrs == [p for p, _ in want]
    for p, a in want:
        assert np.array_equal(d2h(p, a.size), a)
    assert ctx.live_count() == 3
    for p in addrs:
        ctx.vmm_free(p)
    base.close()
    delta.close()
    ctx.close()
