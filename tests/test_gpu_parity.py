"""Bit-exact parity of the HIP path with the CPU oracle, through the C ABI.

Every comparison is element by element: allocation table, per-chunk CRC-32C,
ZERO/DIRTY flags, serialized data, dense device image, dirty-id lists,
restored memory and verification reports.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from paper_2008_10596_amd import ckpt as K
from tests.gpu_common import (FLAG_ZERO, assert_dense, check_full, check_restored, d2h, host, log, r16,
                              random_allocs, register_all)

pytestmark = pytest.mark.gpu


def full_roundtrip(tensors, C, zero_expect=None, **ctx_kw):
    ctx = K.Context(chunk_bytes=C, flags=K.CKPT_KEEP_DENSE, **ctx_kw)
    ids = register_all(ctx, tensors)
    img = ctx.checkpoint()
    ref = O.checkpoint([host(t) for t in tensors], C)
    check_full(img, ref, tensors, C, ids)
    # dense device image == oracle dense image
    p, nb = img.dense_ptr
    assert nb == ref["data_bytes"]
    assert_dense(d2h(p, nb), ref["dense"][:nb], [t.numel() for t in tensors], C, ref["flags"])
    # restore into fresh buffers
    dsts = [torch.full((t.numel(),), 0xA5, dtype=torch.uint8, device="cuda") for t in tensors]
    rc, rep = ctx.restore(img, dsts)
    assert rc == K.CKPT_OK and rep["n_bad"] == 0
    check_restored(dsts, tensors)
    img.close()
    ctx.close()
    return ref


def test_plain_workload_64_allocations():
    w = synth.plain()
    log("plain workload: %d allocations, %d bytes" % (len(w["sizes"]), int(w["sizes"].sum())))
    tensors = synth.make_device_allocs(w["sizes"], w["zero"], workload=1)
    full_roundtrip(tensors, 4096)


EDGE_SIZES = [0, 1, 2, 3, 4, 5, 7, 15, 16, 17, 31, 33, 63, 64, 65, 1007, 1008, 1009, 1023, 1024,
              1025, 2047, 2048, 4095, 4096, 4097, 4111, 4112, 8191, 8192, 12289, 65535, 65536, 65537,
              100003]


@pytest.mark.parametrize("C", [16, 32, 48, 256, 1008, 1024, 1040, 4096, 4112, 16384, 65536, 262144])
def test_edge_sizes_and_chunk_sizes(C):
    log("edge sizes, C=%d" % C)
    tensors = random_allocs(EDGE_SIZES, seed=C, zero=(9, 20))
    # single non-zero bytes inside otherwise-zero allocations, at chunk edges
    for t, pos in zip(tensors[9:10] + tensors[20:21], (3, 1000)):
        if pos < t.numel():
            t[pos] = 7
    full_roundtrip(tensors, C)


@pytest.mark.parametrize("C", [1024, 4096, 65536])
def test_restore_writes_nothing_past_each_destination(C):
    """Restore destinations are views of one buffer filled with a guard byte;
    every byte outside [dst_k, dst_k + size_k) must keep it, including the
    bytes between a size and the next multiple of 16 (tail pieces)."""
    sizes = [1, 15, 17, C - 4, C + 12, 3 * C - 1, 2 * C, 70001]
    tensors = random_allocs(sizes, seed=C + 1, zero=(6,))
    ctx = K.Context(chunk_bytes=C)
    register_all(ctx, tensors)
    img = ctx.checkpoint()
    gap = 64
    offs, o = [], gap
    for sz in sizes:
        offs.append(o)
        o += (sz + 15) // 16 * 16 + gap
    buf = torch.full((o,), 0xEE, dtype=torch.uint8, device="cuda")
    dsts = [buf[a:a + sz] for a, sz in zip(offs, sizes)]
    rc, rep = ctx.restore(img, dsts)
    assert rc == K.CKPT_OK, rep
    check_restored(dsts, tensors)
    h = host(buf)
    mask = np.ones(o, bool)
    for a, sz in zip(offs, sizes):
        mask[a:a + sz] = False
    assert (h[mask] == 0xEE).all(), np.flatnonzero(h[mask] != 0xEE)[:10]
    # the same through a delta overlay
    for t in tensors:
        t[-1] ^= 0x5A
    torch.cuda.synchronize()
    delta = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=img)
    buf.fill_(0xEE)
    rc, rep = ctx.restore(img, dsts, delta=delta)
    assert rc == K.CKPT_OK, rep
    check_restored(dsts, tensors)
    h = host(buf)
    assert (h[mask] == 0xEE).all()
    img.close()
    delta.close()
    ctx.close()


@pytest.mark.parametrize("block,wpc", [(64, 1), (256, 1), (256, 2), (256, 4), (512, 8), (1024, 1), (1024, 16)])
@pytest.mark.parametrize("C", [4096, 65536])
def test_launch_shapes(block, wpc, C):
    log("launch shape block=%d waves/chunk=%d C=%d" % (block, wpc, C))
    sizes = [C * 3 + 5, C, C - 16, 17, C * 2, 1 << 20]
    tensors = random_allocs(sizes, seed=block * 31 + wpc, zero=(1,))
    full_roundtrip(tensors, C, block_threads=block, waves_per_chunk=wpc)


@pytest.mark.parametrize("hint", [1, 2])
@pytest.mark.parametrize("C,wpc", [(4096, 1), (65536, 1), (65536, 4), (1040, 1), (262144, 2)])
def test_load_hints(hint, C, wpc):
    log("load_hint=%d C=%d waves/chunk=%d" % (hint, C, wpc))
    sizes = [C * 3 + 5, C, C - 16, 17, 1, 4, 3 * 1024 + 7, 1 << 20]
    tensors = random_allocs(sizes, seed=100 + hint * 10 + wpc, zero=(1,))
    full_roundtrip(tensors, C, load_hint=hint, waves_per_chunk=wpc)


def test_zero_chunks_inside_random_allocations():
    C = 4096
    tensors = random_allocs([C * 10 + 100, C * 3], seed=5)
    tensors[0][C * 2:C * 4] = 0          # two interior ZERO chunks
    tensors[0][C * 10:] = 0              # ZERO tail chunk
    tensors[1][:C] = 0
    ref = full_roundtrip(tensors, C)
    assert [int(f) & FLAG_ZERO for f in ref["flags"]] == [0, 0, 1, 1, 0, 0, 0, 0, 0, 0, 1, 1, 0, 0]


def test_empty_and_all_zero_contexts():
    ctx = K.Context()
    img = ctx.checkpoint()
    info = img.info()
    assert info["n_allocs"] == 0 and info["n_chunks"] == 0 and info["serialized_bytes"] == 0
    rc, rep = ctx.restore(img, [])
    assert rc == K.CKPT_OK
    tensors = [torch.zeros(n, dtype=torch.uint8, device="cuda") for n in (0, 5000, 4096)]
    register_all(ctx, tensors)
    img = ctx.checkpoint()
    ref = O.checkpoint([host(t) for t in tensors], 4096)
    check_full(img, ref, tensors, 4096)
    assert img.info()["serialized_bytes"] == 0


def test_registration_order_and_unregister():
    ctx = K.Context(chunk_bytes=1024)
    tensors = random_allocs([3000, 100, 5000, 77, 2048], seed=11)
    ids = register_all(ctx, tensors)
    assert ids == [1, 2, 3, 4, 5]
    ctx.unregister(tensors[1])
    ctx.unregister(tensors[3])
    extra = random_allocs([999], seed=12)[0]
    assert ctx.register(extra) == 6
    live = [tensors[0], tensors[2], tensors[4], extra]
    img = ctx.checkpoint()
    ref = O.checkpoint([host(t) for t in live], 1024)
    check_full(img, ref, live, 1024, ids=[1, 3, 5, 6])


def test_registration_errors():
    ctx = K.Context()
    buf = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr()
    with pytest.raises(K.CkptError) as e:
        ctx.register(base + 8, 64)
    assert e.value.status == K.CKPT_E_INVAL
    with pytest.raises(K.CkptError) as e:
        ctx.register(base, 64, kind=7)
    assert e.value.status == K.CKPT_E_INVAL
    ctx.register(base, 4096)
    for start, n in ((base, 16), (base + 4080, 32), (base - 16, 32), (base + 16, 16)):
        with pytest.raises(K.CkptError) as e:
            ctx.register(start, n)
        assert e.value.status == K.CKPT_E_INVAL, (start - base, n)
    ctx.register(base + 4096, 4096)      # adjacent: fine
    with pytest.raises(K.CkptError) as e:
        ctx.unregister(base + 16)
    assert e.value.status == K.CKPT_E_NOTFOUND
    ctx.unregister(base)
    ctx.register(base, 16)               # the range is free again
    assert ctx.live_count() == 2


# ------------------------------------------------------------ incremental

@pytest.mark.parametrize("C,wpc", [(4096, 1), (65536, 1), (65536, 4), (1040, 1)])
def test_incremental_matches_oracle_and_restores(C, wpc):
    log("incremental C=%d waves/chunk=%d" % (C, wpc))
    sizes = [C * 7 + 123, C * 2, 5000, C * 30, 16]
    tensors = random_allocs(sizes, seed=C + 1)
    ctx = K.Context(chunk_bytes=C, waves_per_chunk=wpc)
    register_all(ctx, tensors)
    base = ctx.checkpoint()
    base_ref = O.checkpoint([host(t) for t in tensors], C)
    check_full(base, base_ref, tensors, C)
    # mutate: rewrite some chunks, zero one, touch a tail byte
    tensors[0][C:2 * C] = torch.randint(0, 256, (C,), dtype=torch.uint8, device="cuda")
    tensors[3][5 * C:6 * C] = 0
    tensors[0][-1] ^= 1
    tensors[4][3] ^= 0x80
    hosts = [host(t) for t in tensors]
    dref = O.delta(hosts, C, base_ref["crc"])
    delta = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    info = delta.info()
    assert info["mode"] == K.CKPT_INCREMENTAL
    assert info["base_serial"] == base.info()["serial"]
    assert np.array_equal(delta.crc, dref["crc"])
    assert np.array_equal(delta.flags, dref["flags"])
    assert np.array_equal(delta.dirty_ids, dref["dirty_ids"])
    assert np.array_equal(delta.data, dref["delta"])
    # restore(base, delta) == current memory
    dsts = [torch.full((t.numel(),), 0x5A, dtype=torch.uint8, device="cuda") for t in tensors]
    rc, rep = ctx.restore(base, dsts, delta=delta)
    assert rc == K.CKPT_OK, rep
    check_restored(dsts, tensors)
    # a second increment against the first (the device-resident CRC chain)
    tensors[1][:10] = 1
    hosts2 = [host(t) for t in tensors]
    dref2 = O.delta(hosts2, C, dref["crc"])
    delta2 = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=delta)
    assert np.array_equal(delta2.dirty_ids, dref2["dirty_ids"])
    assert np.array_equal(delta2.data, dref2["delta"])


HASH_SHAPES = ([(C, block, 1) for C in (16, 48, 256, 1008, 1024, 1040, 2048, 3088, 4096, 4112)
                for block in (64, 256, 1024)] +
               [(4096, 1024, 2), (4096, 256, 4), (16384, 1024, 1), (65536, 1024, 1), (65536, 1024, 4),
                (65536, 256, 2), (262144, 1024, 2), (262144, 512, 8)])


@pytest.mark.parametrize("C,block,wpc", HASH_SHAPES)
def test_incremental_edge_sizes(C, block, wpc):
    """Hash-only pass over the edge sizes: every chunk length from 1 byte to a
    full chunk, rows of four chunks that end inside a tile, all-zero chunks,
    one or several waves per chunk."""
    log("incremental edge sizes C=%d block=%d waves/chunk=%d" % (C, block, wpc))
    tensors = random_allocs(EDGE_SIZES, seed=C + block + wpc, zero=(9, 20))
    ctx = K.Context(chunk_bytes=C, block_threads=block, waves_per_chunk=wpc)
    register_all(ctx, tensors)
    base = ctx.checkpoint()
    base_ref = O.checkpoint([host(t) for t in tensors], C)
    check_full(base, base_ref, tensors, C)
    g = torch.Generator(device="cuda")
    g.manual_seed(C * 7 + block)
    for k, t in enumerate(tensors):
        n = t.numel()
        if n and k % 3 != 2:
            pos = torch.randint(0, n, (1 + n // 5000,), generator=g, device="cuda")
            t[pos] ^= 0x11
    tensors[20][5:9] = 3                      # a chunk of an all-zero allocation gets data
    hosts = [host(t) for t in tensors]
    dref = O.delta(hosts, C, base_ref["crc"])
    delta = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    assert np.array_equal(delta.crc, dref["crc"])
    assert np.array_equal(delta.flags, dref["flags"])
    assert np.array_equal(delta.dirty_ids, dref["dirty_ids"])
    assert np.array_equal(delta.data, dref["delta"])
    for im in (base, delta):
        im.close()
    ctx.close()


def test_incremental_all_dirty_equals_full():
    C = 4096
    tensors = random_allocs([C * 5 + 9, 300, C * 2], seed=77, zero=(1,))
    ctx = K.Context(chunk_bytes=C)
    register_all(ctx, tensors)
    base = ctx.checkpoint()
    for t in tensors:
        synth.fill_random_(t, t.numel() + 3)
    tensors[1].zero_()
    tensors[1][0] = 1                    # the ZERO chunk becomes non-ZERO
    full = K.Context(chunk_bytes=C)
    register_all(full, tensors)
    f = full.checkpoint()
    d = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    assert list(d.dirty_ids) == list(range(d.info()["n_chunks"]))
    assert np.array_equal(d.data, f.data)
    assert np.array_equal(d.crc, f.crc)


def test_incremental_nothing_changed_is_empty():
    ctx = K.Context()
    tensors = random_allocs([10000, 5000], seed=3)
    register_all(ctx, tensors)
    base = ctx.checkpoint()
    d = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    assert d.info()["n_dirty"] == 0 and d.info()["serialized_bytes"] == 0
    assert not (d.flags & 2).any()


def test_incremental_base_mismatch():
    ctx = K.Context()
    tensors = random_allocs([10000, 5000], seed=4)
    register_all(ctx, tensors)
    base = ctx.checkpoint()
    # a new allocation since the base: an id-keyed increment, the new
    # allocation's chunk DIRTY and nothing else
    extra = random_allocs([64], seed=5)[0]
    ctx.register(extra)
    d = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    assert list(d.dirty_ids) == [base.info()["n_chunks"]]
    # another chunk size is a mismatch
    other = K.Context(chunk_bytes=8192)
    register_all(other, tensors)
    with pytest.raises(K.CkptError) as e:
        other.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    assert e.value.status == K.CKPT_E_MISMATCH
    with pytest.raises(K.CkptError) as e:
        other.restore(base, tensors)
    assert e.value.status == K.CKPT_E_MISMATCH


# --------------------------------------------------------------- restore

def test_restore_errors():
    ctx = K.Context()
    tensors = random_allocs([10000, 5000], seed=6)
    register_all(ctx, tensors)
    img = ctx.checkpoint()
    with pytest.raises(K.CkptError) as e:
        ctx.restore(img, tensors[:1])
    assert e.value.status == K.CKPT_E_MISMATCH
    small = [torch.empty(10000, dtype=torch.uint8, device="cuda"), torch.empty(4999, dtype=torch.uint8, device="cuda")]
    with pytest.raises(K.CkptError) as e:
        ctx.restore(img, small)
    assert e.value.status == K.CKPT_E_MISMATCH
    buf = torch.empty(20000, dtype=torch.uint8, device="cuda")
    with pytest.raises(K.CkptError) as e:
        ctx.restore(img, [buf.data_ptr() + 8, buf.data_ptr() + 10016], dst_bytes=[10000, 5000])
    assert e.value.status == K.CKPT_E_INVAL
    # a delta taken against another image
    img2 = ctx.checkpoint()
    d = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=img2)
    with pytest.raises(K.CkptError) as e:
        ctx.restore(img, tensors, delta=d)
    assert e.value.status == K.CKPT_E_MISMATCH


def test_restore_size_rule():
    """Every destination must have exactly its allocation's size: larger and
    smaller are refused before anything is written; without sizes (raw
    addresses, dst_bytes NULL) the caller's word is taken and exactly the
    allocations' bytes are written."""
    ctx = K.Context()
    tensors = random_allocs([10000, 5000], seed=16)
    register_all(ctx, tensors)
    img = ctx.checkpoint()
    for sizes in ([10000, 5001], [10000, 4999], [10016, 5000], [9999, 5000]):
        dsts = [torch.full((s,), 0x77, dtype=torch.uint8, device="cuda") for s in sizes]
        with pytest.raises(K.CkptError) as e:
            ctx.restore(img, dsts)
        assert e.value.status == K.CKPT_E_MISMATCH, sizes
        assert all(bool((d == 0x77).all()) for d in dsts), "a refused restore wrote memory"
    buf = torch.full((20000,), 0x77, dtype=torch.uint8, device="cuda")
    ptrs = [buf.data_ptr(), buf.data_ptr() + 10240]
    for db in ([10000, 5008], [10000, 4992], [10240, 5000]):
        with pytest.raises(K.CkptError) as e:
            ctx.restore(img, ptrs, dst_bytes=db)
        assert e.value.status == K.CKPT_E_MISMATCH, db
    assert bool((buf == 0x77).all())
    rc, rep = ctx.restore(img, ptrs, dst_bytes=[10000, 5000])
    assert rc == K.CKPT_OK, rep
    buf.fill_(0x77)
    rc, rep = ctx.restore(img, ptrs)          # dst_bytes NULL
    assert rc == K.CKPT_OK, rep
    h = host(buf)
    assert np.array_equal(h[:10000], host(tensors[0]))
    assert np.array_equal(h[10240:15240], host(tensors[1]))
    assert (h[10000:10240] == 0x77).all() and (h[15240:] == 0x77).all(), "bytes past an allocation written"
    img.close()
    ctx.close()


def test_corruption_is_reported_exactly():
    C = 1024
    sizes = [C * 9 + 40, C * 4]
    tensors = random_allocs(sizes, seed=8)
    tensors[1][:C] = 0                           # chunk 10 is ZERO
    ctx = K.Context(chunk_bytes=C)
    register_all(ctx, tensors)
    img = ctx.checkpoint()
    ref = O.checkpoint([host(t) for t in tensors], C)
    data = img.data                              # writable view of the pinned host image
    # flip one bit in serialized chunk 3 (all chunks before it are non-ZERO, full size)
    data[3 * C + 100] ^= 0x10
    dsts = [torch.empty(s, dtype=torch.uint8, device="cuda") for s in sizes]
    rc, rep = ctx.restore(img, dsts)
    assert rc == K.CKPT_E_CORRUPT and rep["n_bad"] == 1 and rep["ids"] == [3]
    # the data is still written, as stored
    h = [host(d) for d in dsts]
    assert h[0][3 * C + 100] == ref["serialized"][3 * C + 100] ^ 0x10
    data[3 * C + 100] ^= 0x10
    # a ZERO chunk whose stored CRC was changed
    img.crc[10] ^= 1
    rc, rep = ctx.restore(img, dsts)
    assert rc == K.CKPT_E_CORRUPT and rep["ids"] == [10]
    img.crc[10] ^= 1
    rc, rep = ctx.restore(img, dsts)
    assert rc == K.CKPT_OK
    # many bad chunks: count and the first 64 ids, ascending
    crc = img.crc
    crc ^= np.uint32(0xDEAD)
    rc, rep = ctx.restore(img, dsts)
    assert rc == K.CKPT_E_CORRUPT and rep["n_bad"] == img.info()["n_chunks"]
    assert rep["ids"] == list(range(min(64, img.info()["n_chunks"])))


def _flip(t, i, bit):
    t[i:i + 1] = torch.bitwise_xor(t[i:i + 1], bit)


def test_delta_corruption_is_the_union_of_both_passes():
    """Restore of a base plus an increment: a chunk is bad when it fails the
    base pass or the overlay, and is counted once.  Every case is compared
    with the union of the oracle's two reports, and the restored memory with
    the oracle's."""
    C = 1024
    sizes = [C * 9 + 40, C * 4, C * 3 + 500]   # chunks 0-9 (9: 40 B) | 10-13 | 14-17 (17: 500 B)
    tensors = random_allocs(sizes, seed=18)
    ctx = K.Context(chunk_bytes=C)
    register_all(ctx, tensors)
    base = ctx.checkpoint()
    h0 = [host(t) for t in tensors]
    ref_base = O.checkpoint(h0, C)
    check_full(base, ref_base, tensors, C)
    _flip(tensors[0], 2 * C + 5, 0x40)           # chunk 2
    _flip(tensors[0], 9 * C + 3, 0x01)           # chunk 9, a tail
    tensors[1][:C] = 0                           # chunk 10 becomes ZERO
    _flip(tensors[2], 3 * C + 100, 0x80)         # chunk 17, a tail
    d = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=base)
    h1 = [host(t) for t in tensors]
    dref = O.delta(h1, C, ref_base["crc"])
    assert list(dref["dirty_ids"]) == [2, 9, 10, 17]
    assert np.array_equal(d.dirty_ids, dref["dirty_ids"]) and np.array_equal(d.data, dref["delta"])
    assert np.array_equal(d.crc, dref["crc"]) and np.array_equal(d.flags, dref["flags"])
    lens = [min(C, s - st) for s in sizes for st in range(0, s, C)]
    b_at = [sum(r16(x) for x in lens[:g]) for g in range(len(lens))]   # no ZERO chunk in the base
    d_at = {2: 0, 9: 1024, 17: 1072}                                   # increment pieces
    # (name, base data bytes to flip, base CRCs to change, increment data bytes, increment CRCs)
    cases = [
        ("increment byte", [], [], [d_at[9] + 7], []),
        ("increment CRC of the ZERO chunk", [], [], [], [10]),
        ("same chunk in both passes", [b_at[9] + 1], [], [d_at[9] + 2], []),
        ("base repaired by the increment, base only, increment only",
         [b_at[2] + 9, b_at[5]], [], [], [17]),
        ("every increment CRC", [], [], [], [2, 9, 10, 17]),
        ("base CRC and increment byte", [], [12, 13], [d_at[17] + 499], []),
    ]
    for name, bdata, bcrc, ddata, dcrc in cases:
        ser_b, crc_b = ref_base["serialized"].copy(), ref_base["crc"].copy()
        ser_d, crc_d = dref["delta"].copy(), dref["crc"].copy()
        for i in bdata:
            base.data[i] ^= 0x08
            ser_b[i] ^= 0x08
        for g in bcrc:
            base.crc[g] ^= 0x100
            crc_b[g] ^= 0x100
        for i in ddata:
            d.data[i] ^= 0x08
            ser_d[i] ^= 0x08
        for g in dcrc:
            d.crc[g] ^= 0x100
            crc_d[g] ^= 0x100
        bufs, _, ids_b = O.restore(sizes, C, crc_b, ref_base["flags"], ser_b)
        _, ids_d = O.restore_delta(bufs, sizes, C, crc_d, dref["flags"], dref["dirty_ids"], ser_d)
        want = sorted(set(int(x) for x in ids_b) | set(int(x) for x in ids_d))
        dsts = [torch.full((s,), 0x5A, dtype=torch.uint8, device="cuda") for s in sizes]
        rc, rep = ctx.restore(base, dsts, delta=d)
        log("%s: gpu %s, oracle base %s + increment %s" % (name, rep, list(ids_b), list(ids_d)))
        assert want, name
        assert rc == K.CKPT_E_CORRUPT, name
        assert rep["n_bad"] == len(want) and rep["ids"] == want, (name, rep, want)
        for k, dst in enumerate(dsts):
            assert np.array_equal(host(dst), bufs[k]), (name, k)
        for i in bdata:
            base.data[i] ^= 0x08
        for g in bcrc:
            base.crc[g] ^= 0x100
        for i in ddata:
            d.data[i] ^= 0x08
        for g in dcrc:
            d.crc[g] ^= 0x100
    dsts = [torch.empty_like(t) for t in tensors]
    rc, rep = ctx.restore(base, dsts, delta=d)
    assert rc == K.CKPT_OK, rep
    check_restored(dsts, tensors)
    d.close()
    base.close()
    ctx.close()


@pytest.mark.parametrize("C", [1024, 4096, 65536])
def test_zero_chunks_verified_on_every_path(C):
    """Full-length ZERO chunks are restored without hashing (their CRC is the
    CRC of C zero bytes); ZERO tails are hashed.  Both must verify, and a
    changed stored CRC on either must be reported exactly."""
    sizes = [3 * C, 2 * C + 48, C]
    tensors = random_allocs(sizes, seed=11)
    tensors[0][C:2 * C] = 0                      # chunk 1: full ZERO
    tensors[1][2 * C:] = 0                       # chunk 5: ZERO tail of 48 bytes
    tensors[2].zero_()                           # chunk 6: full ZERO
    ctx = K.Context(chunk_bytes=C)
    register_all(ctx, tensors)
    img = ctx.checkpoint()
    ref = O.checkpoint([host(t) for t in tensors], C)
    assert np.array_equal(img.flags, ref["flags"]) and np.array_equal(img.crc, ref["crc"])
    assert [g for g in range(len(ref["flags"])) if ref["flags"][g] & FLAG_ZERO] == [1, 5, 6]
    dsts = [torch.full((s,), 0x5A, dtype=torch.uint8, device="cuda") for s in sizes]
    rc, rep = ctx.restore(img, dsts)
    assert rc == K.CKPT_OK, rep
    check_restored(dsts, tensors)
    for g in (1, 5, 6):
        img.crc[g] ^= 0x80
        rc, rep = ctx.restore(img, dsts)
        assert rc == K.CKPT_E_CORRUPT and rep["ids"] == [g], (g, rep)
        img.crc[g] ^= 0x80
    img.close()
    ctx.close()


def test_many_bad_report_first_64_of_many():
    C = 256
    tensors = random_allocs([C * 500 + 7], seed=9)
    ctx = K.Context(chunk_bytes=C)
    register_all(ctx, tensors)
    img = ctx.checkpoint()
    bad = [5, 17, 64, 65, 100, 250, 499, 500] + list(range(300, 400))
    for g in bad:
        img.crc[g] ^= 0x100
    rc, rep = ctx.restore(img, [torch.empty_like(tensors[0])])
    assert rc == K.CKPT_E_CORRUPT
    assert rep["n_bad"] == len(set(bad))
    assert rep["ids"] == sorted(set(bad))[:64]


# ------------------------------------------------------------ serialization

def test_serialize_load_roundtrip_and_restore():
    C = 4096
    tensors = random_allocs([50000, 4096, 123], seed=10, zero=(1,))
    ctx = K.Context(chunk_bytes=C)
    register_all(ctx, tensors)
    img = ctx.checkpoint()
    blob = img.serialize()
    img2 = K.Image.load(blob, ctx)
    assert img2.serialize() == blob
    for name in ("crc", "flags", "data", "allocs", "addrs"):
        assert np.array_equal(getattr(img2, name), getattr(img, name)), name
    assert list(img.addrs) == [t.data_ptr() for t in tensors]
    # version-1 data (no address section) still loads, with addresses 0
    n = len(tensors)
    v1 = bytearray(blob[:88 + n * 40] + blob[88 + n * 48:])
    v1[8:12] = (1).to_bytes(4, "little")
    img1 = K.Image.load(bytes(v1), ctx)
    assert list(img1.addrs) == [0] * n
    for name in ("crc", "flags", "data", "allocs"):
        assert np.array_equal(getattr(img1, name), getattr(img, name)), name
    img1.close()
    dsts = [torch.empty_like(t) for t in tensors]
    rc, _ = ctx.restore(img2, dsts)
    assert rc == K.CKPT_OK
    check_restored(dsts, tensors)
    # truncated and bit-flipped (digest) buffers are refused
    with pytest.raises(K.CkptError) as e:
        K.Image.load(blob[:-1], ctx)
    assert e.value.status == K.CKPT_E_INVAL
    bad = bytearray(blob)
    bad[88 + 3 * 48 + 2] ^= 1                   # inside the CRC section
    with pytest.raises(K.CkptError) as e:
        K.Image.load(bytes(bad), ctx)
    assert e.value.status == K.CKPT_E_INVAL


# ------------------------------------------------------------------ batch

def test_batch_equals_each_context_alone():
    C = 4096
    rng = np.random.default_rng(12)
    ctxs, allocs = [], []
    for i in range(12):
        sizes = [int(x) for x in rng.integers(0, 300000, int(rng.integers(1, 6)))]
        t = random_allocs(sizes, seed=100 + i, zero=(0,) if i % 3 == 0 else ())
        c = K.Context(chunk_bytes=C)
        register_all(c, t)
        ctxs.append(c)
        allocs.append(t)
    ctxs.append(K.Context(chunk_bytes=C))       # an empty context in the batch
    allocs.append([])
    imgs = K.checkpoint_batch(ctxs)
    for c, t, img in zip(ctxs, allocs, imgs):
        ref = O.checkpoint([host(x) for x in t], C)
        check_full(img, ref, t, C)
        dsts = [torch.empty_like(x) for x in t]
        rc, _ = c.restore(img, dsts)
        assert rc == K.CKPT_OK
        check_restored(dsts, t)


# --------------------------------------------------------------- ordering

def test_checkpoint_sees_work_enqueued_before_it():
    """A writer enqueued before the checkpoint (same stream, stream-ordered
    mode; another stream, default device-wide mode) is in the image."""
    n = 64 << 20
    for flags, other_stream in ((K.CKPT_STREAM_ORDERED, False), (0, True)):
        t = torch.zeros(n, dtype=torch.uint8, device="cuda")
        ctx = K.Context(chunk_bytes=65536, flags=flags)
        ctx.register(t)
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            for _ in range(20):                 # long enough to still be running
                t.add_(1)
        img = ctx.checkpoint(stream=torch.cuda.current_stream() if other_stream else s)
        ref = O.checkpoint([np.full(n, 20, np.uint8)], 65536)
        assert np.array_equal(img.crc, ref["crc"]), "checkpoint missed prior work (flags=%d)" % flags
        ctx.close()


def test_timing_is_reported():
    ctx = K.Context(flags=K.CKPT_TIMING)
    tensors = random_allocs([8 << 20, 4 << 20], seed=13)
    register_all(ctx, tensors)
    ctx.checkpoint()
    t = ctx.timing()
    assert t["pack_ms"] > 0 and t["d2h_ms"] > 0
    assert t["pack_read_bytes"] == 12 << 20


def test_drain_direct_matches():
    C = 4096
    tensors = random_allocs([3 << 20, 4096 * 3 + 1], seed=14)
    tensors[0][: 1 << 20] = 0
    ctx = K.Context(chunk_bytes=C, flags=K.CKPT_DRAIN_DIRECT)
    register_all(ctx, tensors)
    img = ctx.checkpoint()
    ref = O.checkpoint([host(t) for t in tensors], C)
    check_full(img, ref, tensors, C)


def test_staging_budget():
    ctx = K.Context(staging_budget=1 << 20)
    ctx.register(torch.empty(2 << 20, dtype=torch.uint8, device="cuda"))
    with pytest.raises(K.CkptError) as e:
        ctx.checkpoint()
    assert e.value.status == K.CKPT_E_BUDGET


@pytest.mark.parametrize("segment_mib", [0, 1, 0xFFFFFFFF])
def test_reserved_staging_matches_the_oracle(segment_mib):
    """CKPT_RESERVE_STAGING: the staging budget is one block made at
    ckpt_init; checkpoints (full, drained in segments or in one pass, and
    incremental) and restores take their staging from it and equal the oracle."""
    C = 4096
    log("reserved staging, segment_mib=%d" % segment_mib)
    sizes = [3 << 20, 12345, 0, 1 << 20, 4096 * 5 + 7, 2 << 20]
    tensors = random_allocs(sizes, seed=31, zero=(3,))
    dense_b = sum(r16(s) for s in sizes)
    budget = 2 * dense_b + (8 << 20)
    ctx = K.Context(chunk_bytes=C, staging_budget=budget, segment_mib=segment_mib,
                    flags=K.CKPT_RESERVE_STAGING)
    ids = register_all(ctx, tensors)
    img = ctx.checkpoint()
    ref = O.checkpoint([host(t) for t in tensors], C)
    check_full(img, ref, tensors, C, ids)
    tensors[0][5000:9000] = 7
    tensors[5][-3:] = 1
    d = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=img)
    dref = O.delta([host(t) for t in tensors], C, ref["crc"])
    assert np.array_equal(d.dirty_ids, dref["dirty_ids"]) and np.array_equal(d.data, dref["delta"])
    dsts = [torch.full((t.numel(),), 0xA5, dtype=torch.uint8, device="cuda") for t in tensors]
    rc, rep = ctx.restore(img, dsts, delta=d)
    assert rc == K.CKPT_OK and rep["n_bad"] == 0
    check_restored(dsts, tensors)
    # an image larger than the reservation is refused, and nothing is allocated for it
    big = torch.empty(budget, dtype=torch.uint8, device="cuda")
    ctx.register(big)
    with pytest.raises(K.CkptError) as e:
        ctx.checkpoint()
    assert e.value.status == K.CKPT_E_BUDGET
    d.close()
    img.close()
    ctx.close()


def test_reserved_staging_needs_a_budget():
    with pytest.raises(K.CkptError) as e:
        K.Context(flags=K.CKPT_RESERVE_STAGING)
    assert e.value.status == K.CKPT_E_INVAL


# ------------------------------------------------------------------- graphs

def test_graph_replays_match_eager_and_oracle():
    """CKPT_GRAPH: the captured prologue is replayed with new tables; every
    replay equals the eager path and the oracle, with eager torch work and
    synchronizations between replays and recaptures when the table grows."""
    C = 4096
    ctx_g = K.Context(chunk_bytes=C, flags=K.CKPT_GRAPH)
    ctx_e = K.Context(chunk_bytes=C)
    tensors = random_allocs([100000, 4096 * 5 + 3, 77], seed=41)
    for t in tensors:
        ctx_g.register(t)
        ctx_e.register(t)
    for rep in range(6):
        log("graph replay %d: %d allocations" % (rep, len(tensors)))
        synth.fill_random_(tensors[rep % len(tensors)], 1000 + rep)      # eager work between replays
        if rep == 2:
            tensors[0][:8192] = 0
        torch.cuda.synchronize()
        g = ctx_g.checkpoint()
        e = ctx_e.checkpoint()
        ref = O.checkpoint([host(t) for t in tensors], C)
        check_full(g, ref, tensors, C)
        for key in ("crc", "flags", "data", "allocs"):
            assert np.array_equal(getattr(g, key), getattr(e, key)), (rep, key)
        if rep in (1, 3):                  # grow the table past the captured capacity
            extra = random_allocs([300000 * (rep + 1)] * 40, seed=500 + rep)
            for t in extra:
                ctx_g.register(t)
                ctx_e.register(t)
            tensors += extra
        if rep == 4:
            ctx_g.unregister(tensors[1])
            ctx_e.unregister(tensors[1])
            tensors.pop(1)


def test_batch_replays_and_no_graph_agree():
    C = 4096
    rng = np.random.default_rng(44)
    leader_g = K.Context(chunk_bytes=C)
    leader_n = K.Context(chunk_bytes=C, flags=K.CKPT_NO_GRAPH)
    for rep in range(3):
        members, allocs = [], []
        for i in range(5 + 4 * rep):
            sizes = [int(x) for x in rng.integers(1, 200000, int(rng.integers(1, 5)))]
            t = random_allocs(sizes, seed=rep * 100 + i)
            c = K.Context(chunk_bytes=C)
            for x in t:
                c.register(x)
            members.append(c)
            allocs.append(t)
        a = K.checkpoint_batch([leader_g] + members)
        b = K.checkpoint_batch([leader_n] + members)
        assert a[0].info()["n_allocs"] == 0
        for img_a, img_b, t in zip(a[1:], b[1:], allocs):
            ref = O.checkpoint([host(x) for x in t], C)
            check_full(img_a, ref, t, C)
            for key in ("crc", "flags", "data", "allocs"):
                assert np.array_equal(getattr(img_a, key), getattr(img_b, key)), key


def test_batch_no_drain_dense_views():
    C = 4096
    leader = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN)
    members, allocs = [], []
    for i in range(4):
        t = random_allocs([5000 * (i + 1), 4096, 17], seed=70 + i)
        c = K.Context(chunk_bytes=C)
        for x in t:
            c.register(x)
        members.append(c)
        allocs.append(t)
    imgs = K.checkpoint_batch([leader] + members)
    for img, t in zip(imgs[1:], allocs):
        ref = O.checkpoint([host(x) for x in t], C)
        assert img.info()["serialized_bytes"] == 0 and img.info()["drained"] == 0
        assert np.array_equal(img.crc, ref["crc"]) and np.array_equal(img.flags, ref["flags"])
        p, nb = img.dense_ptr
        assert_dense(d2h(p, nb), ref["dense"], [x.numel() for x in t], C, ref["flags"])


# ---------------------------------------------------------------- autotuner

def test_autotuner_shapes_match_the_oracle(tmp_path):
    """autotune.tune on a small uneven batch; then, for every chunk size it
    swept, a batch run in that size's best (waves, block, hint) shape -- the global
    best among them -- must give each context the oracle's image.  A second
    tune call with the same cache file reuses the result."""
    from paper_2008_10596_amd import autotune
    rng = np.random.default_rng(31)
    sets, hosts = [], []
    for i in range(9):
        n = int(rng.integers(1, 7))
        sizes = [int(x) for x in rng.integers(0, 700000, n)]
        t = random_allocs(sizes, seed=300 + i)
        for k, a in enumerate(t):                 # some zero 64 KiB cells
            for cell in range(0, a.numel(), 65536):
                if rng.random() < 0.2:
                    a[cell:cell + 65536] = 0
        sets.append(t)
        hosts.append([host(a) for a in t])
    alloc_sets = [[(a.data_ptr(), a.numel()) for a in t] for t in sets]
    chunks = (4096, 16384, 65536, 262144)
    cache = str(tmp_path / "tune.json")
    res = autotune.tune(alloc_sets, chunks=chunks, waves=(1, 2, 4), blocks=(256, 1024), reps=1,
                        cache_path=cache)
    assert not res["cached"]
    assert {t["chunk_bytes"] for t in res["trials"]} == set(chunks)
    best_per_c = {}
    for t in res["trials"]:
        c = t["chunk_bytes"]
        if c not in best_per_c or t["device_ms"] < best_per_c[c]["device_ms"]:
            best_per_c[c] = t
    assert res["best"] in best_per_c.values()
    assert {t["load_hint"] for t in res["trials"]} == {1, 2}
    for C, t in sorted(best_per_c.items()):
        W, B, H = t["waves_per_chunk"], t["block_threads"], t["load_hint"]
        log("C=%d: best W=%d block=%d hint=%d (%.0f GB/s)" % (C, W, B, H, t["gbps"]))
        members = []
        for tens in sets:
            c = K.Context(chunk_bytes=C)
            register_all(c, tens)
            members.append(c)
        leader = K.Context(chunk_bytes=C, waves_per_chunk=W, block_threads=B, load_hint=H)
        imgs = K.checkpoint_batch([leader] + members)
        for i, tens in enumerate(sets):
            check_full(imgs[i + 1], O.checkpoint(hosts[i], C), tens, C)
        for im in imgs:
            im.close()
        for c in members + [leader]:
            c.close()
    again = autotune.tune(alloc_sets, chunks=chunks, waves=(1, 2, 4), blocks=(256, 1024), reps=1,
                          cache_path=cache)
    assert again["cached"] and again["best"] == res["best"]


# ------------------------------------------------------------- work split

@pytest.mark.parametrize("C", [4096, 65536])
def test_consecutive_launches_on_one_plan(C):
    """The chunk and gather kernels take their tiles from counters in the
    context's plan, which each launch leaves at zero.  Launches of very
    different sizes on one context (fewer tiles than workgroups, then many;
    pack, hash-only and restore in 1 MiB segments) must each cover every
    chunk exactly: any tile left untaken shows as a CRC, flag or byte
    mismatch."""
    MiB = 1 << 20
    small = random_allocs([100], seed=51)
    large = random_allocs([9 * MiB + 3, 5 * MiB, 4096 * 7 + 5, 12 * MiB], seed=52, zero=(1,))
    large[3][2 * MiB:4 * MiB] = 0
    ctx = K.Context(chunk_bytes=C, segment_mib=1)
    for rep in range(2):
        for live in (small, large, small + large, small):
            for t in live:
                ctx.register(t)
            ref = O.checkpoint([host(t) for t in live], C)
            img = ctx.checkpoint()
            check_full(img, ref, live, C)
            live[-1][-1] ^= 0x11                     # one dirty chunk for the hash-only pass
            dref = O.delta([host(t) for t in live], C, ref["crc"])
            delta = ctx.checkpoint(mode=K.CKPT_INCREMENTAL, base=img)
            assert np.array_equal(delta.crc, dref["crc"]), rep
            assert np.array_equal(delta.flags, dref["flags"]), rep
            assert np.array_equal(delta.dirty_ids, dref["dirty_ids"]) and dref["dirty_ids"].size == 1, rep
            dsts = [torch.full_like(t, 0x3C) for t in live]
            rc, rpt = ctx.restore(img, dsts, delta=delta)
            assert rc == K.CKPT_OK and rpt["n_bad"] == 0, (rep, rpt)
            check_restored(dsts, live)
            delta.close()
            img.close()
            for t in live:
                ctx.unregister(t)
    ctx.close()


# ------------------------------------------------------------- segments

@pytest.mark.parametrize("C", [4096, 65536])
def test_segmented_drain_and_restore_equal_one_pass(C):
    """Drain and refill in 1 MiB segments (more segments than device slots, so
    slots are reused; whole segments of ZERO chunks skipped; allocations and
    outputs cut by segment bounds) give the oracle's image and memory, as one
    pass does."""
    MiB = 1 << 20
    sizes = [3 * MiB + 5, 17, 5 * MiB, 2 * MiB + 4096 * 3 + 1, 700000, 6 * MiB]
    tensors = random_allocs(sizes, seed=41, zero=(2,))
    tensors[5][MiB:3 * MiB] = 0                    # ZERO chunks inside an allocation
    hosts = [host(t) for t in tensors]
    ref = O.checkpoint(hosts, C)
    imgs = {}
    for seg in (1, 0xFFFFFFFF):
        ctx = K.Context(chunk_bytes=C, segment_mib=seg, flags=K.CKPT_TIMING)
        register_all(ctx, tensors)
        img = ctx.checkpoint()
        check_full(img, ref, tensors, C)
        t = ctx.timing()
        log("segment_mib=%d: gather %.3f ms, d2h %.3f ms, total %.3f ms"
            % (seg, t["gather_ms"], t["d2h_ms"], t["total_ms"]))
        for seg_r in (1, 0xFFFFFFFF):
            rctx = K.Context(chunk_bytes=C, segment_mib=seg_r)
            dsts = [torch.full_like(x, 0x5A) for x in tensors]
            rc, rep = rctx.restore(img, dsts)
            assert rc == K.CKPT_OK, (seg, seg_r, rep)
            check_restored(dsts, tensors)
            # a corrupted chunk in a late segment is still reported exactly
            g = int(ref["n_chunks"]) - 2
            img.crc[g] ^= 0x4
            rc, rep = rctx.restore(img, dsts)
            img.crc[g] ^= 0x4
            assert rc == K.CKPT_E_CORRUPT and rep["ids"] == [g], (seg, seg_r, rep)
            rctx.close()
        imgs[seg] = img
    for key in ("crc", "flags", "data"):
        assert np.array_equal(getattr(imgs[1], key), getattr(imgs[0xFFFFFFFF], key)), key


def test_segmented_batch_drain_cuts_outputs():
    """A batched drain in segments: a segment's bytes are cut at the
    contexts' bounds, so each context's image equals the oracle's."""
    C = 4096
    rng = np.random.default_rng(43)
    sets, hosts = [], []
    for i in range(7):
        sizes = [int(x) for x in rng.integers(1, 1500000, int(rng.integers(1, 5)))]
        t = random_allocs(sizes, seed=430 + i, zero=(0,) if i == 3 else ())
        sets.append(t)
        hosts.append([host(a) for a in t])
    members = []
    for t in sets:
        c = K.Context(chunk_bytes=C)
        register_all(c, t)
        members.append(c)
    leader = K.Context(chunk_bytes=C, segment_mib=1)
    imgs = K.checkpoint_batch([leader] + members)
    for i, t in enumerate(sets):
        check_full(imgs[i + 1], O.checkpoint(hosts[i], C), t, C)
    for im in imgs:
        im.close()
    for c in members + [leader]:
        c.close()


def test_increment_drains_on_the_side_stream():
    """An increment's delta is gathered on the caller's stream and copied to
    the host on the context's side stream; the image is complete when the call
    returns and equals the oracle's."""
    C = 4096
    tensors = random_allocs([3 << 20, 100000], seed=44)
    ctx = K.Context(chunk_bytes=C, flags=K.CKPT_TIMING)
    register_all(ctx, tensors)
    s = torch.cuda.Stream()
    base = ctx.checkpoint(stream=s)
    ref = O.checkpoint([host(t) for t in tensors], C)
    tensors[0][5 * C:7 * C] = 7
    torch.cuda.synchronize()
    d = ctx.checkpoint(stream=s, mode=K.CKPT_INCREMENTAL, base=base)
    dref = O.delta([host(t) for t in tensors], C, ref["crc"])
    assert list(d.dirty_ids) == [5, 6]
    assert np.array_equal(d.data, dref["delta"]) and np.array_equal(d.crc, dref["crc"])
    t = ctx.timing()
    assert t["d2h_ms"] > 0 and t["gather_ms"] > 0
    d.close()
    base.close()
    ctx.close()
