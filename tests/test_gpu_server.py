"""The serving loop (continuous batching): each request's result is the same
alone and in a mix, equal to the plain path and to the oracle."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2008_10596_amd import ckpt as K
from tests.gpu_common import (check_full, check_restored, h2d, host, log, managed_alloc, managed_free,
                              prefetch_to_host, random_allocs)

pytestmark = pytest.mark.gpu
C = 4096


def make_requests(seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(10):
        n = int(rng.integers(1, 9))
        sizes = [int(x) for x in rng.integers(0, 3 << 20, n)]
        sizes[0] = int(rng.integers(1, 50000))
        zero = (1,) if i % 3 == 0 and n > 1 else ()
        reqs.append(random_allocs(sizes, seed=seed * 100 + i, zero=zero))
    return reqs


def image_arrays(img):
    return {k: getattr(img, k).copy() for k in ("crc", "flags", "data", "allocs")}


def run_server(srv, items):
    """items: list of (op, bufs, image); submits all, then waits for all."""
    tickets = [srv.submit(op, bufs, image=img) for op, bufs, img in items]
    return [srv.wait(t) for t in tickets]


def test_server_alone_equals_mix_and_plain():
    reqs = make_requests(21)
    # images to restore from, taken with the plain path
    plain_imgs = []
    for bufs in reqs[:4]:
        ctx = K.Context(chunk_bytes=C)
        for b in bufs:
            ctx.register(b)
        plain_imgs.append(ctx.checkpoint())
    restore_dsts = [[torch.full_like(b, 0x77) for b in bufs] for bufs in reqs[:4]]
    items = [(K.CKPT_REQ_CHECKPOINT, bufs, None) for bufs in reqs]
    items += [(K.CKPT_REQ_RESTORE, d, img) for d, img in zip(restore_dsts, plain_imgs)]

    # alone: one request at a time
    srv = K.Server(chunk_bytes=C, staging_budget=1 << 30, step_bytes=1 << 20)
    alone = []
    for it in items:
        r = run_server(srv, [it])[0]
        assert r["status"] == K.CKPT_OK, r
        alone.append(image_arrays(r["image"]) if r["image"] else [host(d) for d in it[1]])
    srv.close()
    for d, bufs in zip(restore_dsts, reqs[:4]):
        check_restored(d, bufs)
        for x in d:
            x.fill_(0x33)

    # mix: everything at once, small steps and a budget that forces queueing
    srv = K.Server(chunk_bytes=C, staging_budget=64 << 20, step_bytes=256 << 10, max_active=6)
    mixed = run_server(srv, items)
    st = srv.stats()
    log("server mix stats: %s" % st)
    assert st["completed"] == len(items) and st["failed"] == 0
    assert st["max_concurrent"] > 1 and st["steps"] > len(items)
    srv.close()
    for i, (r, it) in enumerate(zip(mixed, items)):
        assert r["status"] == K.CKPT_OK, (i, r)
        if it[0] == K.CKPT_REQ_CHECKPOINT:
            got = image_arrays(r["image"])
            for key in ("crc", "flags", "data", "allocs"):
                assert np.array_equal(got[key], alone[i][key]), (i, key)
        else:
            for a, b in zip([host(d) for d in it[1]], alone[i]):
                assert np.array_equal(a, b), i
    for d, bufs in zip(restore_dsts, reqs[:4]):
        check_restored(d, bufs)
    # checkpoint results equal the oracle (and the plain path's images)
    for i, bufs in enumerate(reqs):
        ref = O.checkpoint([host(b) for b in bufs], C)
        img = mixed[i]["image"]
        check_full(img, ref, bufs, C, ids=list(range(1, len(bufs) + 1)))
        if i < 4:
            for key in ("crc", "flags", "data"):
                assert np.array_equal(getattr(img, key), getattr(plain_imgs[i], key))


def test_server_restore_reports_corruption():
    bufs = random_allocs([100000, 5000], seed=5)
    ctx = K.Context(chunk_bytes=C)
    for b in bufs:
        ctx.register(b)
    img = ctx.checkpoint()
    img.data[4096 * 3 + 5] ^= 1
    srv = K.Server(chunk_bytes=C, staging_budget=64 << 20)
    dsts = [torch.empty_like(b) for b in bufs]
    r = srv.wait(srv.submit(K.CKPT_REQ_RESTORE, dsts, image=img))
    assert r["status"] == K.CKPT_E_CORRUPT and r["n_bad"] == 1
    srv.close()


def test_server_errors():
    srv = K.Server(chunk_bytes=C, staging_budget=8 << 20)
    big = torch.empty(16 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(K.CkptError) as e:
        srv.submit(K.CKPT_REQ_CHECKPOINT, [big])
    assert e.value.status == K.CKPT_E_BUDGET
    with pytest.raises(K.CkptError) as e:
        srv.submit(K.CKPT_REQ_CHECKPOINT, [big.data_ptr() + 8], sizes=[64])
    assert e.value.status == K.CKPT_E_INVAL
    small = random_allocs([1000, 2000], seed=9)
    ctx = K.Context(chunk_bytes=C)
    for b in small:
        ctx.register(b)
    img = ctx.checkpoint()
    with pytest.raises(K.CkptError) as e:
        srv.submit(K.CKPT_REQ_RESTORE, [torch.empty(1000, dtype=torch.uint8, device="cuda")], image=img)
    assert e.value.status == K.CKPT_E_MISMATCH
    with pytest.raises(K.CkptError) as e:
        srv.poll(12345)
    assert e.value.status == K.CKPT_E_NOTFOUND
    t = srv.submit(K.CKPT_REQ_CHECKPOINT, small)
    r = srv.wait(t)
    assert r["status"] == K.CKPT_OK
    with pytest.raises(K.CkptError) as e:
        srv.poll(t)                                    # retired
    assert e.value.status == K.CKPT_E_NOTFOUND
    srv.close()


def test_managed_allocations_checkpoint_and_restore():
    """Managed (hipMallocManaged) allocations, some pages moved host-side
    first, are captured like device memory (plain path and server)."""
    rng = np.random.default_rng(31)
    sizes = [3 << 20, 5000, 2 << 20]
    hosts = [rng.integers(0, 256, s, dtype=np.uint8) for s in sizes]
    ptrs = [managed_alloc(s) for s in sizes]
    try:
        for p, h in zip(ptrs, hosts):
            h2d(p, h)
        moved = prefetch_to_host(ptrs[0], 1 << 20)
        log("managed prefetch to host supported: %s" % moved)
        ref = O.checkpoint(hosts, C)
        ctx = K.Context(chunk_bytes=C)
        for p, s in zip(ptrs, sizes):
            ctx.register(p, s, kind=K.CKPT_MANAGED)
        img = ctx.checkpoint()
        assert np.array_equal(img.crc, ref["crc"]) and np.array_equal(img.data, ref["serialized"])
        assert list(img.allocs["kind"]) == [K.CKPT_MANAGED] * 3
        srv = K.Server(chunk_bytes=C, staging_budget=64 << 20)
        r = srv.wait(srv.submit(K.CKPT_REQ_CHECKPOINT, ptrs, sizes=sizes, kinds=[K.CKPT_MANAGED] * 3))
        assert r["status"] == K.CKPT_OK
        assert np.array_equal(r["image"].crc, ref["crc"]) and np.array_equal(r["image"].data, ref["serialized"])
        dsts = [torch.empty(s, dtype=torch.uint8, device="cuda") for s in sizes]
        rc, _ = ctx.restore(img, dsts)
        assert rc == K.CKPT_OK
        for d, h in zip(dsts, hosts):
            assert np.array_equal(host(d), h)
        srv.close()
    finally:
        torch.cuda.synchronize()
        for p in ptrs:
            managed_free(p)


def test_server_host_budget_queues_checkpoints():
    """A checkpoint is admitted only while the pinned bytes handed out (images
    the caller holds included) plus the admitted checkpoints' charges plus its
    own stay within the host budget.  With room for two images: A and B run,
    C waits while their images are held, a restore R behind C passes it, and
    C and D run once A's and B's images are freed.  Every image equals the
    oracle's."""
    import gc
    import time
    MiB = 1 << 20
    reqs = [random_allocs([16 * MiB] * 4, seed=700 + i) for i in range(4)]      # A, B, C, D
    hosts = [[host(b) for b in bufs] for bufs in reqs]
    ctx = K.Context(chunk_bytes=C)
    small = random_allocs([300000, 5000], seed=710)
    for b in small:
        ctx.register(b)
    rimg = ctx.checkpoint()                                   # the image R restores from
    srv = K.Server(chunk_bytes=C, staging_budget=1 << 30, aux_threads=1, host_budget=1 << 40)
    srv.wait(srv.submit(K.CKPT_REQ_CHECKPOINT, small))["image"].close()   # server buffers warm
    srv.close()
    gc.collect()
    gc.disable()
    try:
        data = 64 * MiB
        N = data // C
        charge = data + data // 4 + 5 * N + (5 * N) // 4 + 8 * MiB + 64
        base, _ = K.host_memory()
        budget = base + 2 * charge + 4 * MiB + 8 * MiB       # two charges, server buffers, slack
        log("host memory: live %d B before; charge %d B; budget %d B" % (base, charge, budget))
        srv = K.Server(chunk_bytes=C, staging_budget=1 << 30, aux_threads=1, host_budget=budget)
        dsts = [torch.full_like(b, 0x77) for b in small]
        ta = srv.submit(K.CKPT_REQ_CHECKPOINT, reqs[0])
        tb = srv.submit(K.CKPT_REQ_CHECKPOINT, reqs[1])
        tc = srv.submit(K.CKPT_REQ_CHECKPOINT, reqs[2])
        tr = srv.submit(K.CKPT_REQ_RESTORE, dsts, image=rimg)
        td = srv.submit(K.CKPT_REQ_CHECKPOINT, reqs[3])
        ra, rb = srv.wait(ta), srv.wait(tb)
        assert ra["status"] == K.CKPT_OK and rb["status"] == K.CKPT_OK
        rr = srv.wait(tr)                                     # passes the waiting checkpoint
        assert rr["status"] == K.CKPT_OK
        check_restored(dsts, small)
        time.sleep(0.3)
        assert srv.poll(tc) is None, "C ran while A's and B's images were held"
        assert srv.poll(td) is None
        st = srv.stats()
        log("held: %s" % st)
        assert st["host_waits"] >= 1 and st["host_peak"] <= budget
        ra["image"].close()
        rb["image"].close()
        rc_, rd = srv.wait(tc), srv.wait(td)
        assert rc_["status"] == K.CKPT_OK and rd["status"] == K.CKPT_OK
        for i, r in enumerate((ra, rb, rc_, rd)):
            if i >= 2:
                check_full(r["image"], O.checkpoint(hosts[i], C), reqs[i], C, ids=[1, 2, 3, 4])
                r["image"].close()
        assert srv.stats()["failed"] == 0
        srv.close()
        # a checkpoint that can never fit the host budget is refused at submit
        # (its device staging fits)
        srv = K.Server(chunk_bytes=C, staging_budget=1 << 30, host_budget=8 * MiB)
        with pytest.raises(K.CkptError) as e:
            srv.submit(K.CKPT_REQ_CHECKPOINT, reqs[0][:1])
        assert e.value.status == K.CKPT_E_BUDGET
        srv.close()
    finally:
        gc.enable()
    rimg.close()
    ctx.close()
