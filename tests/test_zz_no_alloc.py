"""The allocation-free entry point (ckpt_checkpoint_noalloc), through the C
ABI, against ckpt_checkpoint on the same registrations (dense image, CRC and
flag arrays, bit for bit) and against the oracle: two calls in a row, the
second with a smaller input, incremental passes, and the size and argument
errors."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from paper_2008_10596_amd import ckpt as K
from tests.gpu_common import assert_dense, d2h, host, log, random_allocs, register_all

pytestmark = pytest.mark.gpu

SENT_DENSE, SENT_FLAG, SENT_CRC = 0x5A, 0xEE, 0x13579BDF


def outputs(n_chunks, dense_bytes, slack=4096):
    """Output buffers larger than needed, filled with sentinels."""
    dense = torch.full((dense_bytes + slack,), SENT_DENSE, dtype=torch.uint8, device="cuda")
    crc = torch.full((n_chunks + 7,), SENT_CRC, dtype=torch.int32, device="cuda")
    flags = torch.full((n_chunks + 7,), SENT_FLAG, dtype=torch.uint8, device="cuda")
    return dense, crc, flags


def existing(ctx, mode=K.CKPT_FULL, base=None):
    """ckpt_checkpoint on the same context: (dense bytes, crc, flags)."""
    img = ctx.checkpoint(mode=mode, base=base)
    dense = None
    if mode == K.CKPT_FULL:
        p, nb = img.dense_ptr
        dense = d2h(p, nb)
    return img, dense, img.crc.copy(), img.flags.copy()


def check_against(ctx, tensors, C, dense_t, crc_t, flags_t, N, D, base_img=None, mode=K.CKPT_FULL):
    torch.cuda.synchronize()
    img, dense_e, crc_e, flags_e = existing(ctx, mode=mode, base=base_img)
    crc_n = crc_t.cpu().numpy().view(np.uint32)
    flags_n = flags_t.cpu().numpy()
    assert np.array_equal(crc_n[:N], crc_e), "CRC differs from ckpt_checkpoint"
    assert np.array_equal(flags_n[:N], flags_e), "flags differ from ckpt_checkpoint"
    assert (crc_n[N:] == SENT_CRC).all() and (flags_n[N:] == SENT_FLAG).all(), "wrote past N"
    if mode == K.CKPT_FULL:
        # the dense images agree on every byte but those of ZERO chunks, which
        # the pack may leave unwritten
        sizes = [t.numel() for t in tensors]
        dense_n = dense_t.cpu().numpy()
        assert_dense(dense_n[:D], dense_e, sizes, C, flags_e)
        assert (dense_n[D:] == SENT_DENSE).all(), "wrote past the dense image"
        ref = O.checkpoint([host(t) for t in tensors], C)
        assert np.array_equal(crc_n[:N], ref["crc"])
        assert_dense(dense_n[:D], ref["dense"][:D], sizes, C, ref["flags"])
        if base_img is None:
            assert np.array_equal(flags_n[:N], ref["flags"])
    return img


@pytest.mark.parametrize("C", [4096, 1024, 65536])
def test_two_calls_second_smaller_match_checkpoint(C):
    log("noalloc: two calls, C=%d" % C)
    rng = np.random.default_rng(C)
    sizes = [int(x) for x in synth.log_uniform(rng, 72, 256, 4 << 20)] + [0, 1, 17, 4097, 65537]
    tensors = random_allocs(sizes, seed=C + 1, zero=(3, 40))
    tensors[10][: min(8192, tensors[10].numel())] = 0
    ctx = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN | K.CKPT_KEEP_DENSE)
    register_all(ctx, tensors)
    N, D = ctx.noalloc_sizes()
    log("  first: %d allocations, %d chunks, %d bytes" % (len(tensors), N, D))
    dense, crc, flags = outputs(N, D)
    s = torch.cuda.Stream()
    assert ctx.checkpoint_noalloc(crc, flags, dense=dense, stream=s) == (N, D)
    s.synchronize()
    img1 = check_against(ctx, tensors, C, dense, crc, flags, N, D)
    img1.close()
    # the second call: a smaller input (allocations released), into the same
    # buffers re-filled with sentinels; the array keeps the first call's contents
    for t in tensors[::2]:
        ctx.unregister(t)
    kept = tensors[1::2]
    N2, D2 = ctx.noalloc_sizes()
    assert N2 < N and D2 < D
    dense.fill_(SENT_DENSE)
    crc.fill_(SENT_CRC)
    flags.fill_(SENT_FLAG)
    log("  second: %d allocations, %d chunks, %d bytes" % (len(kept), N2, D2))
    assert ctx.checkpoint_noalloc(crc, flags, dense=dense, stream=s) == (N2, D2)
    s.synchronize()
    img2 = check_against(ctx, kept, C, dense, crc, flags, N2, D2)
    img2.close()
    ctx.close()


def test_two_contexts_share_the_array_in_order():
    """A large pass on one context, then a smaller one on another, on one
    stream: each equals its own context's ckpt_checkpoint."""
    C = 4096
    big = random_allocs([3 << 20, 1 << 20, 12345, 77 << 10], seed=5)
    small = random_allocs([4096, 100], seed=6)
    ca = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN | K.CKPT_KEEP_DENSE)
    cb = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN | K.CKPT_KEEP_DENSE)
    register_all(ca, big)
    register_all(cb, small)
    Na, Da = ca.noalloc_sizes()
    Nb, Db = cb.noalloc_sizes()
    oa, ob = outputs(Na, Da), outputs(Nb, Db)
    s = torch.cuda.Stream()
    ca.checkpoint_noalloc(oa[1], oa[2], dense=oa[0], stream=s)
    cb.checkpoint_noalloc(ob[1], ob[2], dense=ob[0], stream=s)
    s.synchronize()
    check_against(ca, big, C, *oa, Na, Da).close()
    check_against(cb, small, C, *ob, Nb, Db).close()
    ca.close()
    cb.close()


@pytest.mark.parametrize("C", [4096, 65536])
def test_dirty_and_incremental_against_a_base(C):
    log("noalloc: base CRC and hash-only pass, C=%d" % C)
    tensors = random_allocs([5 << 20, 300000, 4096 * 3 + 5, 1 << 20], seed=C + 9)
    ctx = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN | K.CKPT_KEEP_DENSE)
    register_all(ctx, tensors)
    N, D = ctx.noalloc_sizes()
    base = ctx.checkpoint()
    base_crc = torch.from_numpy(base.crc.view(np.int32).copy()).to("cuda")
    tensors[0][C * 3 + 17] ^= 0xFF
    tensors[2][-1] ^= 1
    tensors[3][: C] = 0
    # FULL with a base: DIRTY against it
    dense, crc, flags = outputs(N, D)
    ctx.checkpoint_noalloc(crc, flags, dense=dense, base_crc=base_crc)
    check_against(ctx, tensors, C, dense, crc, flags, N, D, base_img=base).close()
    # INCREMENTAL: the hash-only pass (no dense image)
    _, crc2, flags2 = outputs(N, 0)
    assert ctx.checkpoint_noalloc(crc2, flags2, base_crc=base_crc, mode=K.CKPT_INCREMENTAL) == (N, D)
    torch.cuda.synchronize()
    img = check_against(ctx, tensors, C, None, crc2, flags2, N, D, base_img=base, mode=K.CKPT_INCREMENTAL)
    assert (flags2.cpu().numpy()[:N] & 2).sum() >= 3
    img.close()
    base.close()
    ctx.close()


def test_sizes_and_errors():
    C = 4096
    tensors = random_allocs([10000, 4096, 0], seed=3)
    ctx = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN)
    register_all(ctx, tensors)
    N, D = ctx.noalloc_sizes()
    assert (N, D) == (3 + 1, 10000 + 4096)
    dense, crc, flags = outputs(N, D)
    with pytest.raises(K.CkptError) as e:
        ctx.checkpoint_noalloc(crc, flags, dense=dense, dense_bytes=D - 1)
    assert e.value.status == K.CKPT_E_MISMATCH
    with pytest.raises(K.CkptError) as e:
        ctx.checkpoint_noalloc(crc, flags, dense=dense, chunk_cap=N - 1)
    assert e.value.status == K.CKPT_E_MISMATCH
    with pytest.raises(K.CkptError) as e:
        ctx.checkpoint_noalloc(crc, flags, mode=K.CKPT_INCREMENTAL)
    assert e.value.status == K.CKPT_E_INVAL
    with pytest.raises(K.CkptError) as e:
        ctx.checkpoint_noalloc(crc, flags, dense=dense[1:])
    assert e.value.status == K.CKPT_E_INVAL
    # sentinels untouched by the refused calls
    torch.cuda.synchronize()
    assert (flags.cpu().numpy() == SENT_FLAG).all() and (dense.cpu().numpy() == SENT_DENSE).all()
    ctx.close()
    # more allocations than the array holds: refused before any device work
    many = K.Context(chunk_bytes=C)
    base_addr = 1 << 40
    for k in range(65537):
        many.register(base_addr + 16 * k, 0)
    with pytest.raises(K.CkptError) as e:
        many.checkpoint_noalloc(crc, flags, dense=dense)
    assert e.value.status == K.CKPT_E_BUDGET
    many.close()
