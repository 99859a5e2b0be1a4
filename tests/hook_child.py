"""Child process of the allocation-hook tests (run as `python -m tests.hook_child`).

torch takes a new allocator only before its first device allocation, so each
mode runs in a fresh process and prints one JSON line:

  log           install the hook, allocate and free tensors, and check that
                the context's live set is exactly the live tensors, in
                allocation order, and that the checkpoint equals the oracle's;
  save PATH     the same with address-stable memory, then write the image to
                PATH and print each tensor's address and SHA-256;
  restore PATH  without the hook, restore the image at its addresses and print
                the SHA-256 of the bytes found there;
  cache MODE    the log check with the block cache on (MODE "plain" or
                "stable"), then: a freed block is handed out again to the next
                allocation of its class, registered with its own size; with
                "stable", an image taken before a free is restored at its
                addresses while the freed block sits in the cache;
  save_cache PATH  "save" with the cache on;
  oom           the cache under memory pressure: a cached block is released
                when a new allocation does not fit beside it, and a request
                that fits only at its own size (not at its class size) gets
                a block of that size, released again when freed.
"""
import hashlib
import json
import sys

import numpy as np
import torch

from paper_2008_10596_amd import ckpt as K

C = 4096


def tensors():
    """Seeded tensors, some freed again, made with elementwise ops only (no
    library workspaces).  Returns the live ones in allocation order."""
    g = torch.Generator(device="cuda")
    g.manual_seed(12701)
    a = torch.randn(1000, generator=g, device="cuda")
    b = torch.zeros(5000, dtype=torch.uint8, device="cuda")
    tmp = a * 3.0
    c = torch.arange(70000, dtype=torch.int32, device="cuda")
    d = (tmp + 1.0).sin()
    del tmp
    e = torch.randint(0, 256, (3 * 4096 + 17,), dtype=torch.uint8, generator=g, device="cuda")
    f = torch.empty(64, dtype=torch.float64, device="cuda").fill_(2.5)
    del c
    w = torch.nn.Parameter(torch.randn(64, 32, generator=g, device="cuda"))
    torch.cuda.synchronize()
    return [a, b, d, e, f, w]


def host_bytes(t):
    return t.detach().contiguous().view(torch.uint8).reshape(-1).cpu().numpy()


def check(ctx, live, img):
    from oracle import oracle as O
    from paper_2008_10596_amd import hook
    st = hook.stats()
    ref = O.checkpoint([host_bytes(t) for t in live], C)
    return {
        "live_count": ctx.live_count(), "n_live": len(live),
        "stats_live": st["allocs"] - st["frees"], "failures": st["failures"],
        "order": [int(x) for x in img.addrs] == [t.data_ptr() for t in live],
        "crc": bool(np.array_equal(img.crc, ref["crc"])),
        "flags": bool(np.array_equal(img.flags, ref["flags"])),
        "data": bool(np.array_equal(img.data, ref["serialized"])),
    }


def run_log():
    from paper_2008_10596_amd import hook
    ctx = K.Context(chunk_bytes=C)
    hook.install(ctx)
    live = tensors()
    img = ctx.checkpoint()
    out = check(ctx, live, img)
    del live
    torch.cuda.synchronize()
    out["after_free"] = ctx.live_count()
    print(json.dumps(out), flush=True)


def run_cache(mode):
    from paper_2008_10596_amd import hook
    from tests.gpu_common import d2h
    stable = mode == "stable"
    ctx = K.Context(chunk_bytes=C)
    hook.install(ctx, address_stable=stable, cache=True)
    live = tensors()
    img = ctx.checkpoint()
    out = check(ctx, live, img)
    sha0 = [hashlib.sha256(host_bytes(t).tobytes()).hexdigest() for t in live]
    cs = hook.cache_stats()
    out["cached_after_frees"] = cs["blocks"]
    # the freed block of e comes back for the next allocation of its size
    e = live.pop(3)
    pe, ne = e.data_ptr(), e.numel()
    del e
    torch.cuda.synchronize()
    h0 = hook.cache_stats()["hits"]
    x = torch.full((ne - 5,), 9, dtype=torch.uint8, device="cuda")
    out["reused"] = x.data_ptr() == pe
    out["hit"] = hook.cache_stats()["hits"] == h0 + 1
    torch.cuda.synchronize()
    out["after_reuse"] = check(ctx, live + [x], ctx.checkpoint())
    # a block freed on one stream is handed out again on that stream only
    side = torch.cuda.Stream()
    n2 = 70000
    with torch.cuda.stream(side):
        y = torch.empty(n2, dtype=torch.uint8, device="cuda")
        py = y.data_ptr()
        del y
    zt = torch.empty(n2, dtype=torch.uint8, device="cuda")   # default stream
    out["other_stream_fresh"] = zt.data_ptr() != py
    with torch.cuda.stream(side):
        y2 = torch.empty(n2, dtype=torch.uint8, device="cuda")
        out["same_stream_reused"] = y2.data_ptr() == py
        del y2
    del zt
    torch.cuda.synchronize()
    if stable:
        # x's block goes back to the cache; the image still has e at that address
        del x
        torch.cuda.synchronize()
        rc, rep, addrs = ctx.restore_at(img)
        sizes = [int(v) for v in img.allocs["size"]]
        out["restore_rc"] = rc
        out["restore_bad"] = rep["n_bad"]
        out["restore_addrs"] = addrs == [int(a) for a in img.addrs]
        out["restore_sha"] = [hashlib.sha256(d2h(p, n).tobytes()).hexdigest() for p, n in zip(addrs, sizes)] == sha0
        out["cached_after_restore"] = hook.cache_stats()["blocks"]
    else:
        del x
        torch.cuda.synchronize()
    out["cached_before_trim"] = hook.cache_stats()["blocks"]
    out["trimmed"] = hook.trim()
    out["cached_after_trim"] = hook.cache_stats()["blocks"]
    del live
    torch.cuda.synchronize()
    out["live_at_end"] = ctx.live_count()
    print(json.dumps(out), flush=True)


def class_bytes(b):
    """The cache's size class of a request (four classes per power of two)."""
    if b <= 512:
        return 512
    e = (b - 1).bit_length() - 1
    step = 1 << (e - 2)
    return -(-b // step) * step


def run_oom():
    from paper_2008_10596_amd import hook
    ctx = K.Context(chunk_bytes=C)
    hook.install(ctx, cache=True)
    free, _ = torch.cuda.mem_get_info()
    out = {"free": free}
    a = torch.empty(int(0.4 * free), dtype=torch.uint8, device="cuda")
    del a
    torch.cuda.synchronize()
    out["cached_a"] = hook.cache_stats()["blocks"]
    b = torch.empty(int(0.7 * free), dtype=torch.uint8, device="cuda")   # does not fit beside a's block
    out["after_b"] = {"cached": hook.cache_stats()["blocks"], "live": ctx.live_count()}
    del b
    torch.cuda.synchronize()
    out["trimmed_b"] = hook.trim() > 0
    # a request below the free memory whose class is above it
    free2, _ = torch.cuda.mem_get_info()
    r = free2 - (4 << 30)
    while r > free2 // 2 and class_bytes(r) <= free2:
        r -= 1 << 30
    out["exact_case"] = class_bytes(r) > free2
    if out["exact_case"]:
        d = torch.empty(r, dtype=torch.uint8, device="cuda")
        out["after_d"] = {"cached": hook.cache_stats()["blocks"], "live": ctx.live_count()}
        del d
        torch.cuda.synchronize()
    out["end"] = {"cached": hook.cache_stats()["blocks"], "live": ctx.live_count()}
    out["failures"] = hook.stats()["failures"]
    print(json.dumps(out), flush=True)


def run_save(path, cache=False):
    from paper_2008_10596_amd import hook
    ctx = K.Context(chunk_bytes=C)
    hook.install(ctx, address_stable=True, cache=cache)
    live = tensors()
    img = ctx.checkpoint()
    out = check(ctx, live, img)
    img.write_file(path)
    out["addrs"] = [t.data_ptr() for t in live]
    out["sha"] = [hashlib.sha256(host_bytes(t).tobytes()).hexdigest() for t in live]
    print(json.dumps(out), flush=True)


def run_restore(path):
    from tests.gpu_common import d2h
    ctx = K.Context(chunk_bytes=C)
    rc, rep, addrs, img = ctx.restore_file_at(path)
    sizes = [int(s) for s in img.allocs["size"]]
    sha = [hashlib.sha256(d2h(p, s).tobytes()).hexdigest() for p, s in zip(addrs, sizes)]
    print(json.dumps({"rc": rc, "n_bad": rep["n_bad"], "addrs": addrs, "sha": sha}), flush=True)


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "log":
        run_log()
    elif mode == "save":
        run_save(sys.argv[2])
    elif mode == "save_cache":
        run_save(sys.argv[2], cache=True)
    elif mode == "cache":
        run_cache(sys.argv[2])
    elif mode == "oom":
        run_oom()
    else:
        run_restore(sys.argv[2])
