"""Autotuner for the batched checkpoint (ckpt_checkpoint_batch).

Sweeps chunk size C, waves per chunk W, workgroup size and the load/store
hint (non-temporal or regular) on the caller's own contexts' allocations, timing the device part of one batched checkpoint (the
replayed graph: table upload, size scan, chunk map, fused pack + CRC + flags)
with the image kept in HBM; the best shape is the fastest.  Each trial also
reports GB/s of the bytes its kernel form moves (one wave per chunk of at most
4 KiB leaves ZERO chunks unwritten; the other forms write every chunk).  For every C, every (W, block) must give the
same CRC and flag arrays -- the launch shape may not change a result -- or
the tuner raises.  Results are cached by device and by a coarse signature of
the workload (context count, total bytes and median allocation size, each
bucketed by powers of two), so a later run on a similar workload reuses them.

A different C gives a different image (another chunk grid); choosing C is a
trade-off the caller makes (larger chunks: faster packing, coarser dirty
tracking for incremental checkpoints).
"""
import hashlib
import json
import math
import os
import statistics
import time

from . import ckpt as K

DEFAULT_CHUNKS = (4096, 16384, 65536, 262144)
DEFAULT_WAVES = (1, 2, 4, 8)
DEFAULT_BLOCKS = (256, 512, 1024)
# ckpt_config.load_hint: 2 non-temporal, 1 regular.  Non-temporal is faster
# where the dense image's chunks start on 128-byte lines; regular where most
# of them do not (many allocations of arbitrary sizes), as in a batch.
DEFAULT_HINTS = (2, 1)


def signature(alloc_sets):
    sizes = sorted(s for allocs in alloc_sets for _, s in allocs)
    total = sum(sizes)
    med = sizes[len(sizes) // 2] if sizes else 0
    b = lambda x: int(math.log2(x)) if x > 0 else -1  # noqa: E731
    return "ctx2^%d:bytes2^%d:median2^%d" % (b(len(alloc_sets)), b(total), b(med))


def device_key(device=0):
    import torch
    p = torch.cuda.get_device_properties(device)
    return "%s:%dcu" % (p.name, p.multi_processor_count)


def _stored(alloc_sets, C, imgs):
    """Bytes of the non-ZERO chunks, each rounded up to 16."""
    import numpy as np
    total = 0
    for allocs, img in zip(alloc_sets, imgs):
        sizes = [s for _, s in allocs if s]
        if not sizes:
            continue
        lens = np.concatenate([np.minimum(C, s - np.arange(0, s, C, dtype=np.int64)) for s in sizes])
        nz = (img.flags[:lens.size] & 1) == 0
        total += int(((lens[nz] + 15) // 16 * 16).sum())
    return total


def _digest(imgs):
    h = hashlib.sha256()
    for img in imgs:
        h.update(img.crc.tobytes())
        h.update(img.flags.tobytes())
    return h.hexdigest()


def tune(alloc_sets, chunks=DEFAULT_CHUNKS, waves=DEFAULT_WAVES, blocks=DEFAULT_BLOCKS, reps=3,
         device=0, stream=None, cache_path=None, log=None, hints=DEFAULT_HINTS):
    """alloc_sets: one list of (device address, bytes) per context.
    Returns {"best": {...}, "trials": [...], "cached": bool}."""
    key = "%s|%s|hints%s" % (device_key(device), signature(alloc_sets), ",".join(str(h) for h in hints))
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return dict(cache[key], cached=True)
    live = sum(s for allocs in alloc_sets for _, s in allocs)
    trials = []
    for C in chunks:
        members = []
        for allocs in alloc_sets:
            c = K.Context(device=device, chunk_bytes=C)
            for p, s in allocs:
                c.register(p, s)
            members.append(c)
        N = sum((s + C - 1) // C for allocs in alloc_sets for _, s in allocs)
        dense = sum((s + 15) // 16 * 16 for allocs in alloc_sets for _, s in allocs)
        stored = None
        ref = None
        for W in waves:
            for B in blocks:
                for H in hints:
                    if W > B // 64 or (C + 1023) // 1024 < W:
                        continue
                    leader = K.Context(device=device, chunk_bytes=C, flags=K.CKPT_NO_DRAIN | K.CKPT_TIMING,
                                       waves_per_chunk=W, block_threads=B, load_hint=H)
                    imgs = K.checkpoint_batch([leader] + members, stream=stream)   # capture + warm
                    d = _digest(imgs[1:])
                    if stored is None:
                        stored = _stored(alloc_sets, C, imgs[1:])
                    if ref is None:
                        ref = d
                    elif d != ref:
                        raise RuntimeError("C=%d W=%d block=%d hint=%d changed the result" % (C, W, B, H))
                    for im in imgs:
                        im.close()
                    ms = []
                    for _ in range(reps):
                        t0 = time.perf_counter()
                        imgs = K.checkpoint_batch([leader] + members, stream=stream)
                        wall = (time.perf_counter() - t0) * 1e3
                        ms.append(leader.timing()["pack_ms"])
                        for im in imgs:
                            im.close()
                    t = statistics.median(ms)
                    alg = live + (stored if W == 1 and C <= 4096 else dense) + 5 * N
                    trial = {"chunk_bytes": C, "waves_per_chunk": W, "block_threads": B, "load_hint": H,
                             "device_ms": round(t, 4), "gbps": round(alg / (t * 1e-3) / 1e9, 2),
                             "wall_ms": round(wall, 3)}
                    trials.append(trial)
                    if log:
                        log("autotune %s" % trial)
                    leader.close()
        for c in members:
            c.close()
    best = min(trials, key=lambda t: t["device_ms"])
    out = {"best": best, "trials": trials, "key": key}
    if cache_path:
        cache[key] = out
        d = os.path.dirname(os.path.abspath(cache_path))
        os.makedirs(d, exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return dict(out, cached=False)
