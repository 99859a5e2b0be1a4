"""Benchmark of the checkpoint drain/refill path on one MI355X.

Headline workload (the JSON `value`): full checkpoint at scale -- 4096
allocations, log-uniform 4 KiB - 64 MiB scaled to 16 GiB, half of them all-zero,
C = 4 KiB.  One step is one ckpt_checkpoint of the whole live set with the
image kept in HBM (CKPT_NO_DRAIN): descriptor upload, size scan, chunk map,
the fused pack + CRC-32C + ZERO/DIRTY kernel, and the CRC/flag arrays copied to
the host.  `value` = algorithmic bytes of a step (every live byte read, the
dense image written, 5 bytes of CRC + flags per chunk) / wall time per step.

The same run then measures, and reports inside the one JSON line: the drain
of that image to pinned host memory and the restore from it; the incremental
workload (hash-only pass + delta); the batched workload (512 contexts, plain
per-allocation and per-context forms against one graph-replayed batched
launch, plus the autotuner sweep); and the serving workload (Poisson arrivals,
p50/p99 latency), each on seeded synthetic inputs generated on the device.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
LINK_PEAK = 64.0e9         # B/s per direction, PCIe 5.0 x16
METRIC = "pack+CRC32C GB/s (% HBM peak), batched vs plain; p50/p99 ckpt latency"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the 16 GiB total (quick runs)")
    ap.add_argument("--chunk", type=int, default=4096)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--wpc", type=int, default=0)
    ap.add_argument("--wgs-per-cu", type=int, default=0)
    ap.add_argument("--load-hint", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the timed pack steps")
    ap.add_argument("--batched-no-graph", action="store_true",
                    help="batched section: plain launches of the same kernels instead of the replayed graph")
    ap.add_argument("--batched-only-graph", action="store_true",
                    help="batched section: the graph-replayed batch only (no plain forms, drain or autotuner; "
                         "profiler runs)")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the copy reference and the plain read/write/copy ceiling sweep (profiler runs)")
    ap.add_argument("--drain-steps", type=int, default=5)
    ap.add_argument("--only", default="", help="comma list of extra sections to run "
                    "(drain,restore_at,incremental,batched,serving,hook); default: all")
    ap.add_argument("--serving-requests", type=int, default=200, help="measured requests per rate")
    ap.add_argument("--serving-rates", default="10,25,50,100,150,200", help="arrival rates (req/s)")
    ap.add_argument("--serving-shapes", type=int, default=24)
    ap.add_argument("--serving-warmup", type=int, default=20, help="warm-up requests per rate")
    ap.add_argument("--serving-host-budget-gib", type=float, default=0,
                    help="server host budget for images (0: the library's default)")
    ap.add_argument("--sections-only", action="store_true",
                    help="diagnostic runs (e.g. counter passes): skip the headline at-scale steps and "
                         "print only the --only sections as JSON")
    ap.add_argument("--hook-child", default="", help=argparse.SUPPRESS)   # internal: one hook timing run
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after the timed steps, one plain device copy of this many bytes "
                         "(calibrates hardware byte counters against a known size)")
    return ap.parse_args()


def tune_kw(args):
    """Launch-configuration overrides from the command line (0 = library default)."""
    return dict(block_threads=args.block, waves_per_chunk=args.wpc, wgs_per_cu=args.wgs_per_cu,
                load_hint=args.load_hint)


def profiled_traffic(summary_glob="k_chunks_pack_*.md"):
    """HBM bytes per launch of the pack kernel from the committed rocprofv3
    counter summary (profiles/), if it was taken from the current kernel
    source; None otherwise."""
    import glob
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_2008_10596_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in glob.glob(os.path.join(ROOT, "profiles", summary_glob)):
        m = re.search(r"machine-readable: traffic_bytes=(\d+) alg_bytes=(\d+) avg_ms=([\d.]+) "
                      r"kernels_sha256=(\w+)", open(path).read())
        if m and m.group(4) == sha:
            return int(m.group(1)), int(m.group(2)), os.path.basename(path)
    return None


def algorithmic_bytes(sizes, C, flags=None):
    """(S, dense, N, alg) of a pack launch: every live byte read, the dense
    image written, 5 bytes of CRC + flags per chunk.  With the chunks' flags
    (the one-wave pack of chunks of at most 4 KiB, which leaves ZERO chunks
    unwritten), only the non-ZERO chunks' bytes (each rounded up to 16) count
    as written."""
    S = int(sum(sizes))
    dense = int(sum((s + 15) // 16 * 16 for s in sizes))
    N = int(sum((s + C - 1) // C for s in sizes))
    if flags is None:
        return S, dense, N, S + dense + 5 * N
    return S, dense, N, S + stored_bytes(sizes, C, flags) + 5 * N


def stored_bytes(sizes, C, flags):
    """Bytes of the non-ZERO chunks, each rounded up to 16 (what the one-wave
    pack of small chunks writes, and what a drained image holds)."""
    import numpy as np
    lens = np.concatenate([np.minimum(C, s - np.arange(0, s, C, dtype=np.int64)) for s in sizes if s]
                          or [np.zeros(0, np.int64)])
    nz = (np.asarray(flags)[:lens.size] & 1) == 0
    return int(((lens[nz] + 15) // 16 * 16).sum())


def elides_zero(C, wpc):
    """The pack kernel form that leaves ZERO chunks unwritten: one wave per
    chunk, chunks of at most four 1 KiB rounds."""
    return wpc in (0, 1) and C <= 4096


def cpu_baseline(tensors, sizes, C, budget_bytes=8 << 30, reps=3):
    """The oracle (plain C, bytewise table CRC) on a bounded sample of the
    same workload: the first allocations up to budget_bytes (about 20 core-
    seconds of oracle work per run on 16 cores).  Host copies are made before
    timing."""
    import ctypes

    import numpy as np

    from oracle import oracle as O
    take, tot = [], 0
    for k, s in enumerate(sizes):
        if tot + s > budget_bytes and take:
            break
        take.append(k)
        tot += int(s)
    hosts = [tensors[k].cpu().numpy() for k in take]
    ss = [int(sizes[k]) for k in take]
    S, dense_b, N, alg = algorithmic_bytes(ss, C)
    threads = len(os.sched_getaffinity(0))
    lib = O.lib()
    dense = np.empty(dense_b, np.uint8)
    crc = np.empty(max(N, 1), np.uint32)
    flags = np.empty(max(N, 1), np.uint8)
    ptrs = O._ptr_array(hosts)
    szs = np.array(ss, np.uint64)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        rc = lib.oracle_checkpoint(len(hosts), ptrs, O._p(szs, O._u64p), C, None, threads,
                                   O._p(dense, O._u8p), O._p(crc, O._u32p), O._p(flags, O._u8p), None, None)
        times.append(time.perf_counter() - t0)
        assert rc == 0
    t = statistics.median(times)
    # one thread, on the allocations that fit the first 512 MiB of the sample
    k1, tot1 = 0, 0
    while k1 < len(ss) and (tot1 + ss[k1] <= (512 << 20) or k1 == 0):
        tot1 += ss[k1]
        k1 += 1
    _, dense1, N1, alg1 = algorithmic_bytes(ss[:k1], C)
    ptrs1 = O._ptr_array(hosts[:k1])
    szs1 = np.array(ss[:k1], np.uint64)
    t1s = []
    for _ in range(reps):
        t0 = time.perf_counter()
        rc = lib.oracle_checkpoint(k1, ptrs1, O._p(szs1, O._u64p), C, None, 1, O._p(dense[:dense1], O._u8p),
                                   O._p(crc, O._u32p), O._p(flags, O._u8p), None, None)
        t1s.append(time.perf_counter() - t0)
        assert rc == 0
    t1 = statistics.median(t1s)
    cpu = ""
    try:
        # the model name, with family and model numbers (some hosts report only
        # the brand in the name) and the logical CPUs the host has
        info = {}
        with open("/proc/cpuinfo") as f:
            for l in f:
                k, _, v = l.partition(":")
                info.setdefault(k.strip(), v.strip())
        cpu = "%s (family %s, model %s, stepping %s; %d logical CPUs on the host)" % (
            info.get("model name", "?"), info.get("cpu family", "?"), info.get("model", "?"),
            info.get("stepping", "?"), os.cpu_count() or 0)
    except OSError:
        pass
    return {"value": round(alg / t / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of %d allocations (%.2f GiB live, %d chunks) of the same workload; "
                      "median of %d runs of oracle_checkpoint (dense image + CRC + flags), host copies "
                      "made before timing" % (len(take), len(sizes), S / 2**30, N, reps),
            "seconds": round(t, 3),
            "value_1_thread": round(alg1 / t1 / 1e9, 3),
            "sample_1_thread": "first %d allocations (%.2f GiB live) of the sample, one thread, median of %d"
                               % (k1, tot1 / 2**30, reps),
            "cpu_model": cpu}


def bench_incremental(K, synth, torch, stream, args, reps=3):
    """Incremental workload: 2048 allocations, 8 GiB random; 5% of the 64 KiB
    cells rewritten; increment = hash-only pass, dirty scan, gather from the
    allocations, drain of the delta."""
    w = synth.incremental()
    sizes = [int(x) for x in w["sizes"]]
    S = sum(sizes)
    tensors = synth.make_device_allocs(sizes, w["zero"], workload=3)
    chunks = (65536, 4096)
    bases, ctxs = {}, {}
    for C in chunks:
        nd = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN, **tune_kw(args))
        for t in tensors:
            nd.register(t)
        bases[C] = nd.checkpoint(stream=stream)
        ctxs[C] = nd
    # the mutation: each picked grid cell rewritten with new random bytes
    g = w["grid"]
    for i, (k, c) in enumerate(zip(w["mut_alloc"], w["mut_cell"])):
        t = tensors[int(k)]
        lo = int(c) * g
        synth.fill_random_(t[lo:min(t.numel(), lo + g)], synth.alloc_seed(3, int(k), phase=1) + i)
    torch.cuda.synchronize()
    out = {"workload": "incremental: %d allocations, %.2f GiB random, %d of the 64 KiB cells rewritten"
                       % (len(sizes), S / 2**30, len(w["mut_alloc"]))}
    for C in chunks:
        ctx = K.Context(chunk_bytes=C, flags=K.CKPT_TIMING, **tune_kw(args))
        for t in tensors:
            ctx.register(t)
        tm, info = [], None
        for r in range(reps + 1):
            d = ctx.checkpoint(stream=stream, mode=K.CKPT_INCREMENTAL, base=bases[C])
            info = d.info()
            if r:
                tm.append(ctx.timing())
            d.close()
        med = lambda key: statistics.median(x[key] for x in tm)  # noqa: E731
        hash_ms = med("pack_ms")
        res = {"chunk_bytes": C, "chunks": info["n_chunks"], "dirty_chunks": info["n_dirty"],
               "delta_bytes": info["serialized_bytes"],
               "hash_ms": round(hash_ms, 4), "hash_gbps": round(S / (hash_ms * 1e-3) / 1e9, 1),
               "hash_frac_hbm": round(S / (hash_ms * 1e-3) / HBM_PEAK, 4),
               "select_gather_ms": round(med("select_ms") + med("gather_ms"), 4),
               "d2h_ms": round(med("d2h_ms"), 3), "total_ms": round(med("total_ms"), 3),
               "delta_vs_full_drain": round(info["serialized_bytes"] / S, 4)}
        log("incremental C=%d: %s" % (C, res))
        out["c%d" % C] = res
        ctx.close()
    for C in chunks:
        bases[C].close()
        ctxs[C].close()
    out["churn"] = bench_churn(K, synth, torch, stream, args, tensors, sizes)
    del tensors
    return out


def bench_churn(K, synth, torch, stream, args, tensors, sizes, C=65536, reps=3):
    """Allocation-set changes between checkpoints: from a drained base, 1% of
    the allocations are freed and as many new ones made (random bytes); the
    increment is matched to the base by registration id, and the merge folds
    base + increment into the current full image on the host."""
    import numpy as np
    ctx = K.Context(chunk_bytes=C, flags=K.CKPT_TIMING, **tune_kw(args))
    for t in tensors:
        ctx.register(t)
    base = ctx.checkpoint(stream=stream)
    rng = np.random.default_rng(synth.BASE_SEED)
    gone = set(rng.choice(len(tensors), len(tensors) // 100, replace=False).tolist())
    fresh = []
    for j, k in enumerate(sorted(gone)):
        ctx.unregister(tensors[k])
        t = torch.empty(sizes[k], dtype=torch.uint8, device="cuda")
        synth.fill_random_(t, synth.alloc_seed(3, k, phase=2))
        fresh.append(t)
    torch.cuda.synchronize()
    for t in fresh:
        ctx.register(t)
    tm = []
    for r in range(reps + 1):
        d = ctx.checkpoint(stream=stream, mode=K.CKPT_INCREMENTAL, base=base)
        if r:
            tm.append(ctx.timing())
        info = d.info()
        if r < reps:
            d.close()
    t0 = time.perf_counter()
    merged = K.merge(base, d)
    merge_s = time.perf_counter() - t0
    mi = merged.info()
    res = {"chunk_bytes": C, "freed": len(gone), "new": len(fresh), "chunks": info["n_chunks"],
           "dirty_chunks": info["n_dirty"],
           "hash_ms": round(statistics.median(x["pack_ms"] for x in tm), 4),
           "total_ms": round(statistics.median(x["total_ms"] for x in tm), 3),
           "merge_s": round(merge_s, 3), "merged_bytes": mi["serialized_bytes"],
           "merge_gbps_host": round(mi["serialized_bytes"] / merge_s / 1e9, 2)}
    log("churn: %s" % res)
    for im in (merged, d, base):
        im.close()
    ctx.close()
    del fresh
    return res


def bench_batched(K, synth, torch, stream, args, reps=3):
    """Batched workload: 512 contexts of 1-64 allocations (log-uniform 1 MiB -
    256 MiB per context), random bytes with 20% of the 256 KiB cells zero.
    First the autotuner (chunk size, waves per chunk, workgroup size, load/store
    hint); then, in its best shape at C = 4 KiB (the section's chunk size),
    one batched call that replays a captured graph against the plain forms
    (one checkpoint call per allocation, or per context) in the same shape.
    Launch-shape flags on the command line override the tuned shape."""
    from paper_2008_10596_amd import autotune
    spec = synth.batched()
    C = 4096
    sets, tensors = [], []
    k = 0
    for ci, cs in enumerate(spec):
        allocs = []
        for j, sz in enumerate(cs["sizes"]):
            t = torch.empty(int(sz), dtype=torch.uint8, device="cuda")
            synth.fill_random_(t, synth.alloc_seed(4, k))
            reg = cs["region"]
            for cell in cs["zero_cells"][j]:
                t[int(cell) * reg:int(cell) * reg + reg] = 0
            allocs.append(t)
            tensors.append(t)
            k += 1
        sets.append(allocs)
    torch.cuda.synchronize()
    sizes = [t.numel() for t in tensors]
    S, dense_b, N, alg = algorithmic_bytes(sizes, C)
    log("batched: %d contexts, %d allocations, %.2f GiB" % (len(sets), len(tensors), S / 2**30))
    members = []
    for allocs in sets:
        c = K.Context(chunk_bytes=C)
        for t in allocs:
            c.register(t)
        members.append(c)
    out = {"workload": "batched: %d contexts, %d allocations, %.2f GiB, 20%% zero 256 KiB cells, C=%d"
                       % (len(sets), len(tensors), S / 2**30, C), "algorithmic_bytes": alg}
    shape = {}
    if not args.batched_only_graph:
        # autotuner sweep on the same allocations
        alloc_sets = [[(t.data_ptr(), t.numel()) for t in allocs] for allocs in sets]
        tuned = autotune.tune(alloc_sets, chunks=(4096, 16384, 65536, 262144), waves=(1, 2, 4),
                              blocks=(256, 1024), reps=2, stream=stream)
        at_c = min((t for t in tuned["trials"] if t["chunk_bytes"] == C), key=lambda t: t["device_ms"])
        out["autotune"] = {"best": tuned["best"], "best_at_c": at_c, "trials": len(tuned["trials"]),
                           "worst_gbps": min(t["gbps"] for t in tuned["trials"]),
                           "c4096_best_gbps": at_c["gbps"]}
        log("autotune: %s" % out["autotune"])
        shape = {"waves_per_chunk": at_c["waves_per_chunk"], "block_threads": at_c["block_threads"],
                 "load_hint": at_c["load_hint"]}
    for key, v in tune_kw(args).items():
        if v:
            shape[key] = v
    out["shape"] = dict(shape)

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        w = []
        for _ in range(n):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            w.append((time.perf_counter() - t0) * 1e3)
        return statistics.median(w)

    # batched, image kept in HBM: one graph replay
    leader = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN | K.CKPT_TIMING |
                       (K.CKPT_NO_GRAPH if args.batched_no_graph else 0), **shape)
    dev_ms = []
    if elides_zero(C, shape.get("waves_per_chunk", 0)):
        # the pack leaves ZERO chunks unwritten: count the bytes it moves
        import numpy as np
        imgs = K.checkpoint_batch([leader] + members, stream=stream)
        flags = np.concatenate([im.flags for im in imgs[1:]])
        for im in imgs:
            im.close()
        S, dense_b, N, alg = algorithmic_bytes(sizes, C, flags)
        out["algorithmic_bytes"] = alg

    def batched_once():
        imgs = K.checkpoint_batch([leader] + members, stream=stream)
        dev_ms.append(leader.timing()["pack_ms"])
        for im in imgs:
            im.close()
    wall = timed(batched_once, reps)
    out["batched_pack"] = {"wall_ms": round(wall, 3), "gbps_wall": round(alg / (wall * 1e-3) / 1e9, 1),
                           "device_ms": round(statistics.median(dev_ms[1:]), 3),
                           "gbps_device": round(alg / (statistics.median(dev_ms[1:]) * 1e-3) / 1e9, 1),
                           "launches": 1}
    log("batched pack: %s" % out["batched_pack"])
    if args.batched_only_graph:
        leader.close()
        for c in members:
            c.close()
        return out
    # plain, image kept in HBM: one checkpoint call per allocation
    pctx = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN | K.CKPT_TIMING, **shape)

    def plain_alloc():
        for t in tensors:
            pctx.register(t)
            pctx.checkpoint(stream=stream).close()
            pctx.unregister(t)
    wall_pa = timed(plain_alloc, 1)
    out["plain_per_allocation_pack"] = {"wall_ms": round(wall_pa, 1),
                                        "gbps_wall": round(alg / (wall_pa * 1e-3) / 1e9, 1),
                                        "launches": 3 * len(tensors)}
    log("plain per allocation: %s" % out["plain_per_allocation_pack"])

    def plain_ctx():
        for allocs in sets:
            for t in allocs:
                pctx.register(t)
            pctx.checkpoint(stream=stream).close()
            for t in allocs:
                pctx.unregister(t)
    wall_pc = timed(plain_ctx, 1)
    out["plain_per_context_pack"] = {"wall_ms": round(wall_pc, 1),
                                     "gbps_wall": round(alg / (wall_pc * 1e-3) / 1e9, 1),
                                     "launches": 3 * len(sets)}
    log("plain per context: %s" % out["plain_per_context_pack"])
    out["batched_speedup_vs_plain_per_allocation"] = round(wall_pa / wall, 2)
    out["batched_speedup_vs_plain_per_context"] = round(wall_pc / wall, 2)
    # with the drain to pinned host memory: in the replayed graph (the gather
    # stores into each image's pinned buffer), and without graphs (segments
    # through device staging and the runtime's copies)
    ser = {}

    def drained(leader_flags, key):
        dl = K.Context(chunk_bytes=C, flags=K.CKPT_TIMING | leader_flags, **shape)

        def once():
            imgs = K.checkpoint_batch([dl] + members, stream=stream)
            ser[key] = sum(im.info()["serialized_bytes"] for im in imgs)
            for im in imgs:
                im.close()
        w = timed(once, 2)
        dl.close()
        return {"wall_ms": round(w, 1), "serialized_bytes": ser[key],
                "link_gbps": round(ser[key] / (w * 1e-3) / 1e9, 2)}
    out["batched_with_drain"] = drained(0, "graph")
    out["batched_with_drain_no_graph"] = drained(K.CKPT_NO_GRAPH, "plain")
    log("batched with drain: %s; without graphs: %s" % (out["batched_with_drain"], out["batched_with_drain_no_graph"]))
    leader.close()
    pctx.close()
    for c in members:
        c.close()
    del tensors, sets
    return out


def bench_restore_at(K, torch, tensors, sizes, C, stream, reps=3):
    """Restore at the recorded addresses: the at-scale allocations as
    address-stable memory, drained once; then the image is restored in place
    (allocations live) and after every allocation was released (re-created
    at its address, then refilled), both timed on the host around the call."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    vctx = K.Context(chunk_bytes=C)
    ptrs = []
    for t, s in zip(tensors, sizes):
        p, _ = vctx.vmm_alloc(s)
        assert hip.hipMemcpy(p, t.data_ptr(), s, 3) == 0   # device to device
        ptrs.append(p)
    img = vctx.checkpoint(stream=stream)
    vctx.restore_at(img, stream=stream)   # warm
    inplace, recreate = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        rc, _, _ = vctx.restore_at(img, stream=stream)
        inplace.append((time.perf_counter() - t0) * 1e3)
        assert rc == K.CKPT_OK
        for p in ptrs:
            vctx.vmm_free(p)
        t0 = time.perf_counter()
        rc, _, addrs = vctx.restore_at(img, stream=stream)
        recreate.append((time.perf_counter() - t0) * 1e3)
        assert rc == K.CKPT_OK and addrs == ptrs
    a, b = statistics.median(inplace), statistics.median(recreate)
    out = {"allocations": len(sizes), "live_bytes": sum(sizes),
           "serialized_bytes": img.info()["serialized_bytes"],
           "in_place_ms": round(a, 3), "recreate_ms": round(b, 3),
           "recreate_overhead_ms": round(b - a, 3),
           "recreate_overhead_us_per_allocation": round((b - a) * 1e3 / max(len(sizes), 1), 2),
           "verified": "every chunk's CRC on every restore (status CKPT_OK)"}
    img.close()
    vctx.close()
    return out


def hbm_ceilings(torch, nbytes, reps=3):
    """Plain read, write and copy kernels (libckpt_probe.so, not on the path)
    swept over pieces per lane in flight, workgroups per CU and load/store
    hints: the most this GPU moves for each kind of traffic.  read and write
    touch nbytes; the copies read nbytes / 2 and write nbytes / 2 (copy: both
    hints alike; copy_nt_loads / copy_nt_stores: only the loads / only the
    stores non-temporal).  The _dyn kinds take tiles of 256 KiB from a counter
    instead of a fixed grid-stride split."""
    import ctypes
    from paper_2008_10596_amd import build as B
    if not os.path.exists(B.PROBE_LIB):
        raise RuntimeError("libckpt_probe.so is not built")
    lib = ctypes.CDLL(B.PROBE_LIB)
    lib.probe_launch.restype = ctypes.c_int
    lib.probe_launch.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(3)
    b.fill_(5)
    sink = torch.zeros(4, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    half = nbytes // 2 // 16 * 16
    table, best = [], {}
    kinds = ((0, "read"), (1, "write"), (2, "copy"), (3, "copy_nt_loads"), (4, "copy_nt_stores"),
             (5, "read_dyn"), (6, "write_dyn"), (7, "copy_dyn"))
    for kind, name in kinds:
        for loads in (4, 8, 16):
            for per_cu in (1, 2):
                for nt in ((1,) if kind in (3, 4) else (0, 1)):
                    if kind in (0, 5):
                        args = (a.data_ptr(), sink.data_ptr(), nbytes)
                    elif kind in (1, 6):
                        args = (None, b.data_ptr(), nbytes)
                    else:
                        args = (a.data_ptr(), a.data_ptr() + half, half)   # the copies move half each way
                    def launch():
                        rc = lib.probe_launch(kind, args[0], args[1], args[2], loads, nt, cus * per_cu, 1024,
                                              ctypes.c_void_p(stream.cuda_stream))
                        if rc != 0:
                            raise RuntimeError("probe_launch: %d" % rc)
                    launch()
                    ms = []
                    for _ in range(reps):
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record()
                        launch()
                        e1.record()
                        e1.synchronize()
                        ms.append(e0.elapsed_time(e1))
                    m = statistics.median(ms)
                    moved = nbytes if kind in (0, 1, 5, 6) else 2 * half
                    row = {"kind": name, "loads_per_lane": loads, "wgs_per_cu": per_cu, "nontemporal": nt,
                           "ms": round(m, 4), "gbps": round(moved / (m * 1e-3) / 1e9, 1)}
                    table.append(row)
                    if name not in best or row["gbps"] > best[name]["gbps"]:
                        best[name] = row
    del a, b, sink
    torch.cuda.empty_cache()
    return {"best": {k: dict(v, frac=round(v["gbps"] * 1e9 / HBM_PEAK, 4)) for k, v in best.items()},
            "bytes_moved": nbytes, "workgroup_threads": 1024,
            "sweep": [[r["kind"], r["loads_per_lane"], r["wgs_per_cu"], r["nontemporal"], r["gbps"]] for r in table],
            "sweep_columns": ["kind", "loads_per_lane", "wgs_per_cu", "nontemporal", "gbps"]}


def copy_reference(torch, nbytes, reps=5):
    """A plain device-to-device copy (torch copy_, i.e. the runtime's own copy)
    of nbytes into a fresh buffer, timed with events on the current stream:
    what moving the same read + write bytes costs without the method."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    m = statistics.median(ms)
    return {"bytes_read_plus_written": 2 * nbytes, "ms": round(m, 4), "gbps": round(2 * nbytes / (m * 1e-3) / 1e9, 1),
            "kind": "device-to-device copy_ of %.0f GiB into a fresh buffer, median of %d" % (nbytes / 2**30, reps)}


def sink_deflate(K, img, ctx, path):
    """Write img as the compressed container and read it back; rates are
    per byte of the serialized image (what a caller saves), file bytes apart."""
    ser = img.info()["serialized_bytes"]
    t0 = time.perf_counter()
    nbytes = img.write_file(path, deflate=True)
    w_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    back = K.Image.read_file(path, ctx)
    r_s = time.perf_counter() - t0
    same = back.info()["crc_digest"] == img.info()["crc_digest"] and bool((back.data[:1 << 20] ==
                                                                          img.data[:1 << 20]).all())
    back.close()
    os.unlink(path)
    return {"serialized_bytes": ser, "file_bytes": nbytes, "ratio": round(nbytes / max(ser, 1), 4),
            "write_s": round(w_s, 3), "write_gbps_serialized": round(ser / w_s / 1e9, 2),
            "read_s": round(r_s, 3), "read_gbps_serialized": round(ser / r_s / 1e9, 2), "read_back_equal": same}


def bench_sink_bf16(K, torch, args, sink_dir):
    """The compressed container on model-weight-like bytes: 16 allocations,
    2 GiB in all, of bfloat16 values drawn from N(0, 1) (seeded)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(12701)
    total = int((2 << 30) * args.scale)
    per = total // 16 // 2 * 2
    ts = [torch.randn(per // 2, generator=g, device="cuda").to(torch.bfloat16).view(torch.uint8) for _ in range(16)]
    torch.cuda.synchronize()
    ctx = K.Context(chunk_bytes=args.chunk)
    for t in ts:
        ctx.register(t)
    img = ctx.checkpoint()
    path = os.path.join(sink_dir, "ckpt_bench_bf16_%d.img" % os.getpid())
    t0 = time.perf_counter()
    plain = img.write_file(path)
    plain_s = time.perf_counter() - t0
    os.unlink(path)
    out = sink_deflate(K, img, ctx, path)
    out["plain_write_s"] = round(plain_s, 3)
    out["plain_write_gbps"] = round(plain / plain_s / 1e9, 2)
    out["workload"] = "16 allocations, %.2f GiB of bfloat16 N(0,1) values" % (16 * per / 2**30)
    img.close()
    ctx.close()
    del ts
    torch.cuda.empty_cache()
    return out


def hook_child(mode):
    """One fresh process: time allocate + free pairs of device tensors with
    torch's own caching allocator ("torch") or through libckpt's allocation
    hook ("hook": hipMalloc + registration; "stable": address-stable memory;
    "_cache": with the hook's block cache)."""
    import torch
    from paper_2008_10596_amd import ckpt as K
    from paper_2008_10596_amd import hook
    ctx = K.Context()
    if mode != "torch":
        hook.install(ctx, address_stable=mode.startswith("stable"), cache=mode.endswith("_cache"))
    sizes = [4096, 1 << 20, 16 << 20]
    out = {}
    for sz in sizes:
        for _ in range(20):                       # warm
            t = torch.empty(sz, dtype=torch.uint8, device="cuda")
            del t
        torch.cuda.synchronize()
        n = 500
        t0 = time.perf_counter()
        for _ in range(n):
            t = torch.empty(sz, dtype=torch.uint8, device="cuda")
            del t
        torch.cuda.synchronize()
        out[str(sz)] = round((time.perf_counter() - t0) / n * 1e6, 2)
    live = ctx.live_count()
    print(json.dumps({"mode": mode, "us_per_alloc_free": out, "live_after": live}), flush=True)


def bench_hook(args):
    """Cost of logging every allocation (each mode in a fresh process, since
    torch takes a new allocator only before its first device allocation)."""
    import subprocess
    res = {}
    for mode in ("torch", "hook", "stable", "hook_cache", "stable_cache"):
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--hook-child", mode],
                           capture_output=True, text=True, timeout=300)
        if r.returncode != 0:
            raise RuntimeError("hook child %s failed: %s" % (mode, r.stderr[-1000:]))
        res[mode] = json.loads(r.stdout.strip().splitlines()[-1])["us_per_alloc_free"]
    return {"us_per_alloc_free_by_bytes": res,
            "note": "torch = its caching allocator; hook = every allocation hipMalloc'd and registered; "
                    "stable = every allocation an address-stable VMM mapping, registered; "
                    "_cache = the hook's block cache on (freed blocks reused on their stream)"}


def bench_serving(K, synth, torch, args):
    """Serving workload (reduced sweep): Poisson arrivals of checkpoint (70%)
    and restore (30%) requests over a pool of request shapes of 1-256
    allocations each (log-uniform 16 MiB - 4 GiB per request, 25% of the
    allocations hipMallocManaged with 30% of their 2 MiB granules moved
    host-side before each checkpoint when the device supports it).  Latency is
    submit to completion; p50/p99 per arrival rate."""
    import ctypes

    import numpy as np
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMallocManaged.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.c_uint]
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemPrefetchAsync.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    rng = synth.rng_for(5)
    GiB, MiB = synth.GiB, synth.MiB
    shapes, managed_ptrs, total = [], [], 0
    for i in range(args.serving_shapes):
        n = int(rng.integers(1, 257))
        tot = int(synth.log_uniform(rng, 1, 16 * MiB, 4 * GiB)[0])
        if total + tot > 40 * GiB:
            tot = max(16 * MiB, 40 * GiB - total)
        sizes = synth.split_total(rng, tot, n) // 16 * 16
        sizes[sizes == 0] = 16
        kinds = (rng.random(n) < 0.25).astype(int)
        bufs, ptrs, keep = [], [], []
        for j, (sz, kd) in enumerate(zip(sizes, kinds)):
            src = torch.empty(int(sz), dtype=torch.uint8, device="cuda")
            synth.fill_random_(src, synth.alloc_seed(5, i * 1000 + j))
            if kd:
                p = ctypes.c_void_p()
                assert hip.hipMallocManaged(ctypes.byref(p), int(sz), 1) == 0
                torch.cuda.synchronize()
                assert hip.hipMemcpy(p.value, src.data_ptr(), int(sz), 3) == 0   # device to device
                ptrs.append(p.value)
                managed_ptrs.append(p.value)
            else:
                ptrs.append(src.data_ptr())
                keep.append(src)
        dst = [torch.empty(int(sz), dtype=torch.uint8, device="cuda") for sz in sizes]
        shapes.append({"ptrs": ptrs, "sizes": [int(x) for x in sizes], "kinds": [int(x) for x in kinds],
                       "keep": keep, "dst": dst, "image": None, "bytes": int(sum(sizes))})
        total += int(sum(sizes))
    torch.cuda.synchronize()
    prefetch_ok = None

    def move_host(sh):
        nonlocal prefetch_ok
        for p, sz, kd in zip(sh["ptrs"], sh["sizes"], sh["kinds"]):
            if not kd or prefetch_ok is False:
                continue
            gran = 2 * MiB
            cells = max(1, (sz + gran - 1) // gran)
            pick = rng.random(cells) < 0.3
            for c in np.flatnonzero(pick):
                rc = hip.hipMemPrefetchAsync(p + int(c) * gran, min(gran, sz - int(c) * gran), -1, None)
                if prefetch_ok is None:
                    prefetch_ok = rc == 0
                if rc != 0:
                    return
    srv = K.Server(chunk_bytes=4096, staging_budget=64 * GiB, step_bytes=256 * MiB, max_active=16,
                   host_budget=int(args.serving_host_budget_gib * GiB))
    out = {"workload": "serving: %d request shapes reused, %.1f GiB of allocations, 1-256 allocations "
                       "per request, 25%% managed; %d warm-up + %d measured requests per rate"
                       % (len(shapes), total / GiB, args.serving_warmup, args.serving_requests),
           "rates": {}}
    # An image stays open while a restore that reads it is in flight, and a
    # shape's managed pages are only moved host-side while none of its
    # requests is in flight.
    refs = {}          # id(image) -> [image, in-flight restores, retired]
    inflight = [0] * len(shapes)

    def retire(img):
        e = refs.get(id(img))
        if e is None:
            img.close()
            return
        e[2] = True
        if e[1] == 0:
            img.close()
            del refs[id(img)]

    fail_status = {}   # status -> count of failed measured requests (per rate)
    warm_failed = {}   # the same for the warm-up requests
    offered = []       # algorithmic bytes of each measured request

    def done(tk_entry, r):
        _, si, img_used, warm = tk_entry
        inflight[si] -= 1
        if r["status"] not in (K.CKPT_OK, K.CKPT_E_CORRUPT):
            tally = warm_failed if warm else fail_status
            tally[r["status"]] = tally.get(r["status"], 0) + 1
        if img_used is not None:
            e = refs[id(img_used)]
            e[1] -= 1
            if e[2] and e[1] == 0:
                img_used.close()
                del refs[id(img_used)]
        if r["image"] is not None:
            sh = shapes[si]
            old = sh["image"]
            sh["image"] = r["image"]
            refs[id(r["image"])] = [r["image"], 0, False]
            if old is not None:
                retire(old)

    def claim_all(tickets):
        # claim results in the order they finish, not in arrival order:
        # finished checkpoints' images hold pinned memory that a checkpoint
        # held back for host memory may be waiting for
        while tickets:
            still = []
            for entry in tickets:
                r = srv.poll(entry[0])
                if r is None:
                    still.append(entry)
                else:
                    done(entry, r)
            if len(still) == len(tickets):
                time.sleep(0.0005)
            tickets = still

    def run_rate(lam, n_total, warm):
        arr = np.cumsum(rng.exponential(1.0 / lam, n_total))
        ops = rng.random(n_total) < 0.7
        which = rng.integers(0, len(shapes), n_total)
        tickets = []
        t0 = time.perf_counter()
        for i in range(n_total):
            if i == warm:
                # measure from here: the warm-up requests finish first
                claim_all(tickets)
                tickets = []
                srv.reset_stats()
                t0 = time.perf_counter() - arr[i]
            delay = arr[i] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            si = int(which[i])
            sh = shapes[si]
            img = sh["image"]
            warm_req = i < warm
            if ops[i] or img is None:
                if inflight[si] == 0:
                    move_host(sh)
                tk = srv.submit(K.CKPT_REQ_CHECKPOINT, sh["ptrs"], sizes=sh["sizes"], kinds=sh["kinds"])
                tickets.append((tk, si, None, warm_req))
                if not warm_req:
                    offered.append(sh["bytes"])
            else:
                refs[id(img)][1] += 1
                tk = srv.submit(K.CKPT_REQ_RESTORE, sh["dst"], image=img)
                tickets.append((tk, si, img, warm_req))
                if not warm_req:
                    offered.append(sh["bytes"])
            inflight[si] += 1
            still = []
            for entry in tickets:
                r = srv.poll(entry[0])
                if r is None:
                    still.append(entry)
                else:
                    done(entry, r)
            tickets = still
        claim_all(tickets)
        return srv.stats()

    knee = p50_first = None
    for lam in [float(x) for x in args.serving_rates.split(",")]:
        fail_status.clear()
        warm_failed.clear()
        offered.clear()
        st = run_rate(lam, args.serving_requests + args.serving_warmup, args.serving_warmup)
        # offered load: the measured requests' live bytes at the arrival rate, the
        # unit of the server's aggregate GB/s (live bytes of completed requests / makespan)
        offered_gbps = statistics.mean(offered) * lam / 1e9 if offered else 0.0
        res = {"p50_ms": round(st["p50_ms"], 2), "p99_ms": round(st["p99_ms"], 2),
               "mean_ms": round(st["mean_ms"], 2), "completed": st["completed"], "failed": st["failed"],
               "gbps": round(st["gbps"], 2), "offered_gbps": round(offered_gbps, 2),
               "makespan_s": round(st["makespan_s"], 3), "steps": st["steps"],
               "max_concurrent": st["max_concurrent"], "host_waits": st["host_waits"],
               "host_peak_gib": round(st["host_peak"] / GiB, 2),
               "warmup_failed": sum(warm_failed.values())}
        if fail_status or warm_failed:
            res["failed_by_status"] = {K.STATUS_NAMES.get(k, str(k)): v
                                       for k, v in list(fail_status.items()) + list(warm_failed.items())}
            res["last_error"] = st.get("last_error", "")
        if p50_first is None:
            p50_first = st["p50_ms"]
        elif knee is None and st["p50_ms"] > 4 * p50_first:
            knee = lam
        out["rates"]["%g" % lam] = res
        log("serving rate %g/s: %s" % (lam, res))
    out["knee_rate"] = knee
    out["knee_rule"] = ("lowest rate whose p50 latency exceeds 4 x the lowest rate's: past it requests queue "
                        "for the host link")
    out["failed_total"] = sum(r["failed"] + r["warmup_failed"] for r in out["rates"].values())
    out["managed_prefetch_to_host"] = bool(prefetch_ok)
    srv.close()
    for e in list(refs.values()):
        e[0].close()
    refs.clear()
    torch.cuda.synchronize()
    for p in managed_ptrs:
        hip.hipFree(p)
    return out


def main():
    args = parse()
    if args.hook_child:
        hook_child(args.hook_child)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(each GPU would drain its own allocations independently).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2008_10596_amd import ckpt as K

    torch.cuda.set_device(0)
    dev = torch.cuda.get_device_properties(0)
    C = args.chunk
    if args.sections_only:
        stream = torch.cuda.current_stream()
        sections = set(args.only.split(",")) if args.only else set()
        out = {"sections_only": True}
        if "incremental" in sections:
            out["incremental"] = bench_incremental(K, synth, torch, stream, args)
        if "batched" in sections:
            out["batched"] = bench_batched(K, synth, torch, stream, args)
        if "serving" in sections:
            out["serving"] = bench_serving(K, synth, torch, args)
        if "hook" in sections:
            out["hook"] = bench_hook(args)
        print(json.dumps(out), flush=True)
        return
    w = synth.at_scale(cap=int(16 * synth.GiB * args.scale))
    sizes = [int(s) for s in w["sizes"]]
    log("workload: %d allocations, %.2f GiB, %d all-zero; device %s, %d CUs"
        % (len(sizes), sum(sizes) / 2**30, int(w["zero"].sum()), dev.name, dev.multi_processor_count))
    t0 = time.time()
    tensors = synth.make_device_allocs(sizes, w["zero"], workload=2)
    torch.cuda.synchronize()
    log("inputs generated on the device in %.1f s" % (time.time() - t0))

    S, dense_b, N, alg = algorithmic_bytes(sizes, C)
    tune = tune_kw(args)
    # The workload's only writer is the current stream, so the checkpoint is
    # ordered after that stream (CKPT_STREAM_ORDERED); the device-wide drain of
    # the default mode is timed separately below.
    ctx = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN | K.CKPT_TIMING | K.CKPT_STREAM_ORDERED, **tune)
    for t in tensors:
        ctx.register(t)
    stream = torch.cuda.current_stream()

    # warm-up in the pattern of the timed loop (two images alive at a time), so
    # that the pinned-buffer pool already holds what the timed steps use
    prev = None
    for i in range(max(args.warmup, 2)):
        img = ctx.checkpoint(stream=stream)
        if prev is not None:
            prev.close()
        prev = img
    flags = prev.flags.copy()
    prev.close()
    log("warmup done")
    alg_dense = alg
    if elides_zero(C, args.wpc):
        # the one-wave pack of chunks of at most 4 KiB leaves ZERO chunks
        # unwritten: the bytes it moves are the live bytes, the non-ZERO
        # chunks' bytes and 5 bytes per chunk
        S, dense_b, N, alg = algorithmic_bytes(sizes, C, flags)
        log("algorithmic bytes per step: %d (%d with every chunk written)" % (alg, alg_dense))
    pack_ms, step_ms = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    # Each image is freed after the next step is issued, as an application
    # that keeps its image does: freeing waits for the image's CRC/flag copy
    # to the host, which otherwise overlaps the next step.  The last image is
    # freed inside the timed region, so every copy is counted.
    prev = None
    for i in range(args.steps):
        ts = time.perf_counter()
        img = ctx.checkpoint(stream=stream)
        step_ms.append((time.perf_counter() - ts) * 1e3)
        pack_ms.append(ctx.timing()["pack_ms"])
        if prev is not None:
            prev.close()
        prev = img
    if prev is not None:
        prev.close()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = alg / (elapsed / args.steps) / 1e9
    pack_avg = statistics.mean(pack_ms)
    achieved = alg / (pack_avg * 1e-3)
    log("step %.3f ms, pack kernel %.3f ms (min %.3f max %.3f): %.1f GB/s kernel, %.1f GB/s step"
        % (ms_per_step, pack_avg, min(pack_ms), max(pack_ms), achieved / 1e9, value))
    # the same steps with the default device-wide drain first
    wctx = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN, **tune)
    for t in tensors:
        wctx.register(t)
    prev = None
    for i in range(2):
        img = wctx.checkpoint(stream=stream)
        if prev is not None:
            prev.close()
        prev = img
    prev.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nwide = max(3, args.steps // 4)
    prev = None
    for i in range(nwide):
        img = wctx.checkpoint(stream=stream)
        if prev is not None:
            prev.close()
        prev = img
    prev.close()
    torch.cuda.synchronize()
    ms_wide = (time.perf_counter() - t0) * 1e3 / nwide
    log("device-wide drain mode: %.3f ms per step" % ms_wide)
    # the copy reference and the ceilings are measured at the end: freeing
    # their buffers keeps the device's copy engines busy clearing memory for a
    # while, which would slow the host-link copies measured in between
    if args.copy_probe:
        a = torch.empty(args.copy_probe, dtype=torch.uint8, device="cuda")
        b = torch.empty(args.copy_probe, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d bytes written" % (args.copy_probe, args.copy_probe))
        del a, b

    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic (seeded, generated on the device)",
        "config": {"workload": "full checkpoint at scale: %d allocations, log-uniform 4 KiB-64 MiB "
                               "scaled to %.2f GiB, half all-zero, C=%d B, image kept in HBM, "
                               "stream-ordered" % (len(sizes), S / 2**30, C),
                   "live_bytes": S, "chunks": N, "chunk_bytes": C,
                   "bytes_per_step": alg, "bytes_per_step_every_chunk_written": alg_dense,
                   "live_gbps": round(S / (elapsed / args.steps) / 1e9, 2),
                   "ms_per_step_device_wide_drain": round(ms_wide, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved / 1e9, 2), "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK, 4), "traffic": None,
                     "kernel": "k_chunks<pack>", "algorithmic_bytes_per_launch": alg,
                     "kernel_ms": round(pack_avg, 4),
                     "copy_reference": None, "ceilings": None},
    }
    prof = profiled_traffic()
    if prof is not None and prof[1] == alg:
        result["roofline"]["traffic"] = prof[0]
        result["roofline"]["traffic_source"] = "profiles/" + prof[2]

    sections = set(args.only.split(",")) if args.only else {"drain", "restore_at", "incremental", "batched",
                                                             "serving", "hook"}
    if args.no_extras:
        sections = set()
    if "drain" in sections:
        # drain: the same checkpoint with the zero-elided image drained to pinned host memory
        dctx = K.Context(chunk_bytes=C, flags=K.CKPT_TIMING, **tune)
        for t in tensors:
            dctx.register(t)
        dctx.checkpoint(stream=stream).close()
        d2h, gat, tot, pk, img = [], [], [], [], None
        for i in range(args.drain_steps):
            if img is not None:
                img.close()
            img = dctx.checkpoint(stream=stream)
            tm = dctx.timing()
            d2h.append(tm["d2h_ms"])
            gat.append(tm["gather_ms"] + tm["select_ms"])
            tot.append(tm["total_ms"])
            pk.append(tm["pack_ms"])
        info = img.info()
        link_b = info["serialized_bytes"] + 5 * info["n_chunks"]
        d2h_ms = statistics.median(d2h)
        # plain copy-engine probe of the same size over the same link
        probe_n = max(info["serialized_bytes"], 1)
        src = torch.empty(probe_n, dtype=torch.uint8, device="cuda")
        dst = torch.empty(probe_n, dtype=torch.uint8, pin_memory=True)
        dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src, non_blocking=True)
        e1.record()
        torch.cuda.synchronize()
        probe_ms = e0.elapsed_time(e1)
        result["drain"] = {
            "serialized_bytes": info["serialized_bytes"], "link_bytes": link_b,
            "d2h_ms": round(d2h_ms, 3), "gbps": round(link_b / (d2h_ms * 1e-3) / 1e9, 2),
            "frac_link_theoretical": round(link_b / (d2h_ms * 1e-3) / LINK_PEAK, 4),
            "probe_gbps": round(probe_n / (probe_ms * 1e-3) / 1e9, 2),
            "select_gather_ms": round(statistics.median(gat), 3),
            "checkpoint_total_ms": round(statistics.median(tot), 3),
            "pack_ms": round(statistics.median(pk), 3),
            # the call's time outside the pack and the link copies (first start to
            # last end): what of the gather and the bookkeeping the link does not hide
            "exposed_ms": round(statistics.median(t - p - d for t, p, d in zip(tot, pk, d2h)), 3),
        }
        log("drain: %s" % result["drain"])
        del src, dst
        # torch keeps freed pinned blocks cached: give the probe's back to the host
        torch._C._host_emptyCache()
        # restore into fresh buffers from the drained image
        dsts = [torch.empty_like(t) for t in tensors]
        rc, rep = dctx.restore(img, dsts, stream=stream)
        assert rc == K.CKPT_OK, rep
        rs = []
        for i in range(args.drain_steps):
            dctx.restore(img, dsts, stream=stream)
            rs.append(dctx.timing())
        ok = all(torch.equal(a, b) for a, b in zip(dsts[:64], tensors[:64]))
        h2d = statistics.median(r["h2d_ms"] for r in rs)
        sc = statistics.median(r["scatter_ms"] for r in rs)
        # The segmented forms run their kernels beside the link copies (which
        # are kernels too); the kernels' own rates come from one-pass calls.
        octx = K.Context(chunk_bytes=C, flags=K.CKPT_TIMING, segment_mib=0xFFFFFFFF, **tune)
        for t in tensors:
            octx.register(t)
        og, osc = [], []
        for i in range(4):   # the first call allocates the staging and pinned buffers
            octx.checkpoint(stream=stream).close()
            og.append(octx.timing()["gather_ms"])
            octx.restore(img, dsts, stream=stream)
            osc.append(octx.timing()["scatter_ms"])
        og, osc = og[1:], osc[1:]
        octx.close()
        g1, s1 = statistics.median(og), statistics.median(osc)
        result["drain"].update({
            "gather_one_pass_ms": round(g1, 3),
            "gather_gbps": round(2 * info["serialized_bytes"] / (g1 * 1e-3) / 1e9, 1)})
        result["restore"] = {
            "h2d_ms": round(h2d, 3), "h2d_gbps": round(info["serialized_bytes"] / (h2d * 1e-3) / 1e9, 2),
            "scatter_verify_ms": round(sc, 3),
            "total_ms": round(statistics.median(r["total_ms"] for r in rs), 3),
            "exposed_ms": round(statistics.median(r["total_ms"] - r["h2d_ms"] for r in rs), 3),
            "scatter_one_pass_ms": round(s1, 3),
            "scatter_gbps": round((info["serialized_bytes"] + S) / (s1 * 1e-3) / 1e9, 1),
            "first_64_allocations_equal": ok,
        }
        log("restore: %s" % result["restore"])
        # the drained image to a file (durable storage), when the file system has room
        sink_dir = os.environ.get("TMPDIR", "/tmp")
        need = img.info()["serialized_bytes"] * 2
        st = os.statvfs(sink_dir)
        if st.f_bavail * st.f_frsize > need:
            path = os.path.join(sink_dir, "ckpt_bench_%d.img" % os.getpid())
            t0 = time.perf_counter()
            nbytes = img.write_file(path)
            w_s = time.perf_counter() - t0
            t0 = time.perf_counter()
            back = K.Image.read_file(path, dctx)
            r_s = time.perf_counter() - t0
            same = back.info()["crc_digest"] == img.info()["crc_digest"]
            back.close()
            os.unlink(path)
            result["sink"] = {"file_bytes": nbytes, "write_s": round(w_s, 3),
                              "gbps": round(nbytes / w_s / 1e9, 2), "read_s": round(r_s, 3),
                              "read_gbps": round(nbytes / r_s / 1e9, 2), "read_back_equal": same,
                              "dir": sink_dir, "mode": "O_DIRECT (buffered where refused), fsync"}
            log("sink: %s" % result["sink"])
            result["sink"]["deflate"] = {"at_scale_random": sink_deflate(K, img, dctx, path)}
            log("sink deflate (random): %s" % result["sink"]["deflate"]["at_scale_random"])
        img.close()
        del dsts
        dctx.close()

    if "restore_at" in sections:
        result["restore_at"] = bench_restore_at(K, torch, tensors, sizes, C, stream)
        log("restore_at: %s" % result["restore_at"])
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(tensors, sizes, C)
        log("cpu baseline: %s" % result["cpu_baseline"])
    ctx.close()
    wctx.close()   # kept until here: see the note on freeing before the link is measured
    del tensors
    torch.cuda.empty_cache()

    if "incremental" in sections:
        result["incremental"] = bench_incremental(K, synth, torch, stream, args)
        torch.cuda.empty_cache()
    if "batched" in sections:
        result["batched"] = bench_batched(K, synth, torch, stream, args)
        torch.cuda.empty_cache()
    if "serving" in sections:
        result["serving"] = bench_serving(K, synth, torch, args)
        torch.cuda.empty_cache()
    if "hook" in sections:
        result["hook"] = bench_hook(args)
        log("hook: %s" % result["hook"])
    if "sink" in result:
        result["sink"]["deflate"]["bf16"] = bench_sink_bf16(K, torch, args, result["sink"]["dir"])
        log("sink deflate (bf16): %s" % result["sink"]["deflate"]["bf16"])
    if not args.no_ceilings:
        copy_ref = copy_reference(torch, int((8 << 30) * args.scale))
        log("copy reference: %s" % copy_ref)
        result["roofline"]["copy_reference"] = dict(copy_ref, pack_vs_copy=round(achieved / 1e9 / copy_ref["gbps"], 4))
        ceilings = hbm_ceilings(torch, int((16 << 30) * args.scale) // 16 * 16)
        log("hbm ceilings: %s" % ceilings["best"])
        result["roofline"]["ceilings"] = ceilings
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
