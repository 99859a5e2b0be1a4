"""Benchmark of the checkpoint drain/refill path on one MI355X.

Default workload: full checkpoint at scale -- 4096 allocations, log-uniform
4 KiB - 64 MiB scaled to 16 GiB, half of them all-zero, C = 4 KiB.  One step is
one ckpt_checkpoint of the whole live set with the image kept in HBM
(CKPT_NO_DRAIN): descriptor upload, size scan, chunk map, the fused pack +
CRC-32C + ZERO/DIRTY kernel, and the CRC/flag arrays copied to the host.
`value` = algorithmic bytes of a step (every live byte read, the dense image
written, 5 bytes of CRC + flags per chunk) / wall time per step.

Printed as one JSON line.  Further phases of the same run (drain to pinned
host memory, restore) are reported inside the line.
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
    ap.add_argument("--lane-pieces", type=int, default=0)
    ap.add_argument("--load-hint", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the timed pack steps")
    ap.add_argument("--drain-steps", type=int, default=3)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after the timed steps, one plain device copy of this many bytes "
                         "(calibrates hardware byte counters against a known size)")
    return ap.parse_args()


def algorithmic_bytes(sizes, C):
    S = int(sum(sizes))
    dense = int(sum((s + 15) // 16 * 16 for s in sizes))
    N = int(sum((s + C - 1) // C for s in sizes))
    return S, dense, N, S + dense + 5 * N


def cpu_baseline(tensors, sizes, C, budget_bytes=2 << 30, reps=3):
    """The oracle (plain C, bytewise table CRC) on a bounded sample of the
    same workload: the first allocations up to budget_bytes.  Host copies are
    made before timing."""
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
    return {"value": round(alg / t / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of %d allocations (%.2f GiB live, %d chunks) of the same workload; "
                      "median of %d runs of oracle_checkpoint (dense image + CRC + flags), host copies "
                      "made before timing" % (len(take), len(sizes), S / 2**30, N, reps),
            "seconds": round(t, 3)}


def main():
    args = parse()
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
    w = synth.at_scale(cap=int(16 * synth.GiB * args.scale))
    sizes = [int(s) for s in w["sizes"]]
    log("workload: %d allocations, %.2f GiB, %d all-zero; device %s, %d CUs"
        % (len(sizes), sum(sizes) / 2**30, int(w["zero"].sum()), dev.name, dev.multi_processor_count))
    t0 = time.time()
    tensors = synth.make_device_allocs(sizes, w["zero"], workload=2)
    torch.cuda.synchronize()
    log("inputs generated on the device in %.1f s" % (time.time() - t0))

    S, dense_b, N, alg = algorithmic_bytes(sizes, C)
    tune = dict(block_threads=args.block, waves_per_chunk=args.wpc, wgs_per_cu=args.wgs_per_cu,
                lane_pieces=args.lane_pieces, load_hint=args.load_hint)
    ctx = K.Context(chunk_bytes=C, flags=K.CKPT_NO_DRAIN | K.CKPT_TIMING, **tune)
    for t in tensors:
        ctx.register(t)
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        ctx.checkpoint(stream=stream).close()
    log("warmup done")
    pack_ms, step_ms = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        img = ctx.checkpoint(stream=stream)
        step_ms.append((time.perf_counter() - ts) * 1e3)
        pack_ms.append(ctx.timing()["pack_ms"])
        img.close()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = alg / (elapsed / args.steps) / 1e9
    pack_avg = statistics.mean(pack_ms)
    achieved = alg / (pack_avg * 1e-3)
    log("step %.3f ms, pack kernel %.3f ms (min %.3f max %.3f): %.1f GB/s kernel, %.1f GB/s step"
        % (ms_per_step, pack_avg, min(pack_ms), max(pack_ms), achieved / 1e9, value))
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
                               "scaled to %.2f GiB, half all-zero, C=%d B, image kept in HBM"
                               % (len(sizes), S / 2**30, C),
                   "live_bytes": S, "chunks": N, "chunk_bytes": C},
        "roofline": {"bound": "hbm", "achieved": round(achieved / 1e9, 2), "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK, 4), "traffic": None,
                     "kernel": "k_chunks<pack>", "algorithmic_bytes_per_launch": alg,
                     "kernel_ms": round(pack_avg, 4)},
    }

    if not args.no_extras:
        # drain: the same checkpoint with the zero-elided image drained to pinned host memory
        dctx = K.Context(chunk_bytes=C, flags=K.CKPT_TIMING, **tune)
        for t in tensors:
            dctx.register(t)
        dctx.checkpoint(stream=stream).close()
        d2h, gat, tot, img = [], [], [], None
        for i in range(args.drain_steps):
            if img is not None:
                img.close()
            img = dctx.checkpoint(stream=stream)
            tm = dctx.timing()
            d2h.append(tm["d2h_ms"])
            gat.append(tm["gather_ms"] + tm["select_ms"])
            tot.append(tm["total_ms"])
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
        }
        log("drain: %s" % result["drain"])
        del src, dst
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
        result["restore"] = {
            "h2d_ms": round(h2d, 3), "h2d_gbps": round(info["serialized_bytes"] / (h2d * 1e-3) / 1e9, 2),
            "scatter_verify_ms": round(sc, 3),
            "scatter_gbps_alg": round((info["serialized_bytes"] + S) / (sc * 1e-3) / 1e9, 2),
            "total_ms": round(statistics.median(r["total_ms"] for r in rs), 3),
            "first_64_allocations_equal": ok,
        }
        log("restore: %s" % result["restore"])
        img.close()
        del dsts
        dctx.close()

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(tensors, sizes, C)
        log("cpu baseline: %s" % result["cpu_baseline"])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
