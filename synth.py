"""Seeded synthetic inputs for the checkpoint workloads.

Holds no part of the method: only allocation-size laws, which allocations or
regions are zero, which chunks a mutation rewrites, and random byte contents.
Both the HIP path (tests, bench) and the oracle read inputs made here.

The paper's own workloads (Rodinia, the CUDA samples, LULESH, HPGMG-FV,
HYPRE; CRAC Sec. 4) are not available and not needed: these seeded allocation
sets stand in for them.  The paper reports device footprints of about 2 GB
(LULESH, Sec. 4.4) and a 2.3 GB image (HYPRE, Sec. 4.5); the per-request
totals below (16 MiB - 4 GiB) span that range.  Base seed 12701 is the seed
the paper fixes for its UnifiedMemoryStreams run (Sec. 4.4); workload i uses
12701 + i, repetition r adds 1000 r.

Random sizes and positions come from numpy's PCG64; byte contents are
generated on the device with a seeded torch generator (one per allocation),
so multi-GiB inputs cost milliseconds.  Host copies for the oracle are read
back from the device.
"""
import math

import numpy as np

BASE_SEED = 12701
KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30


def rng_for(workload, rep=0):
    return np.random.Generator(np.random.PCG64(BASE_SEED + workload + 1000 * rep))


def log_uniform(rng, n, lo, hi):
    """Integers floor(exp(U(ln lo, ln(hi + 1)))) clipped to [lo, hi]."""
    u = rng.uniform(math.log(lo), math.log(hi + 1), n)
    return np.clip(np.floor(np.exp(u)).astype(np.int64), lo, hi)


def split_total(rng, total, n, min_size=16):
    """n sizes >= min_size summing to total, cut at n - 1 sorted uniform points."""
    free = total - min_size * n
    assert free >= 0
    cuts = np.sort(rng.integers(0, free + 1, n - 1)) if n > 1 else np.zeros(0, np.int64)
    parts = np.diff(np.concatenate([[0], cuts, [free]]))
    return (parts + min_size).astype(np.int64)


# ---------------------------------------------------------------- recipes

def plain(n=64, lo=256, hi=1 * MiB, rep=0):
    """Plain full checkpoint + restore: n allocations, log-uniform byte counts,
    all contents random."""
    rng = rng_for(1, rep)
    sizes = log_uniform(rng, n, lo, hi)
    return {"sizes": sizes, "zero": np.zeros(n, bool)}


def at_scale(n=4096, lo=4 * KiB, hi=64 * MiB, cap=16 * GiB, n_zero=None, rep=0):
    """Full checkpoint at scale: log-uniform sizes; if their sum exceeds cap,
    every size is scaled by cap / sum and floored to a 4 KiB multiple (at
    least 4 KiB).  A seeded half of the allocations is all-zero."""
    rng = rng_for(2, rep)
    sizes = log_uniform(rng, n, lo, hi).astype(np.float64)
    if sizes.sum() > cap:
        sizes = sizes * (cap / sizes.sum())
    sizes = np.maximum(np.floor(sizes / (4 * KiB)) * 4 * KiB, 4 * KiB).astype(np.int64)
    n_zero = n // 2 if n_zero is None else n_zero
    zero = np.zeros(n, bool)
    zero[rng.choice(n, n_zero, replace=False)] = True
    return {"sizes": sizes, "zero": zero}


def incremental(n=2048, lo=64 * KiB, hi=64 * MiB, total=8 * GiB, grid=64 * KiB, frac=0.05, rep=0):
    """Incremental checkpoint: log-uniform sizes scaled to sum to `total`
    (floored to 4 KiB, remainder added to the last); all random.  The
    mutation picks round(frac * G) distinct cells of the per-allocation
    `grid`-byte cell grid (G cells in all; a tail cell is partial) and each is
    rewritten with new random bytes."""
    rng = rng_for(3, rep)
    sizes = log_uniform(rng, n, lo, hi).astype(np.float64)
    sizes = np.floor(sizes * (total / sizes.sum()) / (4 * KiB)).astype(np.int64) * 4 * KiB
    sizes = np.maximum(sizes, 4 * KiB)
    sizes[-1] += total - sizes.sum()
    assert sizes.sum() == total and sizes[-1] > 0
    cells = -(-sizes // grid)
    starts = np.concatenate([[0], np.cumsum(cells)[:-1]])
    G = int(cells.sum())
    pick = np.sort(rng.choice(G, int(round(frac * G)), replace=False))
    k = np.searchsorted(starts, pick, side="right") - 1
    c = pick - starts[k]
    return {"sizes": sizes, "zero": np.zeros(n, bool), "mut_alloc": k, "mut_cell": c, "grid": grid}


def batched(n_ctx=512, max_allocs=64, lo=1 * MiB, hi=256 * MiB, region=256 * KiB, p_zero=0.2, rep=0):
    """Batched: n_ctx contexts with U{1..max_allocs} allocations each; each
    context's total is log-uniform and split at sorted uniform cut points
    (every allocation >= 16 B).  Random bytes, then each `region`-aligned cell
    of every allocation is zeroed with probability p_zero."""
    rng = rng_for(4, rep)
    ctxs = []
    for _ in range(n_ctx):
        n = int(rng.integers(1, max_allocs + 1))
        total = int(log_uniform(rng, 1, lo, hi)[0])
        sizes = split_total(rng, total, n)
        zero_cells = [np.flatnonzero(rng.random(-(-int(s) // region)) < p_zero) for s in sizes]
        ctxs.append({"sizes": sizes, "zero_cells": zero_cells, "region": region})
    return ctxs


# ------------------------------------------------------- device contents

def alloc_seed(workload, k, rep=0, phase=0):
    return (BASE_SEED + workload + 1000 * rep) * 1_000_003 + 7919 * k + 104_729 * phase


def fill_random_(t, seed):
    """Fill a uint8 device tensor with seeded random bytes (torch generator)."""
    import torch
    n = t.numel()
    if n == 0:
        return t
    g = torch.Generator(device=t.device)
    g.manual_seed(int(seed) & ((1 << 63) - 1))
    # written in place: no intermediate tensor and no copy kernel
    torch.randint(0, 256, (n,), dtype=torch.uint8, device=t.device, generator=g, out=t)
    return t


def make_device_allocs(sizes, zero, workload, rep=0, device="cuda"):
    """One uint8 tensor per size; random unless zero[k]."""
    import torch
    out = []
    for k, s in enumerate(sizes):
        t = torch.empty(int(s), dtype=torch.uint8, device=device)
        if zero[k]:
            t.zero_()
        else:
            fill_random_(t, alloc_seed(workload, k, rep))
        out.append(t)
    return out
