"""The seeded input recipes: the laws each one states, and determinism."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O


def test_log_uniform_bounds_and_spread():
    rng = np.random.default_rng(1)
    x = synth.log_uniform(rng, 20000, 256, 1 << 20)
    assert x.min() >= 256 and x.max() <= 1 << 20
    # log-uniform: about as many values per octave in every octave
    counts = np.histogram(np.log2(x), bins=np.arange(8, 21))[0]
    assert counts.min() > 0.8 * counts.mean() and counts.max() < 1.2 * counts.mean()


def test_split_total():
    rng = np.random.default_rng(2)
    for n, total in ((1, 100), (7, 1000), (64, 1 << 20)):
        parts = synth.split_total(rng, total, n)
        assert parts.sum() == total and len(parts) == n and parts.min() >= 16


def test_plain_recipe():
    w = synth.plain()
    assert len(w["sizes"]) == 64 and not w["zero"].any()
    assert w["sizes"].min() >= 256 and w["sizes"].max() <= 1 << 20


def test_at_scale_recipe():
    w = synth.at_scale()
    s = w["sizes"]
    assert len(s) == 4096 and s.sum() <= 16 * synth.GiB
    assert (s % 4096 == 0).all() and s.min() >= 4096
    assert w["zero"].sum() == 2048
    w2 = synth.at_scale()
    assert np.array_equal(s, w2["sizes"]) and np.array_equal(w["zero"], w2["zero"])
    assert not np.array_equal(s, synth.at_scale(rep=1)["sizes"])


def test_incremental_recipe():
    w = synth.incremental()
    s, g = w["sizes"], w["grid"]
    assert len(s) == 2048 and s.sum() == 8 * synth.GiB and s.min() >= 4096
    cells = -(-s // g)
    G = int(cells.sum())
    assert len(w["mut_alloc"]) == round(0.05 * G)
    pairs = set(zip(w["mut_alloc"].tolist(), w["mut_cell"].tolist()))
    assert len(pairs) == len(w["mut_alloc"])                        # distinct cells
    assert all(0 <= c < cells[k] for k, c in pairs)


def test_batched_recipe():
    spec = synth.batched()
    assert len(spec) == 512
    for cs in spec:
        assert 1 <= len(cs["sizes"]) <= 64 and cs["sizes"].min() >= 16
        for sz, zc in zip(cs["sizes"], cs["zero_cells"]):
            assert all(0 <= c < -(-int(sz) // cs["region"]) for c in zc)
    zero_frac = np.mean([len(zc) / -(-int(sz) // cs["region"]) for cs in spec
                         for sz, zc in zip(cs["sizes"], cs["zero_cells"])])
    assert 0.15 < zero_frac < 0.25


def test_fill_random_is_seeded_and_in_place():
    base = torch.zeros(3000, dtype=torch.uint8)
    synth.fill_random_(base[1000:2000], 5)
    assert base[:1000].sum() == 0 and base[2000:].sum() == 0
    a = torch.empty(777, dtype=torch.uint8)
    b = torch.empty(777, dtype=torch.uint8)
    synth.fill_random_(a, 9)
    synth.fill_random_(b, 9)
    assert torch.equal(a, b)
    synth.fill_random_(b, 10)
    assert not torch.equal(a, b)
    big = torch.empty(1 << 20, dtype=torch.uint8)
    synth.fill_random_(big, 1)
    counts = np.bincount(big.numpy(), minlength=256)
    assert counts.min() > 0.8 * counts.mean()


@pytest.mark.parametrize("C", [4096, 65536])
def test_bench_algorithmic_bytes_match_the_layout(C):
    import bench
    sizes = [int(x) for x in synth.plain()["sizes"]]
    S, dense, N, alg = bench.algorithmic_bytes(sizes, C)
    _, _, data_bytes, n_chunks = O.layout(sizes, C)
    assert S == sum(sizes) and dense == data_bytes and N == n_chunks
    assert alg == S + dense + 5 * N


@pytest.mark.parametrize("C", [4096, 1024])
def test_bench_bytes_with_flags_are_the_serialized_bytes(C):
    """With the chunks' flags, the bench counts as written exactly what a
    drained image holds: the oracle's serialized bytes."""
    import bench
    rng = np.random.default_rng(C)
    sizes = [int(x) for x in rng.integers(0, 20000, 40)]
    allocs = []
    for k, n in enumerate(sizes):
        a = rng.integers(0, 256, n, dtype=np.uint8)
        if k % 3 == 0:
            a[:] = 0                                  # whole allocation ZERO
        elif k % 3 == 1 and n > C:
            a[:C] = 0                                 # one ZERO chunk
        allocs.append(a)
    ref = O.checkpoint(allocs, C)
    S, dense, N, alg = bench.algorithmic_bytes(sizes, C, ref["flags"])
    assert alg == S + ref["serialized_bytes"] + 5 * N
    assert bench.stored_bytes(sizes, C, ref["flags"]) == ref["serialized_bytes"]
    assert bench.elides_zero(4096, 0) and bench.elides_zero(4096, 1)
    assert not bench.elides_zero(8192, 0) and not bench.elides_zero(4096, 2)
