"""Pins for the oracle's incremental checkpoint against a base with another
allocation table (allocations made and freed between the two checkpoints).

The rule (a chunk is compared with the same chunk of the base allocation with
the same registration id, size and kind; an allocation without one is
entirely DIRTY) is checked three ways that do not use the function itself:
it reduces to the pinned C incremental checkpoint when the table is
unchanged; on tiny inputs it equals a brute force over the chunk bytes with
the bitwise CRC-32C of the definition; and the cases a positional match, a
match that ignores size or kind, or a dropped ZERO rule would get wrong are
spelled out.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle.crc_bitwise import crc32c_bitwise


C = 64


def rnd(n, seed):
    return np.random.default_rng(seed).integers(0, 256, n, dtype=np.uint8)


def base_of(allocs, ids, kinds):
    full = O.checkpoint(allocs, C)
    return {"base_ids": ids, "base_kinds": kinds, "base_sizes": [a.size for a in allocs], "base_crc": full["crc"]}


def brute(allocs, ids, kinds, base_allocs, base_ids, base_kinds):
    """DIRTY per chunk from the bytes, with the definition's bitwise CRC."""
    out = []
    for k, a in enumerate(allocs):
        j = base_ids.index(ids[k]) if ids[k] in base_ids else None
        ok = j is not None and base_allocs[j].size == a.size and base_kinds[j] == kinds[k]
        for c in range((a.size + C - 1) // C):
            piece = a[c * C:(c + 1) * C].tobytes()
            same = ok and crc32c_bitwise(piece) == crc32c_bitwise(base_allocs[j][c * C:(c + 1) * C].tobytes())
            out.append(not same)
    return np.array(out, bool)


def test_unchanged_table_reduces_to_the_c_delta():
    allocs = [rnd(300, 1), rnd(64, 2), np.zeros(130, np.uint8), rnd(1, 3)]
    ids, kinds = [1, 2, 3, 4], [0, 0, 1, 0]
    b = base_of(allocs, ids, kinds)
    new = [a.copy() for a in allocs]
    new[0][70] ^= 1
    new[2][129] = 5
    got = O.delta_by_id(new, ids, kinds, C, **b)
    ref = O.delta(new, C, b["base_crc"])
    for key in ("crc", "flags", "dirty_ids", "delta"):
        assert np.array_equal(got[key], ref[key]), key


def test_table_changes_match_the_brute_force():
    base_allocs = [rnd(200, 4), rnd(129, 5), rnd(64, 6), np.zeros(100, np.uint8), rnd(70, 7)]
    base_ids, base_kinds = [1, 2, 3, 4, 5], [0, 0, 0, 0, 1]
    b = base_of(base_allocs, base_ids, base_kinds)
    # 1 freed; 2 kept and edited; 3 kept; 4 kept (zero); 5 now DEVICE (kind
    # changed); 6 and 7 new; 3's chunk untouched
    a2 = base_allocs[1].copy()
    a2[128] ^= 0x80
    allocs = [a2, base_allocs[2].copy(), base_allocs[3].copy(), base_allocs[4].copy(), rnd(150, 8),
              np.zeros(64, np.uint8)]
    ids, kinds = [2, 3, 4, 5, 6, 7], [0, 0, 0, 0, 0, 0]
    got = O.delta_by_id(allocs, ids, kinds, C, **b)
    want = brute(allocs, ids, kinds, base_allocs, base_ids, base_kinds)
    assert np.array_equal((got["flags"] & O.FLAG_DIRTY) != 0, want)
    # spelled out: a2 chunks 0,1 clean, chunk 2 (byte 128) dirty; 3 clean;
    # 4 clean; 5 all dirty (kind); 6 all dirty (new); 7 dirty and ZERO
    assert list(got["dirty_ids"]) == [2, 6, 7, 8, 9, 10, 11]
    assert list(got["flags"][[4, 5, 11]]) == [O.FLAG_ZERO, O.FLAG_ZERO, O.FLAG_ZERO | O.FLAG_DIRTY]
    # the delta data is the dirty non-ZERO chunks, padded to 16
    assert got["delta"].size == 16 + 64 + 16 + 64 + 64 + 32


def test_same_id_with_another_size_is_all_dirty():
    base_allocs = [rnd(256, 9)]
    b = base_of(base_allocs, [1], [0])
    grown = np.concatenate([base_allocs[0], rnd(10, 10)])
    got = O.delta_by_id([grown], [1], [0], C, **b)
    assert list(got["dirty_ids"]) == [0, 1, 2, 3, 4]
    shrunk = base_allocs[0][:192].copy()
    got = O.delta_by_id([shrunk], [1], [0], C, **b)
    assert list(got["dirty_ids"]) == [0, 1, 2]


def test_position_is_not_identity():
    """The first allocation freed: the rest shift down by one row but keep
    their ids, so nothing is dirty (a positional match would mark all)."""
    base_allocs = [rnd(64, 11), rnd(64, 12), rnd(128, 13)]
    b = base_of(base_allocs, [1, 2, 3], [0, 0, 0])
    got = O.delta_by_id(base_allocs[1:], [2, 3], [0, 0], C, **b)
    assert got["dirty_ids"].size == 0 and got["delta"].size == 0


def test_overlaying_the_delta_on_the_base_gives_the_new_bytes():
    """Restore semantics: base bytes of matched allocations, then each dirty
    chunk from the delta (ZERO: zeros), equal the new allocations."""
    base_allocs = [rnd(300, 14), rnd(100, 15), rnd(90, 16)]
    base_ids = [1, 2, 3]
    b = base_of(base_allocs, base_ids, [0, 0, 0])
    a1 = base_allocs[0].copy()
    a1[5:9] = 0
    a1[250] = 1
    allocs = [a1, base_allocs[2].copy(), rnd(77, 17)]
    ids = [1, 3, 4]
    got = O.delta_by_id(allocs, ids, [0, 0, 0], C, **b)
    bufs = [base_allocs[base_ids.index(i)].copy() if i in base_ids else np.full(a.size, 0xA5, np.uint8)
            for i, a in zip(ids, allocs)]
    _, cb, _, _ = O.layout([a.size for a in allocs], C)
    pos = 0
    for g in got["dirty_ids"]:
        k = int(np.searchsorted(cb, g, side="right")) - 1
        c = int(g) - int(cb[k])
        n = min(C, allocs[k].size - c * C)
        if got["flags"][g] & O.FLAG_ZERO:
            bufs[k][c * C:c * C + n] = 0
        else:
            bufs[k][c * C:c * C + n] = got["delta"][pos:pos + n]
            pos += (n + 15) // 16 * 16
    assert pos == got["delta"].size
    for x, a in zip(bufs, allocs):
        assert np.array_equal(x, a)
