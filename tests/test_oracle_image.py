"""Pins for the oracle's layout, chunk records, images, deltas and restore:
closed forms, brute force on tiny inputs, and invariants."""
import numpy as np
import pytest

from oracle import crc_bitwise as cb

FLAG_ZERO, FLAG_DIRTY = 1, 2


def rand_allocs(rng, sizes, zero_idx=()):
    out = []
    for k, s in enumerate(sizes):
        a = rng.integers(0, 256, int(s), dtype=np.uint8)
        if k in zero_idx:
            a[:] = 0
        out.append(a)
    return out


def r16(x):
    return (x + 15) // 16 * 16


# ----------------------------------------------------------------- layout

def test_layout_closed_forms(oracle):
    rng = np.random.default_rng(1)
    for C in (16, 32, 4096, 65536):
        sizes = rng.integers(0, 200000, 50).astype(np.uint64)
        sizes[[3, 17]] = 0
        off, cb_, data_bytes, N = oracle.layout(sizes, C)
        ext = [r16(int(s)) for s in sizes]
        nc = [-(-int(s) // C) for s in sizes]
        assert data_bytes == sum(ext)
        assert N == sum(nc)
        assert list(off) == [sum(ext[:k]) for k in range(len(sizes))]
        assert list(cb_) == [sum(nc[:k]) for k in range(len(sizes))]
        assert all(int(o) % 16 == 0 for o in off)


def test_layout_rejects_bad_chunk_size(oracle):
    for C in (0, 8, 24, 4100):
        with pytest.raises(ValueError):
            oracle.layout([10, 20], C)


# ------------------------------------------------------- per-chunk records

@pytest.mark.parametrize("C", [16, 48, 64, 4096])
def test_records_match_bruteforce_tiny(oracle, C):
    rng = np.random.default_rng(C)
    sizes = [0, 1, 15, 16, 17, 31, 100, 257, 1000]
    allocs = rand_allocs(rng, sizes, zero_idx=(5,))
    r = oracle.checkpoint(allocs, C)
    crcs, flags = cb.chunk_records(allocs, C)
    assert list(r["crc"]) == crcs
    assert list(r["flags"]) == flags


def test_zero_flag_single_nonzero_byte_every_position(oracle):
    # one non-zero byte at every position of a 3-chunk allocation with a tail
    C, size = 32, 80
    for pos in range(size):
        a = np.zeros(size, np.uint8)
        a[pos] = 1 + pos % 255
        r = oracle.checkpoint([a], C)
        want = [FLAG_DIRTY | (FLAG_ZERO if g != pos // C else 0) for g in range(3)]
        assert list(r["flags"]) == want, pos


def test_dirty_flag_rules(oracle):
    rng = np.random.default_rng(3)
    allocs = rand_allocs(rng, [5000, 300, 9000], zero_idx=(1,))
    C = 1024
    first = oracle.checkpoint(allocs, C)
    assert all(f & FLAG_DIRTY for f in first["flags"])            # no base: all dirty
    same = oracle.checkpoint(allocs, C, base_crc=first["crc"])
    assert not any(f & FLAG_DIRTY for f in same["flags"])          # unchanged: none
    allocs[2][5000] ^= 0x10                                        # chunk 4 of alloc 2
    _, cb_, _, _ = oracle.layout([a.size for a in allocs], C)
    g = int(cb_[2]) + 5000 // C
    changed = oracle.checkpoint(allocs, C, base_crc=first["crc"])
    assert [i for i, f in enumerate(changed["flags"]) if f & FLAG_DIRTY] == [g]


def test_records_independent_of_thread_count(oracle):
    rng = np.random.default_rng(4)
    allocs = rand_allocs(rng, rng.integers(0, 20000, 30), zero_idx=(2, 9))
    a = oracle.checkpoint(allocs, 512, threads=1)
    b = oracle.checkpoint(allocs, 512, threads=7)
    for key in ("crc", "flags", "dense", "serialized"):
        assert np.array_equal(a[key], b[key]), key


# ------------------------------------------------------------------ images

def test_dense_image_layout(oracle):
    rng = np.random.default_rng(5)
    sizes = [0, 1, 17, 4096, 4097, 33]
    allocs = rand_allocs(rng, sizes)
    r = oracle.checkpoint(allocs, 4096)
    off, _, data_bytes, _ = oracle.layout(sizes, 4096)
    assert r["dense"].size == data_bytes
    for k, a in enumerate(allocs):
        o = int(off[k])
        assert np.array_equal(r["dense"][o:o + a.size], a)
        assert not r["dense"][o + a.size:o + r16(a.size)].any()    # pad is zero


def test_serialized_equals_dense_without_zero_chunks(oracle):
    rng = np.random.default_rng(6)
    allocs = [rng.integers(1, 256, int(s), dtype=np.uint8) for s in (100, 5000, 4096, 1)]
    r = oracle.checkpoint(allocs, 4096)
    assert not any(f & FLAG_ZERO for f in r["flags"])
    assert np.array_equal(r["serialized"], r["dense"])


def test_serialized_empty_when_all_zero(oracle):
    allocs = [np.zeros(s, np.uint8) for s in (100, 5000, 4096)]
    r = oracle.checkpoint(allocs, 4096)
    assert r["serialized_bytes"] == 0
    assert all(f & FLAG_ZERO for f in r["flags"])


def test_serialized_is_dense_with_zero_chunks_cut(oracle):
    rng = np.random.default_rng(8)
    C = 256
    allocs = rand_allocs(rng, [1000, 777, 2048, 300], zero_idx=(1,))
    allocs[2][256:512] = 0                       # one interior ZERO chunk
    r = oracle.checkpoint(allocs, C)
    off, _, _, _ = oracle.layout([a.size for a in allocs], C)
    want = []
    g = 0
    for k, a in enumerate(allocs):
        for start in range(0, a.size, C):
            if not r["flags"][g] & FLAG_ZERO:
                length = min(C, a.size - start)
                o = int(off[k]) + start
                want.append(r["dense"][o:o + r16(length)])
            g += 1
    assert np.array_equal(r["serialized"], np.concatenate(want))


# ------------------------------------------------------------------ deltas

def test_all_dirty_delta_equals_full_serialized(oracle):
    rng = np.random.default_rng(9)
    allocs = rand_allocs(rng, [3000, 0, 12345, 64, 8192], zero_idx=(3,))
    C = 1024
    full = oracle.checkpoint(allocs, C)
    fake_base = full["crc"] ^ np.uint32(0xFFFFFFFF)          # differs everywhere
    d = oracle.delta(allocs, C, fake_base)
    assert list(d["dirty_ids"]) == list(range(full["n_chunks"]))
    assert np.array_equal(d["delta"], full["serialized"])
    assert np.array_equal(d["crc"], full["crc"])


def test_unchanged_delta_is_empty(oracle):
    rng = np.random.default_rng(10)
    allocs = rand_allocs(rng, [3000, 12345])
    full = oracle.checkpoint(allocs, 1024)
    d = oracle.delta(allocs, 1024, full["crc"])
    assert d["dirty_ids"].size == 0 and d["delta"].size == 0
    assert not any(f & FLAG_DIRTY for f in d["flags"])


def test_delta_ids_are_exactly_changed_chunks(oracle):
    rng = np.random.default_rng(11)
    C = 512
    allocs = rand_allocs(rng, [5000, 2000, 700])
    base = oracle.checkpoint(allocs, C)
    allocs[0][0] ^= 1          # chunk 0
    allocs[0][4999] ^= 1       # chunk 9 (tail)
    allocs[2][:] = 0           # chunks of alloc 2 become ZERO and DIRTY
    d = oracle.delta(allocs, C, base["crc"])
    _, cb_, _, _ = oracle.layout([a.size for a in allocs], C)
    want = [0, 9, int(cb_[2]), int(cb_[2]) + 1]
    assert list(d["dirty_ids"]) == want
    # delta data: only the two non-ZERO dirty chunks
    assert d["delta"].size == 512 + r16(5000 - 9 * 512)


# ----------------------------------------------------------------- restore

def test_restore_round_trip(oracle):
    rng = np.random.default_rng(12)
    sizes = [0, 1, 15, 16, 4095, 4096, 4097, 10000]
    allocs = rand_allocs(rng, sizes, zero_idx=(4,))
    r = oracle.checkpoint(allocs, 4096)
    bufs, bad, ids = oracle.restore(sizes, 4096, r["crc"], r["flags"], r["serialized"])
    assert bad == 0 and ids.size == 0
    for a, b in zip(allocs, bufs):
        assert np.array_equal(a, b)


def test_restore_base_plus_delta(oracle):
    rng = np.random.default_rng(13)
    C = 1024
    sizes = [3000, 5000, 2048]
    allocs = rand_allocs(rng, sizes)
    base = oracle.checkpoint(allocs, C)
    allocs[1][1024:2048] = rng.integers(0, 256, 1024, dtype=np.uint8)
    allocs[2][:] = 0
    d = oracle.delta(allocs, C, base["crc"])
    bufs, bad, _ = oracle.restore(sizes, C, base["crc"], base["flags"], base["serialized"])
    assert bad == 0
    bad, _ = oracle.restore_delta(bufs, sizes, C, d["crc"], d["flags"], d["dirty_ids"], d["delta"])
    assert bad == 0
    for a, b in zip(allocs, bufs):
        assert np.array_equal(a, b)


def test_single_bit_flip_reports_exactly_that_chunk(oracle):
    rng = np.random.default_rng(14)
    C = 256
    sizes = [1000, 600]
    allocs = rand_allocs(rng, sizes)
    r = oracle.checkpoint(allocs, C)
    for g in range(r["n_chunks"]):
        ser = r["serialized"].copy()
        # byte 3 of serialized chunk g (all chunks non-ZERO here; each padded to 16)
        lens = [min(C, s - st) for s in sizes for st in range(0, s, C)]
        pos = sum(r16(x) for x in lens[:g]) + 3
        ser[pos] ^= 0x04
        _, bad, ids = oracle.restore(sizes, C, r["crc"], r["flags"], ser)
        assert bad == 1 and list(ids) == [g]


def test_corrupt_zero_chunk_crc_is_reported(oracle):
    allocs = [np.zeros(1000, np.uint8)]
    r = oracle.checkpoint(allocs, 256)
    crc = r["crc"].copy()
    crc[2] ^= 1
    bufs, bad, ids = oracle.restore([1000], 256, crc, r["flags"], r["serialized"])
    assert bad == 1 and list(ids) == [2]
    assert not bufs[0].any()


def test_many_bad_chunks_report_first_64_ascending(oracle):
    rng = np.random.default_rng(15)
    C = 16
    allocs = rand_allocs(rng, [16 * 100])
    r = oracle.checkpoint(allocs, C)
    crc = r["crc"] ^ np.uint32(1)
    _, bad, ids = oracle.restore([1600], C, crc, r["flags"], r["serialized"])
    assert bad == 100 and list(ids) == list(range(64))


def test_restore_rejects_short_serialized_data(oracle):
    rng = np.random.default_rng(16)
    allocs = rand_allocs(rng, [1000])
    r = oracle.checkpoint(allocs, 256)
    with pytest.raises(ValueError):
        oracle.restore([1000], 256, r["crc"], r["flags"], r["serialized"][:-16])


# ------------------------------------------- delta restore: its bad-chunk report
#
# The overlay of an increment verifies each DIRTY chunk against the
# increment's CRC and reports failures by global chunk id, exactly as the full
# restore does.  The cases below have dirty ids that do not start at 0 and a
# ZERO dirty chunk among them, so a report by position in the id list (or by
# position in the increment's data) differs from the report by chunk id.

def _delta_case(oracle, seed):
    rng = np.random.default_rng(seed)
    C = 256
    sizes = [1500, 900, 700]                 # chunks 0-5 | 6-9 | 10-12
    allocs = rand_allocs(rng, sizes)
    base = oracle.checkpoint(allocs, C)
    allocs[0][3 * C + 5] ^= 0x40             # chunk 3
    allocs[1][C:2 * C] = 0                   # chunk 7 becomes ZERO (and DIRTY)
    allocs[1][3 * C] ^= 1                    # chunk 9, the 132-byte tail of allocation 1
    allocs[2][2 * C + 10] ^= 0x80            # chunk 12, the 188-byte tail of allocation 2
    d = oracle.delta(allocs, C, base["crc"])
    assert list(d["dirty_ids"]) == [3, 7, 9, 12]
    assert d["flags"][7] & FLAG_ZERO
    # increment pieces: chunk 3 at [0, 256), chunk 9 at [256, 400), chunk 12 at [400, 592)
    assert d["delta"].size == 256 + 144 + 192
    return C, sizes, allocs, base, d


def _restore_base(oracle, C, sizes, base, ser=None, crc=None):
    return oracle.restore(sizes, C, base["crc"] if crc is None else crc, base["flags"],
                          base["serialized"] if ser is None else ser)


def test_delta_restore_clean_overlay(oracle):
    C, sizes, allocs, base, d = _delta_case(oracle, 20)
    bufs, bad, _ = _restore_base(oracle, C, sizes, base)
    assert bad == 0
    bad, ids = oracle.restore_delta(bufs, sizes, C, d["crc"], d["flags"], d["dirty_ids"], d["delta"])
    assert bad == 0 and ids.size == 0
    for a, b in zip(allocs, bufs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("piece,g,pos", [(0, 3, 17), (1, 9, 256 + 131), (2, 12, 400 + 5)])
def test_delta_restore_reports_flipped_piece_by_chunk_id(oracle, piece, g, pos):
    C, sizes, allocs, base, d = _delta_case(oracle, 21)
    bufs, bad, _ = _restore_base(oracle, C, sizes, base)
    assert bad == 0
    data = d["delta"].copy()
    data[pos] ^= 0x20
    bad, ids = oracle.restore_delta(bufs, sizes, C, d["crc"], d["flags"], d["dirty_ids"], data)
    assert bad == 1 and list(ids) == [g]
    # the flipped byte is still written where the chunk belongs
    _, cb_, _, _ = oracle.layout(sizes, C)
    k = int(np.searchsorted(cb_, g, side="right")) - 1
    at = (g - int(cb_[k])) * C + (pos - [0, 256, 400][piece])
    assert bufs[k][at] == allocs[k][at] ^ 0x20


def test_delta_restore_reports_zero_chunk_crc(oracle):
    C, sizes, allocs, base, d = _delta_case(oracle, 22)
    bufs, _, _ = _restore_base(oracle, C, sizes, base)
    crc = d["crc"].copy()
    crc[7] ^= 0x1000
    bad, ids = oracle.restore_delta(bufs, sizes, C, crc, d["flags"], d["dirty_ids"], d["delta"])
    assert bad == 1 and list(ids) == [7]
    assert not bufs[1][C:2 * C].any()          # the ZERO chunk is still filled with zeros


def test_delta_restore_reports_every_bad_dirty_chunk(oracle):
    C, sizes, allocs, base, d = _delta_case(oracle, 23)
    bufs, _, _ = _restore_base(oracle, C, sizes, base)
    crc = d["crc"] ^ np.uint32(1)              # every chunk's stored CRC is wrong
    bad, ids = oracle.restore_delta(bufs, sizes, C, crc, d["flags"], d["dirty_ids"], d["delta"])
    # only the overlaid (DIRTY) chunks are checked in this pass
    assert bad == 4 and list(ids) == [3, 7, 9, 12]


def test_delta_and_base_reports_are_separate_passes(oracle):
    """A chunk can fail in the base pass, in the overlay, or in both; each pass
    reports the chunks it checked.  A bad base chunk that the increment
    overwrites with good data fails the base pass only."""
    C, sizes, allocs, base, d = _delta_case(oracle, 24)
    lens = [min(C, s - st) for s in sizes for st in range(0, s, C)]
    at = [sum(r16(x) for x in lens[:g]) for g in range(len(lens))]   # all base chunks are non-ZERO
    ser = base["serialized"].copy()
    for g in (3, 5, 9):                         # 3 and 9 are overlaid, 5 is not
        ser[at[g] + 7] ^= 0x01
    data = d["delta"].copy()
    data[256 + 9] ^= 0x01                       # chunk 9 bad in the overlay too
    bufs, bad_b, ids_b = _restore_base(oracle, C, sizes, base, ser=ser)
    assert bad_b == 3 and list(ids_b) == [3, 5, 9]
    bad_d, ids_d = oracle.restore_delta(bufs, sizes, C, d["crc"], d["flags"], d["dirty_ids"], data)
    assert bad_d == 1 and list(ids_d) == [9]
    # chunk 3 was repaired by the overlay; chunk 5 keeps the base's bad byte
    assert np.array_equal(bufs[0][3 * C:4 * C], allocs[0][3 * C:4 * C])
    assert bufs[0][5 * C + 7] == allocs[0][5 * C + 7] ^ 0x01


def test_delta_restore_many_bad_report_first_64_ascending(oracle):
    rng = np.random.default_rng(25)
    C = 16
    allocs = rand_allocs(rng, [16 * 120])
    base = oracle.checkpoint(allocs, C)
    allocs[0][16 * 10:] = rng.integers(0, 256, 16 * 110, dtype=np.uint8)   # chunks 10-119 change
    d = oracle.delta(allocs, C, base["crc"])
    assert list(d["dirty_ids"]) == list(range(10, 120))
    bufs, _, _ = oracle.restore([16 * 120], C, base["crc"], base["flags"], base["serialized"])
    bad, ids = oracle.restore_delta(bufs, [16 * 120], C, d["crc"] ^ np.uint32(0x10), d["flags"],
                                    d["dirty_ids"], d["delta"])
    assert bad == 110 and list(ids) == list(range(10, 74))
