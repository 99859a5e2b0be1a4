"""Pins for the oracle's CRC-32C: published values, the bitwise definition,
and GF(2) identities that any correct CRC-32C satisfies."""
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import crc_bitwise as cb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "crc32c_vectors.txt")


def _parse_input(spec):
    kind, _, rest = spec.partition(":")
    if kind == "ascii":
        return rest.encode("ascii")
    if kind == "repeat":
        byte, count = rest.split(":")
        return bytes([int(byte, 16)]) * int(count)
    if kind == "range":
        a, b, s = (int(x) for x in rest.split(":"))
        return bytes(range(a, b, s))
    raise ValueError(spec)


def golden_vectors():
    out = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, spec, want, _src = (x.strip() for x in line.split("|"))
            out.append((name, _parse_input(spec), int(want, 16)))
    return out


VECTORS = golden_vectors()


def test_golden_file_has_the_published_vectors():
    assert {v[0] for v in VECTORS} == {"check_value", "rfc3720_zeros", "rfc3720_ones",
                                        "rfc3720_incr", "rfc3720_decr"}


@pytest.mark.parametrize("name,data,want", VECTORS, ids=[v[0] for v in VECTORS])
def test_published_vectors(oracle, name, data, want):
    assert cb.crc32c_bitwise(data) == want          # Python, bit at a time
    assert oracle.crc32c_bitwise_c(data) == want    # C, bit at a time
    assert oracle.crc32c(data) == want              # C, Sarwate table (the oracle's)


def test_empty_message_is_zero(oracle):
    # init ^ xorout with no bytes processed
    assert oracle.crc32c(b"") == 0 == cb.crc32c_bitwise(b"")


def test_derived_zero_values(oracle):
    # Regression values derived from the definition (not independent): the CRC
    # of zeros is not zero, so ZERO cannot be read off the CRC.
    assert oracle.crc32c(bytes(4096)) == 0x98F94189
    assert oracle.crc32c(bytes(1)) == 0x527D5351


def test_table_entries_match_single_byte_definition(oracle):
    t = oracle.crc32c_table()
    for b in range(256):
        # table[b] is the register after feeding b into a zero register
        assert int(t[b]) == cb.crc32c_bitwise(bytes([b]), init=0, xorout=0), b


def test_table_crc_matches_bitwise_on_random_lengths(oracle):
    rng = np.random.default_rng(2008)
    lengths = list(range(0, 40)) + list(rng.integers(40, 5001, 40))
    for n in lengths:
        data = rng.integers(0, 256, int(n), dtype=np.uint8).tobytes()
        assert oracle.crc32c(data) == cb.crc32c_bitwise(data), n


@settings(max_examples=200, deadline=None)
@given(st.binary(min_size=0, max_size=300))
def test_table_crc_matches_bitwise_property(data):
    from oracle import oracle as o
    assert o.crc32c(data) == cb.crc32c_bitwise(data)


# ---- GF(2) structure: combine law, affine law, chunk-size consistency ------

def shift(reg, nbytes):
    """Feed nbytes zero bytes through the register (no init, no xorout)."""
    return cb.crc32c_bitwise(bytes(nbytes), init=reg, xorout=0)


def combine(crc_a, crc_b, len_b):
    """CRC(A || B) from CRC(A), CRC(B) and len(B): the init/xorout terms of B
    cancel against those carried by A, leaving shift(CRC(A), len B) ^ CRC(B)."""
    return shift(crc_a, len_b) ^ crc_b


def test_combine_law_all_splits(oracle):
    rng = np.random.default_rng(12701)
    for n in (0, 1, 2, 3, 4, 5, 15, 16, 17, 33, 64):
        msg = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
        whole = oracle.crc32c(msg)
        for cut in range(n + 1):
            a, b = msg[:cut], msg[cut:]
            assert combine(oracle.crc32c(a), oracle.crc32c(b), len(b)) == whole, (n, cut)


def test_affine_law(oracle):
    rng = np.random.default_rng(7)
    for n in (1, 7, 16, 100, 4096):
        a = rng.integers(0, 256, n, dtype=np.uint8)
        b = rng.integers(0, 256, n, dtype=np.uint8)
        lhs = oracle.crc32c((a ^ b).tobytes())
        rhs = oracle.crc32c(a.tobytes()) ^ oracle.crc32c(b.tobytes()) ^ oracle.crc32c(bytes(n))
        assert lhs == rhs


def test_chunk_size_consistency(oracle):
    # a 16 KiB chunk's CRC is the fold of its four 4 KiB chunks' CRCs
    rng = np.random.default_rng(16)
    data = rng.integers(0, 256, 16384, dtype=np.uint8).tobytes()
    parts = [oracle.crc32c(data[i:i + 4096]) for i in range(0, 16384, 4096)]
    acc = parts[0]
    for p in parts[1:]:
        acc = combine(acc, p, 4096)
    assert acc == oracle.crc32c(data)
