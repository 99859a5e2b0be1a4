"""Bit-at-a-time CRC-32C and tiny pure-Python chunk records.

TEST INFRASTRUCTURE ONLY: used by tests/ to pin the C oracle; never imported by
the product package.

CRC-32C (Castagnoli) as a bitwise definition: register starts at 0xFFFFFFFF;
each message byte is XORed into the low byte, then eight single-bit steps each
shift right by one and XOR the reflected polynomial 0x82F63B78 when the bit
shifted out was 1; the result is the register XOR 0xFFFFFFFF.  The paper fixes
no checksum: CRC-32C per chunk is this library's choice of check for the
chunks the paper's drain (Sec. 3.2, "Saving the library-allocated arena")
copies out and its refill copies back.

Everything here is written for clarity on inputs of at most a few kilobytes.
"""

POLY_REFLECTED = 0x82F63B78


def crc32c_bitwise(data, init=0xFFFFFFFF, xorout=0xFFFFFFFF):
    """CRC-32C of `data` (bytes-like) one bit at a time."""
    r = init
    for b in bytes(data):
        r ^= b
        for _ in range(8):
            if r & 1:
                r = (r >> 1) ^ POLY_REFLECTED
            else:
                r >>= 1
    return r ^ xorout


def chunk_records(allocs, C, base_crc=None):
    """Per-chunk (crc, flags) for a list of allocations, by direct definition.

    Each allocation is cut into pieces of C bytes (the last may be shorter);
    chunk ids run over allocations in order.  flags bit 0 = every byte is
    zero, bit 1 = no base CRC or the CRC differs from base_crc[g].
    """
    crcs, flags = [], []
    for a in allocs:
        a = bytes(a)
        for start in range(0, len(a), C):
            piece = a[start:start + C]
            g = len(crcs)
            crc = crc32c_bitwise(piece)
            zero = all(x == 0 for x in piece)
            dirty = base_crc is None or base_crc[g] != crc
            crcs.append(crc)
            flags.append(int(zero) | (int(dirty) << 1))
    return crcs, flags
