// crc_tables.cpp -- CRC-32C shift-operator tables for the GPU kernels.
//
// The CRC register is a linear function over GF(2) of its previous value and
// the data, so "feed m zero bytes" is a 32 x 32 bit matrix.  Its columns are
// found by running each single-bit register value through m zero bytes (bit by
// bit, or by powers of the one-byte operator for long runs); a table entry for
// byte position j and byte value b is the XOR of the columns of b's set bits,
// shifted to position j.
#include <vector>

#include "internal.h"

namespace ckpt {

// One zero bit through the reflected register.
static uint32_t step_bit(uint32_t r) { return (r & 1u) ? (r >> 1) ^ kPolyReflected : (r >> 1); }

// The operator m applied to v: the XOR of m's columns at v's set bits.
static uint32_t apply_op(const uint32_t *m, uint32_t v)
{
    uint32_t r = 0;
    for (int i = 0; v; i++, v >>= 1)
        if (v & 1u)
            r ^= m[i];
    return r;
}

uint32_t host_shift(uint32_t reg, uint64_t nbytes)
{
    if (nbytes <= 64) {
        for (uint64_t i = 0; i < 8 * nbytes; i++)
            reg = step_bit(reg);
        return reg;
    }
    // Powers of the one-byte operator (its columns run bit by bit): the
    // operator for 2^k bytes is the square of the one for 2^(k-1), and the
    // register passes the power for each set bit of nbytes.  The powers of one
    // operator commute, so the order does not matter.
    uint32_t op[32], sq[32];
    for (int i = 0; i < 32; i++) {
        uint32_t c = 1u << i;
        for (int b = 0; b < 8; b++)
            c = step_bit(c);
        op[i] = c;
    }
    while (nbytes) {
        if (nbytes & 1)
            reg = apply_op(op, reg);
        nbytes >>= 1;
        if (nbytes) {
            for (int i = 0; i < 32; i++)
                sq[i] = apply_op(op, op[i]);
            for (int i = 0; i < 32; i++)
                op[i] = sq[i];
        }
    }
    return reg;
}

// out[j*256 + b] = shift(b << 8j, m)
static void build_operator(uint32_t *out, uint64_t m)
{
    uint32_t col[32];
    for (int i = 0; i < 32; i++)
        col[i] = host_shift(1u << i, m);
    for (int j = 0; j < 4; j++)
        for (int b = 0; b < 256; b++) {
            uint32_t v = 0;
            for (int i = 0; i < 8; i++)
                if (b & (1 << i))
                    v ^= col[8 * j + i];
            out[j * 256 + b] = v;
        }
}

void build_tables_replicated(uint32_t *out, uint32_t rounds_per_wave, uint32_t gap_bytes)
{
    std::vector<uint32_t> op(kTabWords);
    // the gap operator (one round, or the quad form's skip), 8 copies per entry
    build_operator(op.data(), gap_bytes);
    for (int j = 0; j < 4; j++)
        for (int b = 0; b < 256; b++)
            for (int r = 0; r < 8; r++)
                out[((j << 13) | (b << 5) | (r << 2)) / 4] = op[j * 256 + b];
    // 2-byte chain step: entry t, b = the register value b << 8t moved 2 bytes
    build_operator(op.data(), 2);
    for (int t = 0; t < 2; t++)
        for (int b = 0; b < 256; b++)
            for (int r = 0; r < 32; r++)
                out[(kRepChainOff + ((b << 8) | (t << 7) | (r << 2))) / 4] = op[t * 256 + b];
    uint32_t *tail = out + kRepTreeOff / 4;
    for (int k = 0; k < kTreeLevels; k++)
        build_operator(tail + k * kTabWords, 16ull << k);
    build_operator(tail + kTreeLevels * kTabWords, (uint64_t)rounds_per_wave * kRoundBytes);
}

}  // namespace ckpt
