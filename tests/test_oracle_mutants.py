"""Mutation tests for the oracle's pins.

Each case plants one plausible mistake in a copy of oracle/ckpt_oracle.c (a
wrong constant, a dropped term, an off-by-one, an inverted test), builds it,
and runs the oracle pin suite against that build in a subprocess.  The pins are
only worth something if every such mistake makes at least one of them fail.
"""
import os
import subprocess
import sys

import pytest

from oracle import oracle as o

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = [os.path.join(ROOT, "tests", "test_oracle_crc.py"),
        os.path.join(ROOT, "tests", "test_oracle_image.py")]

MUTANTS = [
    ("crc32_poly_instead_of_crc32c",
     "#define ORACLE_POLY_REFLECTED 0x82F63B78u", "#define ORACLE_POLY_REFLECTED 0xEDB88320u"),
    ("xorout_dropped",
     "        r = crc_table[(r ^ p[i]) & 0xFFu] ^ (r >> 8);\n    return r ^ 0xFFFFFFFFu;",
     "        r = crc_table[(r ^ p[i]) & 0xFFu] ^ (r >> 8);\n    return r;"),
    ("init_zero",
     "    uint32_t r = 0xFFFFFFFFu;\n    for (size_t i = 0; i < n; i++)\n        r = crc_table",
     "    uint32_t r = 0;\n    for (size_t i = 0; i < n; i++)\n        r = crc_table"),
    ("register_shift_wrong", "^ (r >> 8);", "^ (r >> 7);"),
    ("table_index_masks_7_bits", "(r ^ p[i]) & 0xFFu]", "(r ^ p[i]) & 0x7Fu]"),
    ("tail_chunk_dropped", "return (size + C - 1) / C;", "return size / C;"),
    ("no_16_byte_rounding",
     "return (x + ORACLE_ALIGN - 1) / ORACLE_ALIGN * ORACLE_ALIGN;", "return x;"),
    ("chunk_len_off_by_one", "uint64_t rest = size - c * C;", "uint64_t rest = size - c * C - 1;"),
    ("zero_test_skips_first_byte",
     "for (uint64_t i = 0; i < n; i++)\n        if (p[i] != 0)",
     "for (uint64_t i = 1; i < n; i++)\n        if (p[i] != 0)"),
    ("dirty_test_inverted", "j->base_crc[g] != crc", "j->base_crc[g] == crc"),
    ("dense_pad_not_zeroed",
     "            memset(dense + o + sizes[k], 0, round_up16(sizes[k]) - sizes[k]);\n", ""),
    ("dense_offsets_unpadded",
     "            o += round_up16(sizes[k]);\n        }\n    }", "            o += sizes[k];\n        }\n    }"),
    ("serialized_pad_not_zeroed",
     "            memset(ser + s + len, 0, round_up16(len) - len);\n", ""),
    ("serialized_keeps_zero_chunks",
     "        if (flags[g] & ORACLE_FLAG_ZERO)\n            continue;\n        if (ser) {",
     "        if (ser) {"),
    ("delta_ids_skip_zero_chunks",
     "        if (!(flags[g] & ORACLE_FLAG_DIRTY))\n            continue;\n        if (dirty_ids)",
     "        if (!(flags[g] & ORACLE_FLAG_DIRTY) || (flags[g] & ORACLE_FLAG_ZERO))\n            continue;\n        if (dirty_ids)"),
    ("restore_skips_zero_fill", "        memset(dst, 0, len);\n    else", "        ;\n    else"),
    ("restore_never_reports", "        report_bad(rep, g);\n", "        (void)rep;\n"),
    ("delta_report_uses_list_position",
     "            piece = delta + s;\n            s += round_up16(len);\n        }\n"
     "        restore_chunk(dst[k] + c * C, len, flags[g], crc[g], piece, g, &rep);",
     "            piece = delta + s;\n            s += round_up16(len);\n        }\n"
     "        restore_chunk(dst[k] + c * C, len, flags[g], crc[g], piece, i - 1, &rep);"),
    ("delta_pass_never_reports",
     "            piece = delta + s;\n            s += round_up16(len);\n        }\n"
     "        restore_chunk(dst[k] + c * C, len, flags[g], crc[g], piece, g, &rep);",
     "            piece = delta + s;\n            s += round_up16(len);\n        }\n"
     "        { bad_report unused; memset(&unused, 0, sizeof(unused));\n"
     "          restore_chunk(dst[k] + c * C, len, flags[g], crc[g], piece, g, &unused); }"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new):
    src = open(o.SRC).read()
    assert src.count(old) == 1, "mutation site not unique or missing: " + name
    mutant_c = tmp_path / "mutant.c"
    mutant_c.write_text(src.replace(old, new))
    mutant_so = str(tmp_path / "libmutant.so")
    o.build(out=mutant_so, src=str(mutant_c), extra=("-w",))
    env = dict(os.environ, CKPT_ORACLE_LIB=mutant_so)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-p", "no:randomly", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, "mutant %s survived the pins:\n%s" % (name, r.stdout[-2000:])
