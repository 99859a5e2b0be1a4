"""The C ABI library loads and exports every entry point include/ckpt.h
declares; argument checks that need no GPU behave as documented."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ckpt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(ckpt_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def ck():
    from paper_2008_10596_amd import ckpt
    if not os.path.exists(ckpt.LIB_PATH):
        from paper_2008_10596_amd import build
        build.build()
    return ckpt


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for must in ("ckpt_init", "ckpt_destroy", "ckpt_register", "ckpt_unregister", "ckpt_checkpoint",
                 "ckpt_restore", "ckpt_image_info", "ckpt_image_view", "ckpt_image_serialize",
                 "ckpt_image_load", "ckpt_image_free", "ckpt_checkpoint_batch", "ckpt_server_create",
                 "ckpt_server_submit", "ckpt_server_poll", "ckpt_server_wait", "ckpt_server_stats",
                 "ckpt_server_destroy", "ckpt_strerror"):
        assert must in names, must


def test_library_exports_every_declared_symbol(ck):
    lib = ck.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and nothing C++-mangled leaks into the boundary's names
    out = subprocess.run(["nm", "-D", "--defined-only", ck.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(declared_functions()) <= exported


def test_binding_declares_every_symbol(ck):
    bound = {s[0] for s in ck.SIGNATURES}
    assert set(declared_functions()) <= bound


def test_strerror_covers_every_status(ck):
    lib = ck.lib()
    seen = set()
    for st in range(0, -11, -1):
        s = lib.ckpt_strerror(st).decode()
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 11
    assert lib.ckpt_strerror(-100).decode() == "unknown status"


def test_init_rejects_bad_configs_before_touching_a_device(ck):
    lib = ck.lib()
    h = ctypes.c_void_p()
    assert lib.ckpt_init(None, None) == ck.CKPT_E_INVAL
    for field, value in (("chunk_bytes", 8), ("chunk_bytes", 4100), ("block_threads", 100),
                         ("waves_per_chunk", 3), ("waves_per_chunk", 8), ("lane_pieces", 2),
                         ("lane_pieces", 4), ("lane_pieces", 8), ("load_hint", 3), ("table_mode", 1),
                         ("table_mode", 3)):
        cfg = ck.ckpt_config()
        setattr(cfg, field, value)
        if field == "waves_per_chunk" and value == 8:
            cfg.block_threads = 256          # 8 waves do not fit 4-wave workgroups
        assert lib.ckpt_init(ctypes.byref(cfg), ctypes.byref(h)) == ck.CKPT_E_INVAL, (field, value)


def test_image_load_rejects_malformed_buffers(ck):
    lib = ck.lib()
    out = ctypes.c_void_p()
    for buf in (b"", b"CKPTIMG1", b"NOTMAGIC" + bytes(80), b"CKPTIMG1" + bytes(80)):
        b = (ctypes.c_uint8 * max(len(buf), 1)).from_buffer_copy(buf or b"\0")
        assert lib.ckpt_image_load(None, b, len(buf), ctypes.byref(out)) == ck.CKPT_E_INVAL
    # a header that claims more rows than the buffer holds
    hdr = bytearray(b"CKPTIMG1")
    hdr += (1).to_bytes(4, "little") + (0).to_bytes(4, "little") + (4096).to_bytes(4, "little") + (16).to_bytes(4, "little")
    hdr += (1 << 40).to_bytes(8, "little") + bytes(56)
    b = (ctypes.c_uint8 * len(hdr)).from_buffer_copy(bytes(hdr))
    assert lib.ckpt_image_load(None, b, len(hdr), ctypes.byref(out)) == ck.CKPT_E_INVAL


def test_null_arguments_are_rejected(ck):
    lib = ck.lib()
    assert lib.ckpt_register(None, None, 0, 0, None) == ck.CKPT_E_INVAL
    assert lib.ckpt_unregister(None, None) == ck.CKPT_E_INVAL
    assert lib.ckpt_checkpoint(None, None, 0, None, None) == ck.CKPT_E_INVAL
    assert lib.ckpt_restore(None, None, None, None, None, None, 0, None) == ck.CKPT_E_INVAL
    assert lib.ckpt_image_info(None, None) == ck.CKPT_E_INVAL
    assert lib.ckpt_vmm_granularity(None, None) == ck.CKPT_E_INVAL
    assert lib.ckpt_vmm_alloc(None, 4096, None, None, None) == ck.CKPT_E_INVAL
    assert lib.ckpt_vmm_free(None, None) == ck.CKPT_E_INVAL
    assert lib.ckpt_restore_at(None, None, None, None, None, None) == ck.CKPT_E_INVAL
    lib.ckpt_destroy(None)
    lib.ckpt_image_free(None)


def test_host_only_failures_before_any_device_work(ck, tmp_path):
    """Calls that must fail on their arguments or files alone (no GPU here)."""
    lib = ck.lib()
    out = ctypes.c_void_p()
    # files: missing, empty, and not an image
    assert lib.ckpt_image_read_file(None, str(tmp_path / "missing.img").encode(), ctypes.byref(out)) == \
        ck.CKPT_E_NOTFOUND
    bad = tmp_path / "bad.img"
    bad.write_bytes(b"NOTANIMAGE" * 20)
    assert lib.ckpt_image_read_file(None, str(bad).encode(), ctypes.byref(out)) == ck.CKPT_E_INVAL
    bad.write_bytes(b"")
    assert lib.ckpt_image_read_file(None, str(bad).encode(), ctypes.byref(out)) == ck.CKPT_E_INVAL
    assert lib.ckpt_image_read_file(None, None, ctypes.byref(out)) == ck.CKPT_E_INVAL
    # a version-2 header that claims more allocation rows than the file holds
    hdr = bytearray(b"CKPTIMG1")
    hdr += (2).to_bytes(4, "little") + (0).to_bytes(4, "little") + (4096).to_bytes(4, "little") + \
        (16).to_bytes(4, "little")
    hdr += (3).to_bytes(8, "little") + bytes(56)
    bad.write_bytes(bytes(hdr))
    assert lib.ckpt_image_read_file(None, str(bad).encode(), ctypes.byref(out)) == ck.CKPT_E_INVAL
    # hook flags, merge, file restore and sink arguments
    assert lib.ckpt_hook_install(None, 0x80) == ck.CKPT_E_INVAL
    assert lib.ckpt_hook_install(None, 0) == ck.CKPT_OK            # uninstall: nothing installed
    a, f, x = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    assert lib.ckpt_hook_stats(ctypes.byref(a), ctypes.byref(f), ctypes.byref(x)) == ck.CKPT_OK
    assert (a.value, f.value, x.value) == (0, 0, 0)
    assert lib.ckpt_hook_malloc(0, 0, None) is None                 # 0 bytes: NULL, nothing logged
    assert lib.ckpt_hook_install(None, ck.CKPT_HOOK_CACHE | ck.CKPT_HOOK_ADDRESS_STABLE) == ck.CKPT_OK
    assert lib.ckpt_hook_cache_stats(ctypes.byref(a), ctypes.byref(f), ctypes.byref(x)) == ck.CKPT_OK
    assert (a.value, f.value, x.value) == (0, 0, 0)
    assert lib.ckpt_hook_cache_stats(None, ctypes.byref(f), ctypes.byref(x)) == ck.CKPT_E_INVAL
    assert lib.ckpt_hook_trim(ctypes.byref(a)) == ck.CKPT_OK and a.value == 0
    assert lib.ckpt_hook_trim(None) == ck.CKPT_OK
    assert lib.ckpt_hook_install(None, 0) == ck.CKPT_OK
    assert lib.ckpt_image_merge(None, None, ctypes.byref(out)) == ck.CKPT_E_INVAL
    assert lib.ckpt_restore_file_at(None, None, b"x", None, None, None) == ck.CKPT_E_INVAL
    assert lib.ckpt_image_write_file(None, b"x", 0, None) == ck.CKPT_E_INVAL
    assert lib.ckpt_image_write_file(None, b"x", ck.CKPT_FILE_DEFLATE, None) == ck.CKPT_E_INVAL


def _zip_container(version=1, block=4 << 20, head=b"", data_bytes=0, table=(), blocks=b""):
    """A compressed container (the CKPT_FILE_DEFLATE layout), fields as given."""
    out = bytearray(b"CKPTZIP1")
    out += version.to_bytes(4, "little") + block.to_bytes(4, "little")
    out += len(head).to_bytes(8, "little") + data_bytes.to_bytes(8, "little") + len(table).to_bytes(8, "little")
    for t in table:
        out += t.to_bytes(8, "little")
    return bytes(out + head + blocks)


def _empty_image_head(serial=7):
    """The serialized form of an image with no allocations: the fixed header
    alone (its CRC-section digest is FNV-1a's offset basis, no words)."""
    hdr = bytearray(b"CKPTIMG1")
    hdr += (2).to_bytes(4, "little") + (0).to_bytes(4, "little") + (4096).to_bytes(4, "little") + \
        (16).to_bytes(4, "little")
    for v in (0, 0, 0, 0, 0, serial, 0, 0xcbf29ce484222325):   # n N data ser n_dirty serial base digest
        hdr += v.to_bytes(8, "little")
    return bytes(hdr)


def test_file_info_reads_plain_and_compressed_headers(ck, tmp_path):
    """ckpt_image_file_info parses a file's header and tables alone, plain
    or inside the compressed container, with no device."""
    lib = ck.lib()
    m = ck.ckpt_image_meta()
    plain, zipped = tmp_path / "e.img", tmp_path / "e.imgz"
    plain.write_bytes(_empty_image_head(serial=7))
    zipped.write_bytes(_zip_container(head=_empty_image_head(serial=9)))
    for path, serial in ((plain, 7), (zipped, 9)):
        assert lib.ckpt_image_file_info(str(path).encode(), ctypes.byref(m)) == ck.CKPT_OK
        assert (m.mode, m.chunk_bytes, m.n_allocs, m.n_chunks, m.serialized_bytes, m.serial, m.drained) == \
            (ck.CKPT_FULL, 4096, 0, 0, 0, serial, 1)
    assert ck.file_info(str(zipped))["serial"] == 9
    bad = bytearray(_empty_image_head())
    bad[-1] ^= 1                                               # digest no longer matches
    plain.write_bytes(bytes(bad))
    assert lib.ckpt_image_file_info(str(plain).encode(), ctypes.byref(m)) == ck.CKPT_E_INVAL
    assert lib.ckpt_image_file_info(str(tmp_path / "none").encode(), ctypes.byref(m)) == ck.CKPT_E_NOTFOUND
    assert lib.ckpt_image_file_info(None, ctypes.byref(m)) == ck.CKPT_E_INVAL
    assert lib.ckpt_image_file_info(str(zipped).encode(), None) == ck.CKPT_E_INVAL


def test_compressed_container_is_checked_before_any_device_work(ck, tmp_path):
    """Malformed compressed containers fail on their header and block table
    alone: nothing is allocated or inflated."""
    lib = ck.lib()
    out = ctypes.c_void_p()
    path = tmp_path / "z.img"
    raw = 1 << 63

    def rc(data):
        path.write_bytes(data)
        return lib.ckpt_image_read_file(None, str(path).encode(), ctypes.byref(out))

    assert rc(b"CKPTZIP1" + bytes(10)) == ck.CKPT_E_INVAL                    # header cut short
    assert rc(_zip_container(version=2)) == ck.CKPT_E_INVAL                 # unknown version
    assert rc(_zip_container(block=0)) == ck.CKPT_E_INVAL                   # zero block size
    assert rc(_zip_container(data_bytes=(1 << 64) - 1, table=(raw | 5,))) == ck.CKPT_E_INVAL   # DATA too large
    # the block count must be ceil(DATA / block)
    assert rc(_zip_container(data_bytes=5 << 20, table=(raw | (4 << 20),))) == ck.CKPT_E_INVAL
    # a raw block must hold exactly its share of DATA, and carry no plane code
    assert rc(_zip_container(data_bytes=100, table=(raw | 99,), blocks=bytes(99))) == ck.CKPT_E_INVAL
    assert rc(_zip_container(data_bytes=100, table=(raw | (1 << 61) | 100,), blocks=bytes(100))) == \
        ck.CKPT_E_INVAL
    # plane code 3 is not defined
    assert rc(_zip_container(data_bytes=100, table=((3 << 61) | 20,), blocks=bytes(20))) == ck.CKPT_E_INVAL
    # the table may not run past the end of the file
    assert rc(_zip_container(data_bytes=100, table=(raw | 100,), blocks=bytes(60))) == ck.CKPT_E_INVAL
    # nor leave bytes after the last block
    assert rc(_zip_container(data_bytes=100, table=(raw | 100,), blocks=bytes(101))) == ck.CKPT_E_INVAL
    # a consistent table around a head that is not an image header
    assert rc(_zip_container(head=b"NOTANIMAGEHEAD" * 8, data_bytes=100, table=(raw | 100,),
                             blocks=bytes(100))) == ck.CKPT_E_INVAL
