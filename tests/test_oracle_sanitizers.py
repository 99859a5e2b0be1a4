"""The oracle's pins, run against an AddressSanitizer + UndefinedBehaviorSanitizer
build of the oracle (host code only, gcc): any out-of-bounds access, use of
freed memory or undefined behaviour in the oracle aborts the run."""
import os
import subprocess
import sys

import pytest

from oracle import oracle as o

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = [os.path.join(ROOT, "tests", "test_oracle_crc.py"),
        os.path.join(ROOT, "tests", "test_oracle_image.py")]


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="no AddressSanitizer runtime")
def test_oracle_pins_pass_under_asan_ubsan(tmp_path):
    so = str(tmp_path / "liboracle_asan.so")
    o.build(out=so, extra=("-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined"))
    env = dict(os.environ, CKPT_ORACLE_LIB=so, LD_PRELOAD=_runtime("libasan.so"),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-k", "not property", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
