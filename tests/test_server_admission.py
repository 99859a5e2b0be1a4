"""The serving loop's admission policy on the CPU (no device): the host logic
of paper_2008_10596_amd/csrc/admission.h driven through random and hand-made
sequences of submit / admit / finish / image release by
tests/admission_check.cpp, built with AddressSanitizer and
UndefinedBehaviorSanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_admission_state_machine_under_sanitizers(tmp_path):
    exe = str(tmp_path / "admission_check")
    src = os.path.join(ROOT, "tests", "admission_check.cpp")
    inc = os.path.join(ROOT, "paper_2008_10596_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-I", inc, src, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks held" in r.stdout
