"""Build libckpt.so (HIP kernels + host runtime) for gfx950 with hipcc.

Usage: python -m paper_2008_10596_amd.build   (or build() from Python)
The library is built in-tree, next to this file.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libckpt.so")
# plain HBM read/write/copy kernels for the bench's ceilings (not on the path)
PROBE_LIB = os.path.join(HERE, "libckpt_probe.so")
PROBE_SOURCE = "probe.hip"
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["kernels.hip", "crc_tables.cpp", "runtime.cpp", "server.cpp", "vmm.cpp", "hook.cpp", "sink.cpp", "noalloc.cpp"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
    "-I" + INCLUDE, "-I" + CSRC,
    # no packed fp32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def build(verbose=False, extra=()):
    """Compile every source (in parallel) and link libckpt.so and
    libckpt_probe.so.  Always recompiles."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, "--offload-arch=" + ARCH, *COMMON, *extra, "-c", path, "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd))
        cmds.append(cmd)
        objs.append(obj)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "0") or 0) or (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread", "-lz"]
    if verbose:
        print(" ".join(cmd))
    _run(cmd)
    os.replace(tmp, LIB)
    tmp = PROBE_LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, *COMMON, *extra, "-shared", "-o", tmp,
           os.path.join(CSRC, PROBE_SOURCE)]
    if verbose:
        print(" ".join(cmd))
    _run(cmd)
    os.replace(tmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
