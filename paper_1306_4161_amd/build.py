"""Build libhsumma.so (all HIP sources in csrc/) for gfx950, in-tree.

    python -m paper_1306_4161_amd.build             # libhsumma.so
    python -m paper_1306_4161_amd.build --sanitize  # libhsumma_asan.so

Every HIP translation unit is compiled with hipcc for gfx950 only, with the
packed-FP32 instructions disabled, then linked into one shared library next
to this file.  No host compiler flags differ from hipcc's defaults.  The
sanitized variant instruments the host code only (AddressSanitizer and
UndefinedBehaviorSanitizer; every -fsanitize flag goes to the host pass
through -Xarch_host) for CPU runs of the plan, schedule and cost-model
code with the clang ASan runtime preloaded; its device code is the same.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhsumma.so")
ASAN_BUILD = os.path.join(HERE, "_build_asan")
ASAN_LIB = os.path.join(HERE, "libhsumma_asan.so")
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libhsumma.so)")


COMMON = [
    "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-Wno-unused-result",
]


def _compile(src: str, build_dir: str, extra) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [hipcc()] + COMMON + list(extra) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build(verbose: bool = True, sanitize: bool = False, out_dir: str | None = None) -> str:
    """Build the library; out_dir (sanitized builds) puts objects and library there."""
    build_dir, lib = (ASAN_BUILD, ASAN_LIB) if sanitize else (BUILD, LIB)
    if sanitize and out_dir:
        build_dir, lib = os.path.join(out_dir, "obj"), os.path.join(out_dir, "libhsumma_asan.so")
    extra = SANITIZE if sanitize else []
    os.makedirs(build_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, extra), srcs))
    tmp = lib + ".tmp%d" % os.getpid()
    # roctx: named ranges per outer step for rocprofv3 --marker-trace
    link_extra = ["-Xarch_host", "-shared-libasan"] + SANITIZE if sanitize else []
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + link_extra + objs + [
        "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, lib)
    if verbose:
        print("built", lib, file=sys.stderr)
    return lib


if __name__ == "__main__":
    build(sanitize="--sanitize" in sys.argv[1:])
