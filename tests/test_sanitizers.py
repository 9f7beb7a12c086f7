"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The library's host part (plans, schedules, work-item tables, workspace
checks, the communication-cost model, the LU plan) is built with
-fsanitize=address,undefined on the host pass only and the ABI and
cost-model tests run against it with clang's ASan runtime preloaded; the
oracle's C code is built with gcc's sanitizers and its pins run with gcc's
runtimes preloaded.  Each suite runs in a subprocess (the runtime must be
the process's first library); a report aborts it.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(compiler, name):
    try:
        out = subprocess.run([compiler, "-print-file-name=" + name], capture_output=True,
                             text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return out if os.path.isabs(out) and os.path.exists(out) else None


def _pytest(files, env):
    cmd = [sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider"] + files
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
    return r.stdout


def test_library_host_code_under_asan_ubsan(tmp_path):
    clang = "/opt/rocm/llvm/bin/clang"
    rt = _runtime(clang, "libclang_rt.asan-x86_64.so") if os.path.exists(clang) else None
    if rt is None or shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("ROCm clang ASan runtime or hipcc not available")
    from paper_1306_4161_amd import build
    lib = build.build(verbose=False, sanitize=True, out_dir=str(tmp_path))
    env = dict(os.environ, LD_PRELOAD=rt, HSUMMA_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    _pytest(["tests/test_abi.py", "tests/test_cost_model.py"], env)


def test_oracle_under_asan_ubsan(tmp_path):
    asan, ubsan = _runtime("gcc", "libasan.so"), _runtime("gcc", "libubsan.so")
    if asan is None or ubsan is None:
        pytest.skip("gcc sanitizer runtimes not available")
    env = dict(os.environ, LD_PRELOAD=asan + ":" + ubsan, HSUMMA_ORACLE_SANITIZE="1",
               HSUMMA_ORACLE_LIBRARY=str(tmp_path / "liboracle_asan.so"),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    _pytest(["tests/test_oracle.py", "tests/test_lu_ref.py", "tests/test_split_ref.py"], env)
