"""Host code under AddressSanitizer, UndefinedBehaviorSanitizer and
ThreadSanitizer (CPU only).

The C oracle (with clang) and the library's host set-up code (setup.cpp:
coefficient fit, Courant limit, electron loading, laser fields, with g++) are
built with -fsanitize=address,undefined, and driven over modes 0..3 by the small
programs in tests/sanitize/.  Any out-of-bounds access, leak or undefined
behaviour aborts the run.  The host set-up code is also built with
-fsanitize=thread and called from several threads at once, since contexts may
be created on different threads.  (Device code is not built with sanitizers
here.)
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_and_run(cmd, exe, tmp_path, env_extra=None):
    if shutil.which(cmd[0]) is None:
        pytest.skip(f"{cmd[0]} not available")
    r = subprocess.run(cmd + ["-o", str(exe)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               **(env_extra or {}))
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "runtime error" not in r.stderr, (r.returncode, r.stderr[-3000:])
    return r.stdout


# clang for the C oracle: gcc's AddressSanitizer (gcc 11) leaves _Complex
# double loads and stores uninstrumented, and every oracle field array is
# complex (a write one element past a field array went unreported under gcc
# and is reported under clang)
CLANG = shutil.which("clang") or "/opt/rocm/llvm/bin/clang"


def test_oracle_under_sanitizers(tmp_path):
    cc = CLANG if os.path.exists(CLANG) else "gcc"
    out = _build_and_run([cc, "-std=c11", *SAN, os.path.join(ROOT, "tests", "sanitize", "oracle_run.c"),
                          os.path.join(ROOT, "oracle", "q3d_oracle.c"), "-lm"], tmp_path / "oracle_run", tmp_path)
    assert "oracle ok" in out


def test_host_setup_under_sanitizers(tmp_path):
    out = _build_and_run(["g++", "-std=c++17", *SAN, "-pthread", "-I", os.path.join(ROOT, "include"),
                          os.path.join(ROOT, "tests", "sanitize", "host_run.cpp"),
                          os.path.join(ROOT, "paper_2303_12874_amd", "csrc", "setup.cpp")], tmp_path / "host_run",
                         tmp_path)
    assert "host ok" in out


def test_host_setup_from_threads_under_thread_sanitizer(tmp_path):
    out = _build_and_run(["g++", "-std=c++17", "-fsanitize=thread", "-fno-omit-frame-pointer", "-g", "-O1", "-pthread",
                          "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize", "host_threads.cpp"),
                          os.path.join(ROOT, "paper_2303_12874_amd", "csrc", "setup.cpp")], tmp_path / "host_threads",
                         tmp_path, {"TSAN_OPTIONS": "halt_on_error=1"})
    assert "threads ok" in out


def test_cell_sort_integrity_flags_on_host(tmp_path):
    """The checks the sort kernels make (which bit a bad tile range, slot,
    source or count raises) and the message the synchronising calls return,
    built for the host under the sanitizers."""
    out = _build_and_run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
                          os.path.join(ROOT, "tests", "sanitize", "sort_flags.cpp"),
                          os.path.join(ROOT, "paper_2303_12874_amd", "csrc", "setup.cpp")], tmp_path / "sort_flags",
                         tmp_path)
    assert "sort flags ok" in out
