"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two builds with gcc/g++ and -fsanitize=address,undefined (no recovery):
  * the FP64 oracle (oracle/oracle.c) driven by tests/sanitize/oracle_driver.c
    on small seeded systems, including multi-image periodic boxes, an open
    domain with ghosts, isolated and single atoms;
  * the library's model-header reader (paper_2506_04055_amd/csrc/
    header_json.h, host-only C++) driven by tests/sanitize/json_fuzz.cpp with
    valid, truncated, mutated and random headers.
Any sanitizer report makes the program exit non-zero.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _build_and_run(tmp_path, compiler, sources, extra, name):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    exe = str(tmp_path / name)
    r = subprocess.run([compiler, *SAN, *extra, *sources, "-o", exe, "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "gcc", [os.path.join(ROOT, "oracle", "oracle.c"),
                                           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")],
                         ["-std=gnu11", "-fopenmp"], "oracle_san")
    assert out.count(" ok") == 6


def test_header_reader_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "g++", [os.path.join(ROOT, "tests", "sanitize", "json_fuzz.cpp")],
                         ["-std=c++17"], "json_san")
    assert "0 failures" in out
