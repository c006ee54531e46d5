"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU
oracle (every counter on random small hypergraphs, with the identities that
tie them together) and the library's host-only pattern tables.  Built with
g++ (host code only; no device code is instrumented), run here on the CPU."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import patterns

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def build_and_run(cmd, exe, args=()):
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([exe, *args], capture_output=True, text=True, env=ENV, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
    return res.stdout


def test_oracle_under_sanitizers(tmp_path):
    canon = tmp_path / "canon.bin"
    parent = tmp_path / "parent.bin"
    np.ascontiguousarray(patterns.canonical_code_to_id3(), dtype=np.int32).tofile(canon)
    np.ascontiguousarray(patterns.id3_to_id26(), dtype=np.int32).tofile(parent)
    exe = str(tmp_path / "oracle_san")
    out = build_and_run(["g++", "-std=c++17", "-fopenmp", *SAN, "-o", exe,
                         os.path.join(ROOT, "oracle", "mochy_oracle.cpp"),
                         os.path.join(ROOT, "tests", "sanitize", "oracle_driver.cpp")],
                        exe, [str(canon), str(parent)])
    assert "oracle ok" in out


def test_library_host_tables_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tables_san")
    out = build_and_run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                         "-I", os.path.join(ROOT, "include"),
                         "-I", os.path.join(ROOT, "paper_2310_15668_amd", "csrc"), "-o", exe,
                         os.path.join(ROOT, "paper_2310_15668_amd", "csrc", "patterns.cpp"),
                         os.path.join(ROOT, "tests", "sanitize", "library_host_driver.cpp")], exe)
    assert "431 3h ids, 26 h ids" in out
