"""The library's host-side set-up code under AddressSanitizer and UBSan.

Compiles tests/sanitize/host_checks.cpp together with the host-only library
sources (mesh construction, P1 assembly, colouring and restriction tables,
Morton orders, the dense Jacobi eigensolver) by clang++ with
-fsanitize=address,undefined (host code only: these sources hold no device
code), and runs it: every level of four surfaces is built and checked, the
dense eigensolver is checked on four coarse levels, and malformed inputs must
be rejected.  Any sanitizer report aborts the run.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1511_07042_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
HOST_SOURCES = ["mesh.cpp", "assemble.cpp", "dense_host.cpp", "order.cpp"]


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not installed")
def test_host_setup_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_checks")
    cmd = [CLANG, "-x", "c++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-w",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           "-I" + CSRC, os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp")]
    cmd += [os.path.join(CSRC, s) for s in HOST_SOURCES] + ["-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
