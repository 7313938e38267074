"""Sanitizer builds of the host-side code (CPU only).

* The FP64 oracle is rebuilt with AddressSanitizer and UndefinedBehaviorSanitizer
  and the oracle's own test files run again against that build in a child
  process (the sanitizer runtimes preloaded there; skipped where the process
  already runs under a preloaded library, which a sanitizer runtime must
  precede).
* The frame server's host bookkeeping (tests/server_host_check.cpp: the device
  arena allocator, the per-frame inlier-mask re-basing, the entry points'
  argument checks) is built with g++ under both sanitizers and run.

Equivalent commands, for a shell:
  gcc -O1 -g -fno-omit-frame-pointer -fsanitize=address,undefined \\
      -fno-sanitize-recover=undefined -std=c11 -ffp-contract=off -fPIC -shared \\
      -o /tmp/liboracle_asan.so oracle/rv_oracle.c oracle/rv_oracle_paper.c -lm -lpthread
  RV_ORACLE_LIB=/tmp/liboracle_asan.so ASAN_OPTIONS=detect_leaks=0 \\
      LD_PRELOAD="$(gcc -print-file-name=libasan.so) $(gcc -print-file-name=libubsan.so)" \\
      python -m pytest tests/test_oracle_*.py tests/test_parity_protocol.py
  g++ -std=c++17 -O1 -g -fsanitize=address,undefined -D__HIP_PLATFORM_AMD__ \\
      -I/opt/rocm/include -Iinclude -o /tmp/server_host_check tests/server_host_check.cpp \\
      -L/opt/rocm/lib -lamdhip64 -lpthread && /tmp/server_host_check
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=undefined"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _preloaded():
    if os.environ.get("LD_PRELOAD"):
        return True
    try:
        return bool(open("/etc/ld.so.preload").read().strip())
    except OSError:
        return False


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_tests_under_asan_and_ubsan(tmp_path):
    if _preloaded():
        pytest.skip("a preloaded library is present; the sanitizer runtime must come first")
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if asan is None or ubsan is None:
        pytest.skip("gcc sanitizer runtimes not found")
    lib = tmp_path / "liboracle_asan.so"
    subprocess.run(["gcc", *SAN, "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-o", str(lib), os.path.join(ROOT, "oracle", "rv_oracle.c"),
                    os.path.join(ROOT, "oracle", "rv_oracle_paper.c"), "-lm", "-lpthread"],
                   check=True)
    env = dict(os.environ, RV_ORACLE_LIB=str(lib), LD_PRELOAD=f"{asan} {ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    files = ["tests/test_oracle_estimate.py", "tests/test_oracle_philox.py",
             "tests/test_oracle_paper.py", "tests/test_oracle_band.py",
             "tests/test_parity_protocol.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *files],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists("/opt/rocm/include"),
                    reason="g++ or the ROCm headers not found")
def test_server_host_logic_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "server_host_check"
    subprocess.run(["g++", "-std=c++17", *SAN, "-Wno-subobject-linkage", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-o", str(exe),
                    os.path.join(ROOT, "tests", "server_host_check.cpp"), "-L/opt/rocm/lib",
                    "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lpthread"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "server host checks passed" in r.stdout
