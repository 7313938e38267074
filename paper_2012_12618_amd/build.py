"""Build the gfx950 shared library ``_lib/librv.so`` from ``csrc/rv.hip`` (kernels
and estimator entry points), ``csrc/rv_paper.hip`` (paper-literal variant) and
``csrc/rv_server.cpp`` (frame server); the measurement program
``_lib/issue_probe`` from ``csrc/issue_probe.hip`` (instruction issue rates,
run by ``bench.py --workload issue-rates``); and ``_lib/rv_cli`` from
``csrc/rv_cli.cpp`` (a frame from raw files through the C ABI alone).

Usage: ``python -m paper_2012_12618_amd.build`` (also called by the repository's
``__graft_entry__.build()``).  hipcc cross-compiles for gfx950 without a GPU.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", n) for n in ("rv.hip", "rv_paper.hip", "rv_server.cpp")]
INCLUDE = os.path.join(ROOT, "include")
LIB_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIB_DIR, "librv.so")
PROBE_SRC = os.path.join(HERE, "csrc", "issue_probe.hip")
PROBE = os.path.join(LIB_DIR, "issue_probe")
CLI_SRC = os.path.join(HERE, "csrc", "rv_cli.cpp")
CLI = os.path.join(LIB_DIR, "rv_cli")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc_path() -> str:
    return os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _hipcc(cmd: list[str], verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the GPU-only target feature; that warning is harmless.
    noise = "not a recognized feature for this target"
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines() if ln.strip() and noise not in ln]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))


def build(verbose: bool = False, extra_flags: list[str] | None = None) -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB + ".tmp"
    _hipcc([hipcc_path(), *HIP_FLAGS, *(extra_flags or []), "-I", INCLUDE, "-o", tmp, *SRCS], verbose)
    os.replace(tmp, LIB)
    probe_flags = [f for f in HIP_FLAGS if f not in ("-fPIC", "-shared")]
    _hipcc([hipcc_path(), *probe_flags, "-o", PROBE + ".tmp", PROBE_SRC], verbose)
    os.replace(PROBE + ".tmp", PROBE)
    _hipcc([hipcc_path(), *probe_flags, "-I", INCLUDE, "-o", CLI + ".tmp", CLI_SRC, "-L", LIB_DIR,
            "-lrv", "-Wl,-rpath,$ORIGIN"], verbose)
    os.replace(CLI + ".tmp", CLI)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
