"""Builds libpatnufft.so in-tree with hipcc for gfx950.

Usage: ``python -m paper_0808_3510_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpatnufft.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["plan.cpp", "capi.cpp", "kernels.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


SAN_LIB = os.path.join(ROOT, "_build", "libpatnufft_hostsan.so")


def build_host_sanitized(verbose: bool = False) -> str:
    """The library with its host side (plan, C ABI, launchers) built with
    AddressSanitizer and UndefinedBehaviorSanitizer, for the CPU checks of the
    host logic.  Load it with the ASan runtime preloaded (``asan_runtime()``).
    Not for the GPU: its device code is built at -O1."""
    os.makedirs(os.path.dirname(SAN_LIB), exist_ok=True)
    # (device code at -O1 for a quick build; the sanitizers apply to the host
    # side only, each -fsanitize= behind -Xarch_host)
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xarch_host", "-shared-libsan", "-I" + os.path.join(ROOT, "include"),
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", SAN_LIB]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building the sanitized host library")
    if verbose:
        sys.stderr.write(res.stderr)
    return SAN_LIB


def asan_runtime() -> str:
    """Path of the compiler's shared ASan runtime (to preload)."""
    res = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("ASan runtime not found")
    return path


def build(verbose: bool = False) -> str:
    cmd = [HIPCC, *FLAGS, "-I" + os.path.join(ROOT, "include"),
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", LIB + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libpatnufft.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
