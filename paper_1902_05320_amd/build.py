"""Build libkbatch.so for gfx950 with hipcc (in-tree, next to this file).

Run as ``python -m paper_1902_05320_amd.build``.  The GPU code is built with
packed-FP32 instruction selection disabled (no floating point is used, the
flag only guards against those instructions being formed).
"""

from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(HERE, "libkbatch.so")
ARCH = "gfx950"

SOURCES = [os.path.join(CSRC, "kbatch.hip"), os.path.join(CSRC, "probes.hip"),
           os.path.join(CSRC, "keccak_p.hip"),
           os.path.join(CSRC, "server.cpp"), os.path.join(CSRC, "tune_cache.cpp")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC or install ROCm)")


def source_hash() -> str:
    """First 16 hex digits of the SHA-256 over the kernel source directory
    (file name, NUL, contents, in name order); built into the library, which
    reports it through keccak_version, so a measurement names the sources of
    the library that ran."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def compile_flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        f"-I{INCLUDE}", f"-I{CSRC}", f'-DKB_SOURCE_HASH="{source_hash()}"',
    ]


def build(verbose: bool = False, extra: list[str] | None = None, out: str = LIB_PATH) -> str:
    cmd = [hipcc()] + compile_flags() + (extra or []) + SOURCES + ["-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the GPU-only target feature; that warning is harmless
    msgs = [ln for ln in (proc.stderr or "").splitlines() if "packed-fp32-ops" not in ln]
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
