"""Builds libtrinv.so (HIP, gfx950) in-tree from csrc/.

Every source is compiled with hipcc for gfx950 only. Packed-FP32 instructions
are disabled for device code (some of their forms have produced wrong results
on this hardware); hipcc's host pass prints a harmless warning about that
feature name, which is filtered from the output.
"""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
CSRC = os.path.join(_HERE, "csrc")
BUILD = os.path.join(_HERE, "_build")
LIB = os.path.join(_HERE, "libtrinv.so")
ARCH = "gfx950"


def _hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def _flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(_ROOT, "include"), "-I", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False, jobs: int = 8, incremental: bool = False) -> str:
    """Compile every source and link libtrinv.so. ``incremental``: skip a
    source whose object is newer than it and than every header."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    headers = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(_ROOT, "include", "*.h"))
    newest_header = max((os.path.getmtime(h) for h in headers), default=0.0)
    cc = _hipcc()

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        if incremental and os.path.exists(obj):
            t = os.path.getmtime(obj)
            if t > os.path.getmtime(src) and t > newest_header:
                return obj
        cmd = [cc] + _flags() + ["-c", src, "-o", obj]
        out = _run(cmd)
        if verbose and out.strip():
            print(out, flush=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
