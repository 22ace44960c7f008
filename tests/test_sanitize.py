"""Host sanitizer build (CPU only): the oracle (gcc) and the host-side C++
sources of the library (hipcc, host pass only) are compiled with
AddressSanitizer and UndefinedBehaviorSanitizer, linked with the library's
ordinary device objects into tests/sanitize_driver.c, and run. The driver
exercises the oracle on small, ragged and degenerate inputs and the C ABI's
argument checks and workspace queries (every call returns before any device
work, so no GPU is needed). Any sanitizer report fails the test.

Leak detection is off: the HIP runtime keeps process-lifetime allocations.
"""

from __future__ import annotations

import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2307_07611_amd", "csrc")
OBJ = os.path.join(ROOT, "paper_2307_07611_amd", "_build")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def _host_san_flags():
    # hipcc: each sanitizer flag applies to the host pass only
    out = []
    for f in SAN:
        out += ["-Xarch_host", f]
    return out


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not shutil.which("gcc"):
        pytest.skip("hipcc or gcc missing")
    dev_objs = sorted(glob.glob(os.path.join(OBJ, "*.hip.o")))
    if not dev_objs:
        pytest.skip("library objects not built (paper_2307_07611_amd/build.py)")
    d = tmp_path_factory.mktemp("san")
    objs = []
    # oracle: plain C, gcc
    o = str(d / "oracle.o")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer"] + SAN +
         ["-c", os.path.join(ROOT, "oracle", "oracle.c"), "-o", o])
    objs.append(o)
    # host-side library sources: hipcc, sanitizers on the host pass
    procs = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))):
        o = str(d / (os.path.basename(src) + ".o"))
        cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer"] + \
            _host_san_flags() + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o", o]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        objs.append(o)
    for cmd, p in procs:
        out, err = p.communicate()
        assert p.returncode == 0, f"{' '.join(cmd)}\n{err[-3000:]}"
    o = str(d / "driver.o")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer"] + SAN +
         ["-I", os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "sanitize_driver.c"), "-o", o])
    objs.append(o)
    exe = str(d / "sanitize_driver")
    _run([hipcc, "--offload-arch=gfx950", "-fopenmp"] + _host_san_flags() + ["-o", exe] + objs + dev_objs + ["-lm"])
    return exe


def test_oracle_and_abi_under_sanitizers(driver):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    report = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, report
    assert "all checks passed" in r.stdout
