"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the CPU-side code,
run on the CPU:

- the oracle (both C files), driven through every entry point on small
  grids and invalid arguments (tests/sanitize/oracle_driver.c);
- the HIP library's host code -- planning (make_plan, plan_segments, the
  workspace and LDS figures), the argument validation of every entry point
  and the batched plan's problem checks -- over some 2.5e7 combinations of
  valid, extreme and invalid arguments (tests/sanitize/host_driver.cpp).
  Only the host half of the library is instrumented (each sanitizer flag is
  scoped to the host compilation); the device code is built as usual but
  never launched.

The binaries are cached under _build/sanitize/, keyed by a hash of their
sources and flags, so the host build (about a minute) runs once per change.
"""
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
SAN = os.path.join(ROOT, "tests", "sanitize")
ORACLE = [os.path.join(ROOT, "oracle", "fmgsr_oracle.c"),
          os.path.join(ROOT, "oracle", "fmgsr_oracle_reaction.c")]
CSRC = os.path.join(ROOT, "paper_1207_6720_amd", "csrc")
HIP_SOURCES = [os.path.join(CSRC, "fmgsr.hip"), os.path.join(CSRC, "fmgsr_batched.hip")]
HIP_HEADERS = [os.path.join(CSRC, h) for h in ("fmgsr_kernels.hpp", "fmgsr_device.hpp",
                                               "fmgsr_host.hpp")] + \
              [os.path.join(ROOT, "include", "fmgsr.h")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ORACLE_FLAGS = ["-std=c11", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
                "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
# every sanitizer flag scoped to the host half of the HIP compilation
HOST_FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize-recover=all",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _cached(name, sources, flags):
    h = hashlib.sha256(" ".join(flags).encode())
    for p in sources:
        with open(p, "rb") as fh:
            h.update(fh.read())
    os.makedirs(OUT, exist_ok=True)
    return os.path.join(OUT, f"{name}-{h.hexdigest()[:16]}")


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, f"{exe} failed ({r.returncode}):\n{r.stdout}\n{r.stderr[-4000:]}"
    return r.stdout


def test_oracle_under_asan_ubsan():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    drv = os.path.join(SAN, "oracle_driver.c")
    exe = _cached("oracle", [drv, *ORACLE], ORACLE_FLAGS)
    if not os.path.exists(exe):
        subprocess.run(["gcc", *ORACLE_FLAGS, "-o", exe + ".tmp", drv, *ORACLE, "-lm"], check=True)
        os.replace(exe + ".tmp", exe)
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1",
                     "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    assert "all calls clean" in out


def test_library_host_code_under_asan_ubsan():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    drv = os.path.join(SAN, "host_driver.cpp")
    exe = _cached("host", [drv, *HIP_SOURCES, *HIP_HEADERS], HOST_FLAGS)
    if not os.path.exists(exe):
        subprocess.run([HIPCC, *HOST_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                        "-o", exe + ".tmp", drv, *HIP_SOURCES], check=True,
                       capture_output=True)
        os.replace(exe + ".tmp", exe)
    # the HIP runtime's own allocations are not the subject here
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
                     "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    assert "calls clean" in out
