"""CPU builds with AddressSanitizer and UndefinedBehaviorSanitizer (every
report fatal) of the two pieces of host code that run without a device:

* the FP64 oracle (oracle/flood_oracle.c), driven by the whole oracle test
  suite in a child process that preloads gcc's libasan and loads the
  sanitized build through FLOOD_ORACLE_LIB;
* the library's host-side argument validation (flood_abi.cpp and
  flood_validate.cpp, built with g++ and no device code), driven by
  tests/host_sanitize.cpp, which checks every refusal of the C ABI.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2302_08341_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _libasan():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip("gcc has no libasan here")
    return p


def test_oracle_suite_under_asan_ubsan(tmp_path):
    asan = _libasan()
    import oracle
    lib = oracle.build_sanitized(str(tmp_path / "liborc_san.so"))
    tests = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    assert len(tests) >= 8
    env = dict(os.environ, FLOOD_ORACLE_LIB=lib, LD_PRELOAD=asan, **ENV)
    probe = subprocess.run([sys.executable, "-c", "import oracle; print(oracle._LIB)"], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0 and probe.stdout.strip() == lib, probe.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + tests,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert " passed" in out


def test_host_validation_under_asan_ubsan(tmp_path):
    _libasan()
    exe = str(tmp_path / "host_sanitize")
    cmd = (["g++", "-std=c++17", "-Wall"] + SAN + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "host_sanitize.cpp"), os.path.join(CSRC, "flood_abi.cpp"),
           os.path.join(CSRC, "flood_validate.cpp"), "-o", exe])
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if b.returncode != 0 and "hip_runtime.h" in b.stderr:
        pytest.skip("no HIP headers here")
    assert b.returncode == 0, b.stderr[-4000:]
    r = subprocess.run([exe], env=dict(os.environ, **ENV), capture_output=True, text=True, timeout=120)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "0 failed" in out and "runtime error" not in out, out
