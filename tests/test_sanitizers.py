"""Host code under AddressSanitizer and UBSan (no GPU involved).

The oracle is rebuilt with -fsanitize=address,undefined and its pin tests
run against that build (LBM_ORACLE_LIBRARY, the sanitizer runtime preloaded
into the test process).  The library's host translation unit and the kernel
units are rebuilt with the sanitizers on the host side only (the device code
at -O0: it is compiled but never run here), linked with a small driver
(tests/sanitize/host_driver.cpp) that runs the host self-tests of the index
arithmetic and the tile builder and argument checks that return before any
device call.  Any sanitizer report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2204_10566_amd", "csrc")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _asan_runtime():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _clean(out: str):
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None or _asan_runtime() is None, reason="gcc with libasan needed")
def test_oracle_pins_under_sanitizers(tmp_path):
    lib = tmp_path / "liblbm_oracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", "-o", str(lib), os.path.join(ROOT, "oracle", "lbm_oracle.c"), "-lm"],
                   check=True)
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), LBM_ORACLE_LIBRARY=str(lib), **SAN_ENV)
    tests = [os.path.join(ROOT, "tests", t) for t in
             ("test_oracle_pins.py", "test_oracle_outlet_shift.py", "test_oracle_feq_order.py")]
    res = subprocess.run([sys.executable, "-m", "pytest", "-p", "no:cacheprovider", "-q", "-x", *tests],
                         capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    _clean(out)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc needed")
def test_library_host_code_under_sanitizers(tmp_path):
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "--offload-arch=gfx950",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_device", "-O0", "-Xarch_device", "-g0",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    from paper_2204_10566_amd.build import UNITS as units  # every translation unit of the library
    procs = [subprocess.Popen(["hipcc", *flags, *extra, "-c", os.path.join(CSRC, src), "-o", str(tmp_path / obj)],
                              stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
             for src, extra, obj in units]
    drv = tmp_path / "driver.o"
    procs.append(subprocess.Popen(["hipcc", *flags, "--offload-host-only", "-c",
                                   os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), "-o", str(drv)],
                                  stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out[-4000:]
    exe = tmp_path / "host_driver"
    subprocess.run(["hipcc", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o",
                    str(exe), str(drv), *[str(tmp_path / obj) for _, _, obj in units], "-lpthread"], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS=SAN_ENV["UBSAN_OPTIONS"]))
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "argument checks: ok" in out
    _clean(out)
