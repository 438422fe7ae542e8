"""Host sanitizer runs (CPU only): the FP64 reference and the host side of the
C ABI built with AddressSanitizer (leaks included) and
UndefinedBehaviorSanitizer, then driven through their entry points
(tests/sanitize/*.c*).  Any out-of-bounds access, leak or undefined operation
makes the driver exit with a report and the test fail."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1807_01769_amd", "csrc")
SAN = "-fsanitize=address,undefined"


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    return env


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", SAN, "-fno-sanitize-recover=all",
          "-fopenmp", "-std=gnu11", os.path.join(HERE, "oracle_check.c"),
          os.path.join(ROOT, "oracle", "fs_oracle.c"), "-lm", "-o", exe])
    r = _run([exe], env=_env(), timeout=600)
    assert "oracle sanitizer run: ok" in r.stdout
    assert "runtime error" not in r.stderr, r.stderr


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_abi_validation_under_asan_ubsan(tmp_path):
    # host-only compilation: the sanitizers instrument the host code, every
    # -fsanitize flag is scoped to the host side
    common = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "--offload-arch=gfx950",
              "--offload-host-only", "-Xarch_host", SAN, "-Xarch_host",
              "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
              "-x", "hip", "-c"]
    api = str(tmp_path / "fs_api.o")
    drv = str(tmp_path / "abi_check.o")
    exe = str(tmp_path / "abi_check")
    _run(["hipcc", *common, os.path.join(CSRC, "fs_api.cpp"), "-o", api])
    _run(["hipcc", *common, os.path.join(HERE, "abi_check.cpp"), "-o", drv])
    _run(["hipcc", "--hip-link", "-Xarch_host", SAN, drv, api, "-o", exe])
    r = _run([exe], env=_env(), timeout=600)
    assert "abi sanitizer run: ok" in r.stdout, r.stdout
    assert "runtime error" not in r.stderr, r.stderr
