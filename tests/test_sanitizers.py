"""Host AddressSanitizer and UndefinedBehaviorSanitizer runs (CPU only):
the oracle built with both sanitizers runs every entry point on small
inputs including its boundary branches, and the library's host code built
with them runs the ABI's host logic (sizes, option and argument checks).
Device code is built as usual: the sanitizers cover host code only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return r.returncode, r.stdout + r.stderr


def _clean(out):
    return "ERROR: AddressSanitizer" not in out and "runtime error" not in out and \
        "ERROR: LeakSanitizer" not in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    rc, out = _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                    os.path.join(ROOT, "oracle", "mhar_ref.c"), "-lm", "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe], env=SAN_ENV)
    assert rc == 0 and _clean(out), out
    assert "0 failed expectations" in out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_abi_host_logic_under_asan_ubsan(tmp_path):
    from paper_2104_07097_amd import build as B
    lib = str(tmp_path / "libmhar_san.so")
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-O3",)]
    rc, out = _run(["hipcc", *flags, "-O1", "-g", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "include"), "-o", lib, *B.SOURCES])
    assert rc == 0, out[-4000:]
    clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
    exe = str(tmp_path / "abi_driver")
    rc, out = _run([clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(ROOT, "tests", "sanitize", "abi_driver.c"), lib,
                    "-Wl,-rpath," + str(tmp_path), "-o", exe])
    assert rc == 0, out[-4000:]
    # the HIP runtime's own allocations at exit are not the library's
    env = dict(SAN_ENV, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    rc, out = _run([exe], env=env)
    assert rc == 0 and _clean(out), out[-4000:]
    assert "0 failed expectations" in out
