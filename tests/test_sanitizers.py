"""CPU runs of the oracle and of the library's host side under
AddressSanitizer and UndefinedBehaviorSanitizer (no GPU): the drivers in
tests/sanitize/ call every entry point on small boxes and on every refused
argument; the sanitizers abort on an invalid access, a leak or an undefined
operation.  The library is built with host-only sanitizers (its device code
is unchanged)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-o", exe, os.path.join(HERE, "oracle_driver.c"),
                    os.path.join(ROOT, "oracle", "nf_oracle.c"), "-lm"], check=True)
    assert "oracle driver ok" in _run(exe)


CLANG = "/opt/rocm/llvm/bin/clang"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not found")
def test_library_host_side_under_asan_and_ubsan(tmp_path):
    from paper_1810_02916_amd import build
    bdir = os.path.join(ROOT, "_build", "asan")
    lib = build.build(lib=os.path.join(bdir, "libnf_asan.so"), build_dir=bdir,
                      extra=build.HOST_SANITIZE)
    exe = str(tmp_path / "abi_driver")
    subprocess.run([CLANG, "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "abi_driver.c"),
                    "-L", bdir, "-lnf_asan", "-Wl,-rpath," + bdir, "-o", exe], check=True)
    assert os.path.exists(lib)
    assert "abi driver ok" in _run(exe)
