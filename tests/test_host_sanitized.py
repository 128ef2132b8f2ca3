"""The host C++ of the library (index-set construction, potential compilation, argument
checks, checkpoint files) under AddressSanitizer and UndefinedBehaviorSanitizer: a build with the host code
instrumented (device code unchanged) runs the host-only test files in a subprocess with
the ASan runtime preloaded; any report fails it.  No GPU is touched.  Set
HS_SANITIZED_LIB to reuse an existing sanitized build instead of compiling one (about
two minutes)."""
import glob
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_host_code_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no clang ASan runtime in this image")
    with tempfile.TemporaryDirectory(prefix="hs_san_") as tmp:
        lib = os.environ.get("HS_SANITIZED_LIB")
        if not lib:
            sys.path.insert(0, ROOT)
            from paper_1403_3511_amd.build import build
            lib = build(out=os.path.join(tmp, "libhs_san.so"), sanitize=True)
        syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
        assert "__asan_report" in syms and "__ubsan_handle" in syms, "library is not instrumented"
        env = dict(os.environ, LD_PRELOAD=rt, HS_LIBRARY=lib,
                   ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        # -s: no output capture in the child, so a sanitizer report written just before the
        # process aborts reaches this test's message
        res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-s", "-x", "-p", "no:cacheprovider",
                              "-m", "not gpu",
                              os.path.join(ROOT, "tests", "test_lib_host.py"),
                              os.path.join(ROOT, "tests", "test_binding_checks.py"),
                              os.path.join(ROOT, "tests", "test_checkpoint.py")],
                             cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
        out = res.stdout + res.stderr
        assert res.returncode == 0, out[-4000:]
        assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
