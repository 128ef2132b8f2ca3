"""Build the HIP library libhs.so for gfx950 in-tree (hipcc, no JIT cache).

Each source is compiled to an object in parallel, then linked.  Every call rebuilds.
Usage: python -m paper_1403_3511_amd.build  (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhs.so")
# the same library with the kernels' neighbour-index checks compiled in (HS_DEBUG_BOUNDS)
OUT_DEBUG = os.path.join(HERE, "libhs_debug.so")
SOURCES = ["api.cpp", "index.cpp", "potential.cpp", "matvec.hip", "matvec_long_f64.hip",
           "matvec_long_f32.hip", "matvec_multi_f64.hip", "matvec_multi_f32.hip", "matvec_m4_f64.hip", "matvec_m4_f32.hip", "matvec_sym_f64.hip",
           "matvec_sym_f32.hip", "lanczos.hip", "step_small_f64.hip", "step_small_f32.hip",
           "batch.hip", "surrogate.hip", "diag.hip", "step_static.hip", "checkpoint.cpp"]
CFLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fno-gpu-rdc", "-Wall", "-Wno-unused-function"]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


# host-side AddressSanitizer and UndefinedBehaviorSanitizer (device code is built as usual)
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-g"]


def _compile(src: str, obj: str, defines=(), extra=()) -> tuple[str, int, str]:
    cmd = [_hipcc(), *CFLAGS, *extra, *["-D" + d for d in defines], "-I", os.path.join(HERE, "..", "include"),
           "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(line for line in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in line and "not a recognized feature" not in line)
    return src, res.returncode, msg


def build_debug(verbose: bool = False) -> str:
    """Compile libhs_debug.so: libhs.so with the neighbour-index checks of HS_DEBUG_BOUNDS."""
    return build(verbose=verbose, out=OUT_DEBUG, defines=("HS_DEBUG_BOUNDS",))


def build(verbose: bool = False, out: str | None = None, defines=(), sanitize: bool = False) -> str:
    """Compile and link libhs.so (into out, default the package directory).  sanitize=True
    instruments the host code with ASan and UBSan; such a library must be loaded with the
    ASan runtime preloaded (see tests/test_host_sanitized.py)."""
    extra = SANITIZE_FLAGS if sanitize else []
    with tempfile.TemporaryDirectory(prefix="hs_build_") as tmp:
        jobs = [(os.path.join(CSRC, s), os.path.join(tmp, s + ".o")) for s in SOURCES]
        workers = min(len(jobs), max(1, (os.cpu_count() or 4)))
        with ThreadPoolExecutor(max_workers=workers) as ex:
            results = list(ex.map(lambda j: _compile(*j, defines, extra), jobs))
        bad = [(s, m) for s, rc, m in results if rc != 0]
        for s, rc, m in results:
            if verbose and m.strip():
                print(m)
        if bad:
            for s, m in bad:
                sys.stderr.write(f"--- {s}\n{m}\n")
            raise RuntimeError("hipcc failed building libhs.so")
        tmp_out = os.path.join(tmp, "libhs.so")
        cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_out,
               *(["-fsanitize=address,undefined", "-shared-libasan"] if sanitize else []),
               *[o for _, o in jobs]]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("link of libhs.so failed")
        _copy(tmp_out, out or OUT)
    return out or OUT


def _copy(src, dst):
    import shutil
    tmpdst = dst + ".tmp"
    shutil.copyfile(src, tmpdst)
    os.chmod(tmpdst, 0o755)
    os.replace(tmpdst, dst)


if __name__ == "__main__":
    print(build(verbose=True))
    if "--debug" in sys.argv:
        print(build_debug(verbose=True))
