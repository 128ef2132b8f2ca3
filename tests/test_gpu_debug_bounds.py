"""The debug build (libhs_debug.so, HS_DEBUG_BOUNDS): every tile record, work item,
suffix-stencil offset, neighbour index and tile position the kernels use passes its check
on every kernel family and set kind (tests/debug_bounds_run.py, run in a child process
with the debug library), and the checks change no result (the same workloads with the
release library in this process)."""
import json
import os
import subprocess
import sys

import pytest

from tests import debug_bounds_run

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEBUG_LIB = os.path.join(ROOT, "paper_1403_3511_amd", "libhs_debug.so")


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


def test_debug_build_checks_pass_and_change_nothing(hs):
    assert os.path.exists(DEBUG_LIB), "libhs_debug.so not built: run __graft_entry__.build()"
    print("debug-bounds child: every kernel family with libhs_debug.so", flush=True)
    env = dict(os.environ, HS_LIBRARY=DEBUG_LIB)
    res = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "debug_bounds_run.py")], cwd=ROOT,
                         env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, (res.stdout + res.stderr)[-4000:]
    child = json.loads(res.stdout.strip().splitlines()[-1])
    assert child["checks"] is True and child["lib"].endswith("libhs_debug.so")
    failed = {k: v["counts"] for k, v in child["cases"].items() if v["counts"][0] != 0}
    assert not failed, failed
    assert not hs.debug_checks()  # this process holds the release library
    rel = debug_bounds_run.run(hs)
    assert set(rel) == set(child["cases"])
    for k, v in rel.items():
        assert v["counts"] == [0, 0], k  # the release build records nothing
        d = child["cases"][k]["norm"]
        assert abs(d - v["norm"]) <= 1e-13 * max(1.0, abs(v["norm"])), (k, d, v["norm"])
