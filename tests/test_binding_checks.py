"""The Python binding checks every buffer before it reaches the C ABI, which carries no
lengths: dtype against the requested complex type, contiguity, element counts, the
workspace size for (dtype, m), devices and aliasing.  Every case here is refused on the
host before any launch, so these tests run without a GPU.  Also the host Gauss-Hermite
rule (Sec. 4.1 quadrature; nodes = eigenvalues of the Jacobi matrix of Sec. 4.2) against
numpy's hermgauss."""
import ctypes as C
import math

import numpy as np
import pytest
import torch


@pytest.fixture(scope="module")
def hs():
    from paper_1403_3511_amd import hs as _hs
    return _hs


@pytest.fixture(scope="module")
def ip(hs):
    from synth import henon_heiles_chain
    tt = henon_heiles_chain(2, 0.111)
    idx = hs.Index(2, 64, upload=False)
    pot = hs.Pot(2, [(t[0], t[1], t[2], t[3], t.degrees) for t in tt], subtract_harmonic=True, upload=False)
    # stand-ins for uploaded blocks: host tensors, so any device check compares cpu to cpu
    idx.dev = torch.zeros(16, dtype=torch.uint8)
    pot.dev = torch.zeros(16, dtype=torch.uint8)
    return idx, pot


def _vec(n, dt=torch.complex128):
    return torch.zeros(n, dtype=dt)


def test_apply_h_refuses_wrong_dtype(hs, ip):
    idx, pot = ip
    with pytest.raises(hs.HSError, match="dtype"):
        hs.apply_h(idx, pot, _vec(idx.size, torch.complex64), _vec(idx.size))
    with pytest.raises(hs.HSError, match="dtype"):
        hs.apply_h(idx, pot, _vec(idx.size), _vec(idx.size), dtype=hs.HS_C64)
    with pytest.raises(hs.HSError, match="dtype code"):
        hs.apply_h(idx, pot, _vec(idx.size), _vec(idx.size), dtype=7)


def test_apply_h_refuses_short_and_strided(hs, ip):
    idx, pot = ip
    with pytest.raises(hs.HSError, match="elements"):
        hs.apply_h(idx, pot, _vec(idx.size - 1), _vec(idx.size))
    with pytest.raises(hs.HSError, match="contiguous"):
        hs.apply_h(idx, pot, _vec(2 * idx.size)[::2], _vec(idx.size))


def test_apply_h_refuses_aliasing(hs, ip):
    idx, pot = ip
    c = _vec(2 * idx.size)
    with pytest.raises(hs.HSError, match="overlap"):
        hs.apply_h(idx, pot, c[:idx.size], c[idx.size // 2:idx.size // 2 + idx.size])


def test_step_refuses_small_workspace(hs, ip):
    idx, pot = ip
    nb = C.c_int64()
    hs.hs_workspace_bytes(idx.h, pot.h, hs.HS_C128, 10, C.byref(nb))
    small = torch.zeros(nb.value - 1, dtype=torch.uint8)
    with pytest.raises(hs.HSError, match="workspace"):
        hs.step(idx, pot, _vec(idx.size), 0.0, 0.01, 10, ws=small)
    # a workspace for m = 0 is too small for a step with m = 10
    hs.hs_workspace_bytes(idx.h, pot.h, hs.HS_C128, 0, C.byref(nb))
    with pytest.raises(hs.HSError, match="workspace"):
        hs.step(idx, pot, _vec(idx.size), 0.0, 0.01, 10, ws=torch.zeros(nb.value, dtype=torch.uint8))
    # the FP32 form needs its own size
    hs.hs_workspace_bytes(idx.h, pot.h, hs.HS_C64, 10, C.byref(nb))
    with pytest.raises(hs.HSError, match="workspace"):
        hs.propagate(idx, pot, _vec(idx.size), 0.0, 0.01, 10, 1, dtype=hs.HS_C128,
                     ws=torch.zeros(nb.value // 2, dtype=torch.uint8))
    # a workspace of exactly the size for the FP32 form passes the checks
    hs._check_step_args("step", idx, pot, hs.HS_C64, 10, _vec(idx.size), torch.zeros(nb.value, dtype=torch.uint8))
    hs.hs_workspace_bytes(idx.h, pot.h, hs.HS_C128, 10, C.byref(nb))
    hs._check_step_args("step", idx, pot, hs.HS_C128, 10, _vec(idx.size), torch.zeros(nb.value, dtype=torch.uint8))
    # the step's state is complex128 in both forms
    with pytest.raises(hs.HSError, match="dtype"):
        hs.step(idx, pot, _vec(idx.size, torch.complex64), 0.0, 0.01, 10, dtype=hs.HS_C64)


def test_unuploaded_blocks_are_refused(hs):
    from synth import henon_heiles_chain
    tt = henon_heiles_chain(2, 0.111)
    idx = hs.Index(2, 64, upload=False)
    pot = hs.Pot(2, [(t[0], t[1], t[2], t[3], t.degrees) for t in tt], subtract_harmonic=True, upload=False)
    with pytest.raises(hs.HSError, match="device block"):
        hs.apply_h(idx, pot, _vec(idx.size), _vec(idx.size))
    with pytest.raises(hs.HSError, match="device block"):
        hs.apply_x(idx, 0, _vec(idx.size), _vec(idx.size))


def test_apply_x_refuses_mismatch(hs, ip):
    idx, pot = ip
    with pytest.raises(hs.HSError, match="elements"):
        hs.apply_x(idx, 0, _vec(idx.size), _vec(3))
    with pytest.raises(hs.HSError, match="dtype"):
        hs.apply_x(idx, 0, _vec(idx.size), _vec(idx.size), dtype=hs.HS_C64)


def test_gh_rule_matches_hermgauss(hs):
    for Q in range(1, 33):
        x = np.empty(Q)
        w = np.empty(Q)
        hs.hs_gh_rule(Q, x.ctypes.data_as(hs._pf64), w.ctypes.data_as(hs._pf64))
        xr, wr = np.polynomial.hermite.hermgauss(Q)
        assert np.max(np.abs(x - xr)) <= 4e-15 * max(1.0, np.max(np.abs(xr))), Q
        assert np.max(np.abs(w / wr - 1.0)) <= 1e-13, Q
        # the rule integrates exp(-x^2) x^(2k) exactly up to degree 2Q - 1
        for k in range(Q):
            exact = math.gamma(k + 0.5)
            assert abs(np.sum(w * x ** (2 * k)) - exact) <= 1e-12 * exact, (Q, k)


def test_gh_rule_refuses_bad_sizes(hs):
    x = np.empty(40)
    with pytest.raises(hs.HSError):
        hs.hs_gh_rule(0, x.ctypes.data_as(hs._pf64), x.ctypes.data_as(hs._pf64))
    with pytest.raises(hs.HSError):
        hs.hs_gh_rule(33, x.ctypes.data_as(hs._pf64), x.ctypes.data_as(hs._pf64))
