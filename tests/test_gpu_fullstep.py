"""The main workload's step at full size: N = 6, product bound 4096 (4,883,360 rows),
chained Henon-Heiles lambda = 0.111 plus the laser term 0.05 sin(2t) on every axis,
coherent packet at x_d = 2, m = 10, h = 0.005 (the step bench.py times).  The first step
against the oracle's exponential-midpoint Lanczos step on the whole set (Sec. 2.1 eq.
expMPR, Sec. 2.2; about 10 oracle H applications, tens of seconds on the host); 100 steps
against the properties that hold at any size: the norm, and agreement of the tilings
(the same operator through other prefix/suffix splits)."""
import numpy as np
import pytest

from oracle.index import IndexSet
from oracle.operators import fast_apply_H
from oracle.propagate import lanczos_expm
from synth import coherent_state
from tests.hsutil import hh_workload, lib_terms, lib_to_lex, oracle_W, rel2

pytestmark = pytest.mark.gpu

N, B, M, H = 6, 4096, 10, 0.005


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


def _start(idx):
    c = coherent_state(idx.multi_indices(), 2.0)
    return c / np.linalg.norm(c)


def test_first_step_against_the_oracle(hs):
    import torch
    tt = hh_workload(N, 0.111, 0.05)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    c_lib = _start(idx)
    c = torch.from_numpy(c_lib.copy()).to("cuda")
    diag = torch.zeros(1 + 2 * M, dtype=torch.float64, device="cuda")
    hs.step(idx, pot, c, 0.0, H, M, ws=hs.workspace(idx, pot, 0, M), diag=diag)
    got_lib = c.cpu().numpy()
    print("gpu step done; oracle step on", idx.size, "rows", flush=True)
    ix = IndexSet(N, B)
    lexpos = lib_to_lex(idx, N, B)
    c_lex = np.empty_like(c_lib)
    c_lex[lexpos] = c_lib
    W = oracle_W(N, tt, 0.5 * H)
    ref, meff, alpha, beta = lanczos_expm(lambda v: fast_apply_H(ix, W, v), c_lex, H, M)
    got = np.empty_like(got_lib)
    got[lexpos] = got_lib
    d = diag.cpu().numpy()
    assert int(d[0]) == meff == M
    np.testing.assert_allclose(d[1:1 + M], alpha, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(d[1 + M:M + meff], beta, rtol=1e-12)
    assert rel2(got, ref) <= 1e-12


def test_hundred_steps_norm_and_tilings(hs):
    """100 steps from the packet: the norm stays 1 to 1e-12; the library's tiling (tile
    dimension 3) and tile dimensions 2 and 4 (other kernels' row orders, other
    prefix/suffix splits, other reductions) agree to 1e-12 after 10 steps."""
    import torch
    tt = hh_workload(N, 0.111, 0.05)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    out = {}
    for d, nsteps in ((3, 100), (2, 10), (4, 10)):
        idx = hs.Index(N, B, d)
        c = torch.from_numpy(_start(idx)).to("cuda")
        ws = hs.workspace(idx, pot, 0, M)
        t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        for i in range(nsteps):
            hs.step(idx, pot, c, 0.0, H, M, ws=ws, t_dev=t_dev)
            if d == 3 and i == 9:
                lexpos = lib_to_lex(idx, N, B)
                x = np.empty(idx.size, dtype=np.complex128)
                x[lexpos] = c.cpu().numpy()
                out[3] = x
        torch.cuda.synchronize()
        print("tile dim", d, "steps", nsteps, flush=True)
        if d == 3:
            assert abs(float(torch.linalg.norm(c)) - 1.0) <= 1e-12
        else:
            lexpos = lib_to_lex(idx, N, B)
            x = np.empty(idx.size, dtype=np.complex128)
            x[lexpos] = c.cpu().numpy()
            out[d] = x
    assert rel2(out[2], out[3]) <= 1e-12
    assert rel2(out[4], out[3]) <= 1e-12
