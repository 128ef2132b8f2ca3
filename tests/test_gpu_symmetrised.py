"""The symmetrised operator D + (F + F_rev)/2 on the GPU against the oracle: every kind of
axis pair the fused kernel distinguishes (prefix-prefix, prefix-suffix, suffix-suffix),
with and without x_l^2 terms, the Lanczos step and the fourth-order operator in this
form, the FP32 form, and at the benchmark's size the symmetry <u, S v> = <S u, v>."""
import math

import numpy as np
import pytest

from oracle.index import IndexSet
from oracle.operators import Potential, fast_apply_H, sym_apply_H
from oracle.propagate import magnus4_operator, propagate
from synth import coherent_state, complex_normal_by_index
from tests.hsutil import hh_workload, lib_terms, lib_to_lex, oracle_W, rel2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


def _to_lib(idx, N, B, c_lex):
    import torch
    lexpos = lib_to_lex(idx, N, B)
    return torch.from_numpy(np.ascontiguousarray(c_lex[lexpos])).to("cuda"), lexpos


def _from_lib(t, lexpos):
    out = np.empty(t.shape[0], dtype=np.complex128)
    out[lexpos] = t.cpu().numpy().astype(np.complex128)
    return out


def _pot(N, harmonic=True, lam=0.111):
    tt = hh_workload(N, lam, 0.05)
    W = (lambda t: oracle_W(N, tt, t)) if harmonic else \
        (lambda t: Potential(N, "mono", 1.0, [(x.coef(t), x.degrees) for x in tt]))
    return tt, W


@pytest.mark.parametrize("N,B,tile,harmonic", [
    (2, 700, 0, True), (3, 300, 0, True), (3, 300, 1, True), (4, 150, 0, False),
    (4, 150, 1, True), (4, 150, 3, True), (4, 150, 4, False), (5, 64, 0, True), (6, 300, 0, True)])
def test_apply_symmetrised(hs, N, B, tile, harmonic):
    import torch
    tt, W_at = _pot(N, harmonic, lam=0.2)
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 40 + N)
    W = W_at(0.3)
    y_ref = sym_apply_H(ix, W, c)
    idx = hs.Index(N, B, tile)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=harmonic)
    assert pot.fused
    pot.set_form(hs.HS_FORM_SYM)
    pot.set_time(0.3)
    cl, lexpos = _to_lib(idx, N, B, c)
    yl = torch.empty_like(cl)
    hs.apply_h(idx, pot, cl, yl)
    torch.cuda.synchronize()
    y = _from_lib(yl, lexpos)
    assert rel2(y, y_ref) <= 1e-12
    # the two forms really differ on this set
    assert rel2(fast_apply_H(ix, W, c), y_ref) > 1e4 * 1e-12
    # float32 form of the same operator
    yl32 = torch.empty(cl.shape[0], dtype=torch.complex64, device="cuda")
    hs.apply_h(idx, pot, cl.to(torch.complex64), yl32, hs.HS_C64)
    torch.cuda.synchronize()
    assert rel2(_from_lib(yl32, lexpos), y_ref) <= 1e-5


@pytest.mark.parametrize("reorth", [True, False])
def test_steps_symmetrised(hs, reorth):
    import torch
    N, B, m, h, n = 3, 300, 8, 0.02, 5
    tt, W_at = _pot(N, True, lam=0.2)
    ix = IndexSet(N, B)
    c0 = coherent_state(ix.k, [0.8, -0.4, 0.3])
    c0 /= np.linalg.norm(c0)
    ref, meffs = propagate(ix, W_at, lambda W: (lambda v: sym_apply_H(ix, W, v)), c0, 0.0, h, n, m,
                           reorth=reorth)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    pot.set_form(hs.HS_FORM_SYM)
    c, lexpos = _to_lib(idx, N, B, c0)
    t = 0.0
    for _ in range(n):
        hs.step(idx, pot, c, t, h, m, reorth=reorth)
        t += h
    torch.cuda.synchronize()
    assert rel2(_from_lib(c, lexpos), ref) <= 1e-11


def test_magnus4_operator_symmetrised(hs):
    """The fourth-order operator in the symmetrised form (four H applications)."""
    import torch
    N, B, t, h = 3, 300, 0.4, 0.5
    tt, W_at = _pot(N, True, lam=0.2)
    c1, c2 = 0.5 - math.sqrt(3.0) / 6.0, 0.5 + math.sqrt(3.0) / 6.0
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 77)
    W1, W2 = W_at(t + c1 * h), W_at(t + c2 * h)
    y_ref = magnus4_operator(lambda v: sym_apply_H(ix, W1, v), lambda v: sym_apply_H(ix, W2, v), h)(c)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    pot.set_form(hs.HS_FORM_SYM)
    d1, d2 = pot.blocks2()
    hs.hs_pot_set_time(pot.h, hs.ptr(d1), t + c1 * h, None, hs.stream_ptr())
    hs.hs_pot_set_time(pot.h, hs.ptr(d2), t + c2 * h, None, hs.stream_ptr())
    cl, lexpos = _to_lib(idx, N, B, c)
    yl = torch.empty_like(cl)
    hs.apply_magnus4(idx, pot, h, cl, yl)
    torch.cuda.synchronize()
    assert rel2(_from_lib(yl, lexpos), y_ref) <= 1e-12


def test_symmetry_at_bench_size(hs):
    """N = 6, product bound 4096: <u, S v> = <S u, v> for random u, v (a property of the
    symmetric operator at any size); the paper's form misses it by far more."""
    import torch
    N, B = 6, 4096
    tt = hh_workload(N, 0.111, 0.05)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    pot.set_time(0.3)
    g = torch.Generator(device="cuda").manual_seed(5)
    u = torch.randn(idx.size, dtype=torch.complex128, device="cuda", generator=g)
    v = torch.randn(idx.size, dtype=torch.complex128, device="cuda", generator=g)
    out = {}
    for form in (hs.HS_FORM_PAPER, hs.HS_FORM_SYM):
        pot.set_form(form)
        su, sv = torch.empty_like(u), torch.empty_like(v)
        hs.apply_h(idx, pot, u, su)
        hs.apply_h(idx, pot, v, sv)
        torch.cuda.synchronize()
        lhs = torch.vdot(u, sv).item()
        rhs = torch.vdot(su, v).item()
        out[form] = abs(lhs - rhs) / abs(lhs)
    assert out[hs.HS_FORM_SYM] <= 1e-13
    assert out[hs.HS_FORM_PAPER] > 1e3 * max(out[hs.HS_FORM_SYM], 1e-16)


def test_one_axis_and_no_coupling_equal_the_paper_form(hs):
    """N = 1, and a potential without coupling terms: both forms are the same operator, and
    the kernels return the same values to rounding (the paper's form may take the
    multi-tile row code, the symmetrised form its own)."""
    import torch
    for N, terms in [(1, [(0.05, (3,)), (0.1, (1,)), (0.2, (2,))]),
                     (3, [(0.05, (3, 0, 0)), (-0.02, (0, 0, 3)), (0.1, (0, 1, 0))])]:
        idx = hs.Index(N, 200)
        pot = hs.Pot(N, terms)
        assert pot.fused
        g = torch.Generator(device="cuda").manual_seed(1)
        x = torch.randn(idx.size, dtype=torch.complex128, device="cuda", generator=g)
        ya, yb = torch.empty_like(x), torch.empty_like(x)
        hs.apply_h(idx, pot, x, ya)
        pot.set_form(hs.HS_FORM_SYM)
        hs.apply_h(idx, pot, x, yb)
        torch.cuda.synchronize()
        assert float(torch.linalg.norm(ya - yb) / torch.linalg.norm(ya)) <= 1e-14
