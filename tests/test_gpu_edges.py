"""Edge cases of the GPU path against the oracle: degenerate index sets, the extreme
Krylov dimensions, a dimension with no specialised kernel, the largest bound, a step with
a potential outside the fused class, and the zero vector."""
import numpy as np
import pytest

from oracle.index import IndexSet
from oracle.operators import Potential, fast_apply_H
from oracle.propagate import lanczos_expm
from synth import coherent_state, complex_normal_by_index
from tests.hsutil import hh_workload, lib_terms, lib_to_lex, oracle_W, rel2

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


def to_lib(idx, N, B, c_lex):
    import torch
    lexpos = lib_to_lex(idx, N, B)
    return torch.from_numpy(np.ascontiguousarray(c_lex[lexpos])).to("cuda"), lexpos


def from_lib(t, lexpos):
    out = np.empty(t.shape[0], dtype=np.complex128)
    out[lexpos] = t.cpu().numpy()
    return out


def apply_case(hs, N, B, terms_lib, W, c_lex, t=0.0, basis="mono", harmonic=True):
    import torch
    idx = hs.Index(N, B)
    pot = hs.Pot(N, terms_lib, basis=basis, subtract_harmonic=harmonic)
    pot.set_time(t)
    c, lexpos = to_lib(idx, N, B, c_lex)
    y = torch.empty_like(c)
    hs.apply_h(idx, pot, c, y)
    torch.cuda.synchronize()
    return from_lib(y, lexpos), pot


def steps_case(hs, N, B, terms_lib, Wfun, c_lex, h, m, n, basis="mono", harmonic=True, reorth=True):
    import torch
    idx = hs.Index(N, B)
    pot = hs.Pot(N, terms_lib, basis=basis, subtract_harmonic=harmonic)
    c, lexpos = to_lib(idx, N, B, c_lex)
    ws = hs.workspace(idx, pot, hs.HS_C128, m)
    diag = torch.zeros(1 + 2 * m, dtype=torch.float64, device="cuda")
    t = 0.0
    for _ in range(n):
        hs.step(idx, pot, c, t, h, m, reorth=reorth, ws=ws, diag=diag)
        t += h
    torch.cuda.synchronize()
    got = from_lib(c, lexpos)
    ix = IndexSet(N, B)
    ref = c_lex.copy()
    t = 0.0
    for _ in range(n):
        W = Wfun(t + 0.5 * h)
        ref, meff, _, _ = lanczos_expm(lambda v: fast_apply_H(ix, W, v), ref, h, m, reorth)
        t += h
    return got, ref, int(diag[0].item())


@pytest.mark.parametrize("N,B", [(3, 1), (4, 2), (5, 3)])
def test_tiny_sets(hs, N, B):
    """B = 1 is the single row k = 0; B = 2 adds the N unit vectors."""
    tt = hh_workload(N, 0.111, 0.05)
    ix = IndexSet(N, B)
    assert ix.size == {1: 1, 2: N + 1}.get(B, ix.size)
    c = complex_normal_by_index(ix.k, 3)
    y_ref = fast_apply_H(ix, oracle_W(N, tt, 0.2), c)
    y, _ = apply_case(hs, N, B, lib_terms(tt), None, c, t=0.2)
    assert rel2(y, y_ref) <= TOL64
    got, ref, meff = steps_case(hs, N, B, lib_terms(tt), lambda t: oracle_W(N, tt, t), c, 0.01, 4, 3)
    assert rel2(got, ref) <= 1e-11


@pytest.mark.parametrize("m", [1, 2, 32])
def test_krylov_dimension_extremes(hs, m):
    N, B = 2, 300
    tt = hh_workload(N, 0.111, 0.05)
    ix = IndexSet(N, B)
    c = coherent_state(ix.k, [1.0, -0.5])
    c /= np.linalg.norm(c)
    got, ref, meff = steps_case(hs, N, B, lib_terms(tt), lambda t: oracle_W(N, tt, t), c, 0.01, m, 5)
    assert meff == m
    assert rel2(got, ref) <= 1e-11


def test_dimension_without_specialised_kernel(hs):
    """N = 12 runs on the generic fused row kernels (no compile-time specialisation)."""
    N, B = 12, 48
    tt = hh_workload(N, 0.111, 0.05)
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 5)
    y_ref = fast_apply_H(ix, oracle_W(N, tt, 0.7), c)
    y, pot = apply_case(hs, N, B, lib_terms(tt), None, c, t=0.7)
    assert pot.fused
    assert rel2(y, y_ref) <= TOL64


def test_largest_bound(hs):
    """B = 65536, N = 1: one fibre of 65536 rows (the weight table's full length)."""
    N, B = 1, 65536
    tt = hh_workload(N, 0.0, 0.05)
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 6)
    y_ref = fast_apply_H(ix, oracle_W(N, tt, 0.4), c)
    y, _ = apply_case(hs, N, B, lib_terms(tt), None, c, t=0.4)
    assert rel2(y, y_ref) <= TOL64


def test_step_with_generic_potential(hs):
    """Hermite-basis terms outside the fused class, through full Lanczos steps."""
    N, B = 3, 120
    degs = [(2, 2, 0), (0, 1, 3), (4, 0, 0), (1, 0, 1), (0, 0, 0)]
    rng = np.random.default_rng(8)
    coefs = rng.standard_normal(len(degs)) * 0.002
    terms = [(float(cf), d) for cf, d in zip(coefs, degs)]
    W = Potential(N, "herm", 1.0, list(zip(coefs, degs)))
    ix = IndexSet(N, B)
    c = coherent_state(ix.k, [0.5, 0.2, -0.3])
    c /= np.linalg.norm(c)
    got, ref, meff = steps_case(hs, N, B, terms, lambda t: W, c, 0.005, 8, 4, basis="herm", harmonic=False)
    assert meff == 8
    assert rel2(got, ref) <= 1e-11


def test_zero_vector_step(hs):
    """||c|| = 0: the step leaves c = 0 and reports m_eff = 0."""
    import torch
    N, B = 2, 64
    tt = hh_workload(N, 0.111, 0.0)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    c = torch.zeros(idx.size, dtype=torch.complex128, device="cuda")
    ws = hs.workspace(idx, pot, hs.HS_C128, 10)
    diag = torch.full((21,), -1.0, dtype=torch.float64, device="cuda")
    hs.step(idx, pot, c, 0.0, 0.01, 10, ws=ws, diag=diag)
    torch.cuda.synchronize()
    assert float(torch.abs(c).max()) == 0.0
    assert diag[0].item() == 0.0
