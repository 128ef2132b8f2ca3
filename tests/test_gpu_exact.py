"""The exact Galerkin operator A = D_K + W_{K,pol} on the GPU (the fast algorithm on a
padded set, restricted to the set) and the unperturbed Lanczos step on it (paper Sec. 6.2,
eq. ErrorPerturbedLanczosAnalysis), against the oracle's densely assembled exact matrix and
its Lanczos exponential; and the perturbation error of the fast algorithm's Lanczos step
against the same difference in the oracle."""
import numpy as np
import pytest

from oracle.index import IndexSet
from oracle.operators import Potential, dense_H, fast_apply_H, torsional_potential
from oracle.propagate import lanczos_expm
from synth import complex_normal_by_index, decay_vector
from tests.hsutil import hh_workload, lib_terms, lib_to_lex, oracle_W, rel2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


def torsional_with_harmonic(N):
    """The perturbation study's potential: the torsional series minus |x|^2 / 2 (x^2 in the
    basis T_r(x / 16): x^2 = 128 (T_0 + T_2))."""
    W = torsional_potential(N)
    terms = list(W.terms)
    terms[0] = (terms[0][0] - 64.0 * N, terms[0][1])
    for l in range(N):
        a = [0] * N
        a[l] = 2
        terms.append((-64.0, tuple(a)))
    return Potential(N, W.basis, W.scale, terms)


def _case(hs, kind, N, B):
    """(oracle potential, library potential, padded set) for the set K_N(B)."""
    if kind == "hh":
        tt = hh_workload(N, 0.111, 0.05)
        W = oracle_W(N, tt, 0.0025)
        pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
        pot.set_time(0.0025)
        pad = hs.Index(N, B, pad=3)
    else:
        W = torsional_with_harmonic(N) if kind == "torsional_ho" else torsional_potential(N)
        pot = hs.Pot(N, [(float(c), a) for c, a in W.terms], basis=W.basis, scale=W.scale)
        pad = hs.Index(N, B - 1 + 4, box=True)  # coordinates <= B - 1, degree 8: 4 more
    return W, pot, pad


@pytest.mark.parametrize("kind,N,B", [("torsional", 2, 11), ("torsional_ho", 2, 31), ("torsional", 3, 41),
                                      ("hh", 3, 12), ("hh", 4, 16)])
def test_exact_apply_vs_dense(hs, kind, N, B):
    import torch
    W, pot, pad = _case(hs, kind, N, B)
    sub = hs.Index(N, B)
    op = hs.ExactOperator(sub, pad)
    ix = IndexSet(N, B)
    lexpos = lib_to_lex(sub, N, B)
    c = complex_normal_by_index(ix.k, 7 + N)
    y_ref = dense_H(ix.k, W) @ c
    x = torch.from_numpy(np.ascontiguousarray(c[lexpos])).to("cuda")
    y = torch.empty_like(x)
    op.apply(pot, x, y)
    torch.cuda.synchronize()
    got = np.empty_like(c)
    got[lexpos] = y.cpu().numpy()
    assert rel2(got, y_ref) <= 1e-12
    # and it is not the fast operator (the sets are reduced: the two differ)
    assert rel2(fast_apply_H(ix, W, c), y_ref) > 1e-9


@pytest.mark.parametrize("reorth", [False, True])
def test_exact_step_vs_oracle_lanczos(hs, reorth):
    """One exponential step, m = 5, h = 1/10, on K_2(11) with the torsional potential and
    the paper's decay vector (beta = 3)."""
    import torch
    N, B, m, h = 2, 11, 5, 0.1
    W, pot, pad = _case(hs, "torsional_ho", N, B)
    sub = hs.Index(N, B)
    op = hs.ExactOperator(sub, pad)
    ix = IndexSet(N, B)
    lexpos = lib_to_lex(sub, N, B)
    v = decay_vector(ix.k, 3.0)
    v /= np.linalg.norm(v)
    H = dense_H(ix.k, W)
    ref, m_eff, _, _ = lanczos_expm(lambda u: H @ u, v, h, m, reorth)
    c = torch.from_numpy(np.ascontiguousarray(v[lexpos])).to("cuda")
    diag = torch.zeros(1 + 2 * m, dtype=torch.float64, device="cuda")
    op.step(pot, c, 0.0, h, m, reorth=reorth, diag=diag)
    torch.cuda.synchronize()
    got = np.empty_like(v)
    got[lexpos] = c.cpu().numpy()
    assert int(diag[0].item()) == m_eff
    assert rel2(got, ref) <= 1e-12


@pytest.mark.parametrize("N,B,h", [(2, 11, 0.1), (2, 21, 0.05), (3, 41, 0.1)])
def test_perturbation_error_vs_oracle(hs, N, B, h):
    """|| V_m exp(-ihT_m) e_1 - V~_m exp(-ihT~_m) e_1 ||_2: the exact operator's Lanczos
    step against the fast algorithm's, from the decay vector, m = 5, no
    re-orthogonalisation, on the GPU and in the oracle."""
    import torch
    m = 5
    W, pot, pad = _case(hs, "torsional_ho", N, B)
    sub = hs.Index(N, B)
    op = hs.ExactOperator(sub, pad)
    ix = IndexSet(N, B)
    lexpos = lib_to_lex(sub, N, B)
    v = decay_vector(ix.k, 3.0)
    v /= np.linalg.norm(v)
    H = dense_H(ix.k, W)
    exact, _, _, _ = lanczos_expm(lambda u: H @ u, v, h, m, False)
    fast, _, _, _ = lanczos_expm(lambda u: fast_apply_H(ix, W, u), v, h, m, False)
    e_ref = float(np.linalg.norm(exact - fast))
    a = torch.from_numpy(np.ascontiguousarray(v[lexpos])).to("cuda")
    b = a.clone()
    op.step(pot, a, 0.0, h, m, reorth=False)
    hs.step(sub, pot, b, 0.0, h, m, reorth=False)
    torch.cuda.synchronize()
    e_gpu = float(torch.linalg.norm(a - b))
    assert e_ref > 1e-9  # a real perturbation
    assert abs(e_gpu - e_ref) <= 1e-13
