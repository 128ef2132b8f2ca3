"""GPU parity of y = H c (fused and generic kernels, float64 and float32) against the CPU
oracle's fast algorithm, through the C ABI."""
import numpy as np
import pytest

from oracle.index import IndexSet
from oracle.operators import Potential, fast_apply_H, fast_H_rows, dense_H
from synth import complex_normal_by_index, coherent_state
from tests.hsutil import lib_terms, lib_to_lex, oracle_W, rel2, hh_workload

pytestmark = pytest.mark.gpu

TOL64 = 1e-12   # float64 parity (relative 2-norm)


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1403_3511_amd import hs as _hs
    return _hs


def run_apply(hs, N, B, timeterms, t, c_lex, dtype=0, tile_dim=0, basis="mono", scale=1.0,
              harmonic=True, lexpos=None, idx=None):
    import torch
    if idx is None:
        idx = hs.Index(N, B, tile_dim)
    pot = hs.Pot(N, timeterms, basis=basis, scale=scale, subtract_harmonic=harmonic)
    pot.set_time(t)
    if lexpos is None:
        lexpos = lib_to_lex(idx, N, B)
    c_lib = c_lex[lexpos]
    tdt = torch.complex128 if dtype == 0 else torch.complex64
    c = torch.from_numpy(c_lib).to("cuda").to(tdt)
    y = torch.empty_like(c)
    hs.apply_h(idx, pot, c, y, dtype)
    torch.cuda.synchronize()
    y_lib = y.cpu().numpy().astype(np.complex128)
    y_lex = np.empty_like(y_lib)
    y_lex[lexpos] = y_lib
    return y_lex, pot


@pytest.mark.parametrize("N,B,lam,laser,t", [
    (1, 50, 0.0, 0.05, 0.3),
    (2, 64, 0.111, 0.0, 0.0),        # Henon-Heiles, workload size of the small config
    (2, 300, 0.111, 0.05, 0.7),
    (3, 500, 0.1, 0.05, 0.2),
    (4, 700, 0.12, 0.05, 1.1),
    (6, 512, 0.111, 0.05, 0.4),
])
def test_hh_fused_float64_parity(hs, N, B, lam, laser, t):
    tt = hh_workload(N, lam, laser)
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 17)
    y_ref = fast_apply_H(ix, oracle_W(N, tt, t), c)
    y, pot = run_apply(hs, N, B, lib_terms(tt), t, c)
    assert pot.fused
    assert rel2(y, y_ref) <= TOL64


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_tile_dims_agree(hs, d):
    N, B = 4, 600
    tt = hh_workload(N, 0.111, 0.05)
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 3)
    y_ref = fast_apply_H(ix, oracle_W(N, tt, 0.25), c)
    y, _ = run_apply(hs, N, B, lib_terms(tt), 0.25, c, tile_dim=d)
    assert rel2(y, y_ref) <= TOL64


def test_generic_program_hermite_degree6(hs):
    """A potential outside the fused class (degree-6 Hermite terms over 3 axes) runs
    through the generic recurrence-pass program."""
    N, B = 3, 200
    rng = np.random.default_rng(5)
    degs = [(2, 2, 2), (6, 0, 0), (1, 3, 2), (0, 0, 4), (3, 1, 0), (0, 2, 1), (0, 0, 0), (1, 1, 1)]
    coefs = rng.standard_normal(len(degs)) * 0.01
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 4)
    W = Potential(N, "herm", 1.3, list(zip(coefs, degs)))
    y_ref = fast_apply_H(ix, W, c)
    y, pot = run_apply(hs, N, B, [(float(cf), d) for cf, d in zip(coefs, degs)], 0.0, c,
                       basis="herm", scale=1.3, harmonic=False)
    assert not pot.fused
    assert rel2(y, y_ref) <= TOL64


def test_chebyshev_basis_fused(hs):
    """Chebyshev-basis Henon-Heiles-type terms are converted to the fused form."""
    N, B, L = 3, 300, 6.0
    degs = [(2, 1, 0), (0, 3, 0), (0, 0, 1), (1, 0, 0), (0, 2, 1)]
    coefs = [0.3, -0.2, 0.1, 0.05, 0.07]
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 6)
    y_ref = fast_apply_H(ix, Potential(N, "cheb", L, list(zip(coefs, degs))), c)
    y, pot = run_apply(hs, N, B, list(zip(coefs, degs)), 0.0, c, basis="cheb", scale=L,
                       harmonic=False)
    assert pot.fused
    assert rel2(y, y_ref) <= TOL64


def test_float32_matvec_error_stated(hs):
    N, B = 4, 700
    tt = hh_workload(N, 0.111, 0.05)
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 8)
    y_ref = fast_apply_H(ix, oracle_W(N, tt, 0.5), c)
    y, _ = run_apply(hs, N, B, lib_terms(tt), 0.5, c, dtype=1)
    err = rel2(y, y_ref)
    print(f"float32 matvec relative error vs float64 oracle: {err:.3e}")
    assert err < 1e-5


def test_harmonic_only_is_diagonal(hs):
    N, B = 3, 100
    tt = hh_workload(N, 0.0, 0.0)
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 2)
    y, _ = run_apply(hs, N, B, lib_terms([x for x in tt if sum(x.degrees) == 2]), 0.0, c)
    D = ix.k.sum(axis=1) + 1.5
    assert np.array_equal(y, D * c)


def test_gap_to_exact_galerkin_reported(hs):
    """Gap between the fast operator and the exact Galerkin matrix on the small config
    (reported, not a pass/fail target beyond sanity)."""
    N, B = 2, 64
    tt = hh_workload(N)
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 0)
    y, _ = run_apply(hs, N, B, lib_terms(tt), 0.0, c)
    ye = dense_H(ix.k, oracle_W(N, tt, 0.0)) @ c
    gap = rel2(y, ye)
    print(f"N=2 B=64 Henon-Heiles: ||H_fast c - H_exact c|| / ||H_exact c|| = {gap:.3e}")
    assert gap < 1.0


def test_full_size_sampled_rows(hs):
    """N = 6, B = 4096 (4,883,360 rows), chained Henon-Heiles + laser, packet at x_d = 2:
    the full-size launch checked on sampled rows computed one by one by the oracle's
    layered-tree evaluation."""
    import torch
    N, B = 6, 4096
    tt = hh_workload(N, 0.111, 0.05)
    idx = hs.Index(N, B)
    k = idx.multi_indices()
    c_lib = coherent_state(k, 2.0)
    c_lib /= np.linalg.norm(c_lib)
    rng = np.random.default_rng(1)
    c_lib = c_lib + 1e-3 * (rng.standard_normal(c_lib.size) + 1j * rng.standard_normal(c_lib.size)) / np.sqrt(c_lib.size)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    pot.set_time(0.3)
    c = torch.from_numpy(c_lib).to("cuda")
    y = torch.empty_like(c)
    hs.apply_h(idx, pot, c, y)
    y_lib = y.cpu().numpy()
    # row lookup by multi-index
    from oracle.index import LexRanker
    lexpos = LexRanker(N, B).rank(k.astype(np.int64))
    inv = np.empty_like(lexpos)
    inv[lexpos] = np.arange(lexpos.size)
    ranker = LexRanker(N, B)
    lookup = lambda m: c_lib[inv[ranker.rank(np.array(m))[0]]]  # noqa: E731
    rows = np.concatenate([np.arange(0, 40), rng.choice(idx.size, 160, replace=False)])
    y_ref = fast_H_rows(N, B, oracle_W(N, tt, 0.3), lookup, k[rows])
    assert rel2(y_lib[rows], y_ref) <= TOL64
