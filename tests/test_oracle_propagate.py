"""Pins of the oracle's Magnus-Lanczos propagator (Sec. 2, Fig. 4): dense exponentials on
tiny sets, norm conservation, harmonic-oscillator phases and coherent-state motion."""
import math

import numpy as np
import pytest

from oracle.index import IndexSet
from oracle.operators import Potential, dense_H, fast_apply_H, subtract_harmonic
from oracle.propagate import dense_expm_apply, lanczos_expm, propagate
from synth import coherent_state, complex_normal_by_index, henon_heiles_chain


def test_lanczos_matches_dense_exponential_on_symmetric_operator():
    """Single-axis potential on the reduced set: the fast operator is symmetric, and
    10 Lanczos steps reproduce exp(-i h A) c from a dense eigendecomposition."""
    N, B = 2, 30
    idx = IndexSet(N, B)
    W = Potential(N, "mono", 1.0, [(0.05, (4, 0)), (-0.1, (0, 3)), (0.2, (1, 0))])
    A = np.stack([fast_apply_H(idx, W, e) for e in np.eye(idx.size, dtype=np.complex128)], axis=1)
    assert np.max(np.abs(A - A.T)) < 1e-12
    c = complex_normal_by_index(idx.k, 3)
    c /= np.linalg.norm(c)
    h = 0.01
    y, m_eff, _, _ = lanczos_expm(lambda v: fast_apply_H(idx, W, v), c, h, 10)
    ref = dense_expm_apply(A, c, h)
    assert m_eff == 10
    # Krylov truncation error at m = 10 is a few 1e-12 here (h ||A|| ~ 1); it falls to
    # rounding level as m grows
    assert np.linalg.norm(y - ref) < 1e-10
    y20, _, _, _ = lanczos_expm(lambda v: fast_apply_H(idx, W, v), c, h, 20)
    assert np.linalg.norm(y20 - ref) < 1e-13


def test_lanczos_exact_in_invariant_subspace():
    """A start vector in a 3-dimensional invariant subspace: breakdown after 3 steps and
    the result is exact (H = D, c supported on 3 basis vectors)."""
    N, B = 2, 20
    idx = IndexSet(N, B)
    W = Potential(N, "mono", 1.0, [])
    c = np.zeros(idx.size, dtype=np.complex128)
    c[[0, 5, 9]] = [1.0, 2.0j, -0.5]
    h = 0.3
    y, m_eff, _, _ = lanczos_expm(lambda v: fast_apply_H(idx, W, v), c, h, 10)
    D = idx.k.sum(axis=1) + 1.0
    assert m_eff == 3
    assert np.allclose(y, np.exp(-1j * h * D) * c, atol=1e-13)


def test_eigenvector_breaks_down_at_once():
    N, B = 3, 16
    idx = IndexSet(N, B)
    c = np.zeros(idx.size, dtype=np.complex128)
    c[0] = 1.0
    y, m_eff, alpha, beta = lanczos_expm(lambda v: fast_apply_H(idx, Potential(N), v), c, 0.1, 10)
    assert m_eff == 1
    assert alpha[0] == pytest.approx(1.5)
    assert y[0] == pytest.approx(np.exp(-0.15j))


def test_harmonic_phases_and_coherent_motion():
    """V = |x|^2/2: c_k(t) = exp(-i (|k| + N/2) t) c_k(0) and <x_1>(t) = x0 cos t."""
    N, B = 2, 64
    idx = IndexSet(N, B)
    V = Potential(N, "mono", 1.0, [(0.5, (2, 0)), (0.5, (0, 2))])
    W = subtract_harmonic(V)
    x0 = 1.0
    c0 = coherent_state(idx.k, [x0, 0.0])
    c0 /= np.linalg.norm(c0)
    h, n = 0.01, 100
    c, _ = propagate(idx, lambda t: W, lambda p: (lambda v: fast_apply_H(idx, p, v)),
                     c0, 0.0, h, n, 10)
    t = h * n
    D = idx.k.sum(axis=1) + 1.0
    assert np.max(np.abs(c - np.exp(-1j * t * D) * c0)) < 1e-11
    X1 = Potential(N, "mono", 1.0, [(1.0, (1, 0))])
    from oracle.operators import fast_apply_W
    xm = np.vdot(c, fast_apply_W(idx, X1, c)).real
    assert xm == pytest.approx(x0 * math.cos(t) * np.sqrt(2) / np.sqrt(2), abs=1e-9)


def test_shifted_oscillator_ehrenfest():
    """V = |x|^2/2 + f x_1 (time independent): <x_1>(t) = x0 cos t - f (1 - cos t),
    exact classical motion for a quadratic potential (Ehrenfest)."""
    N, B = 2, 64
    idx = IndexSet(N, B)
    f = 0.3
    W = Potential(N, "mono", 1.0, [(f, (1, 0))])
    x0 = 1.0
    c0 = coherent_state(idx.k, [x0, 0.0])
    c0 /= np.linalg.norm(c0)
    h, n = 0.02, 100
    c, _ = propagate(idx, lambda t: W, lambda p: (lambda v: fast_apply_H(idx, p, v)),
                     c0, 0.0, h, n, 10)
    t = h * n
    from oracle.operators import fast_apply_W
    X1 = Potential(N, "mono", 1.0, [(1.0, (1, 0))])
    xm = np.vdot(c, fast_apply_W(idx, X1, c)).real
    assert xm == pytest.approx(x0 * math.cos(t) - f * (1 - math.cos(t)), abs=1e-8)


def test_norm_conservation_henon_heiles():
    """Norm conservation under propagation (unitary small exponential, reorthogonalised
    Lanczos basis) for the config-1 workload: N = 2, B = 64, Henon-Heiles."""
    N, B = 2, 64
    idx = IndexSet(N, B)
    terms = henon_heiles_chain(N, 0.111)
    V = Potential(N, "mono", 1.0, [(tt.coef(0.0), tt.degrees) for tt in terms])
    W = subtract_harmonic(V)
    c0 = complex_normal_by_index(idx.k, 0)
    n0 = np.linalg.norm(c0)
    c, m_effs = propagate(idx, lambda t: W, lambda p: (lambda v: fast_apply_H(idx, p, v)),
                          c0, 0.0, 0.01, 100, 10)
    assert all(m == 10 for m in m_effs)
    assert abs(np.linalg.norm(c) - n0) <= 1e-12 * 100 * n0


def test_lanczos_vs_dense_on_hermitian_definition():
    """The dense exact Galerkin H is Hermitian; Lanczos on it equals its exponential."""
    N, B = 2, 24
    idx = IndexSet(N, B)
    terms = henon_heiles_chain(N, 0.111)
    V = Potential(N, "mono", 1.0, [(tt.coef(0.0), tt.degrees) for tt in terms])
    H = dense_H(idx.k, subtract_harmonic(V))
    c = complex_normal_by_index(idx.k, 8)
    y, _, _, _ = lanczos_expm(lambda v: H @ v, c, 0.01, 10)
    assert np.linalg.norm(y - dense_expm_apply(H, c, 0.01)) < 1e-11 * np.linalg.norm(c)
