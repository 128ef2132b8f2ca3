"""Pins of the oracle's operators against what the paper and the mathematics fix:
closed forms of the Hermite recurrence, an independent quadrature of the 1-D Galerkin
entries, the harmonic oscillator, padded exactness, interior rows, Lemma 1, the
adjoint identity, basis changes and the printed error table of Fig. 9."""
import math
import os

import numpy as np
import pytest

from oracle.index import BoxIndex, IndexSet
from oracle.operators import (Potential, dense_H, dense_W, direct_op, error_split,
                              exact_1d, exact_W_separable, fast_apply_H, fast_apply_W,
                              fast_H_rows, gh_1d, gh_W, jacobi_matrix, poly_values,
                              subtract_harmonic, torsional_potential)
from synth import complex_normal_by_index, decay_vector, henon_heiles_chain

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def hh_W(N, lam=0.111, laser=0.0, t=0.0):
    V = Potential(N, "mono", 1.0, [(tt.coef(t), tt.degrees) for tt in
                                    henon_heiles_chain(N, lam, laser)])
    return subtract_harmonic(V)


def matrix_of(op, n):
    return np.stack([op(np.eye(n, dtype=np.complex128)[:, i]) for i in range(n)], axis=1)


# ---- 1-D entries ----------------------------------------------------------------


def test_exact_1d_against_independent_quadrature():
    """(phi_i, x^a phi_k) from the padded Jacobi power equals a high-order Gauss-Hermite
    integral of the explicit Hermite functions phi_k = pi^-1/4 (2^k k!)^-1/2 H_k e^{-x^2/2}
    (closed form of Sec. 1.1), with numpy's Hermite polynomial evaluator."""
    x, w = np.polynomial.hermite.hermgauss(80)
    kmax = 12
    H = np.stack([np.polynomial.hermite.hermval(x, [0] * k + [1]) for k in range(kmax + 1)])
    norm = np.array([math.pi ** -0.25 / math.sqrt(2.0 ** k * math.factorial(k)) for k in range(kmax + 1)])
    psi = H * norm[:, None]
    for a in range(0, 6):
        Q = exact_1d("mono", 1.0, a, kmax)
        ref = (psi * (w * x ** a)) @ psi.T
        assert np.allclose(Q, ref, atol=1e-11, rtol=1e-11)


def test_jacobi_recurrence_closed_form():
    # x phi_k = sqrt((k+1)/2) phi_{k+1} + sqrt(k/2) phi_{k-1}: J[k, k+1] = sqrt((k+1)/2)
    J = jacobi_matrix(6)
    for k in range(6):
        assert J[k, k + 1] == pytest.approx(math.sqrt((k + 1) / 2.0))
        assert J[k + 1, k] == J[k, k + 1]
    assert np.all(np.diag(J) == 0)


@pytest.mark.parametrize("basis,scale", [("cheb", 3.0), ("herm", 1.7), ("mono", 1.0)])
def test_poly_values_closed_forms(basis, scale):
    x = np.linspace(-2, 2, 7)
    y = x / scale
    if basis == "cheb":
        ref = [np.ones_like(y), y, 2 * y * y - 1, 4 * y ** 3 - 3 * y, 8 * y ** 4 - 8 * y ** 2 + 1]
    elif basis == "herm":
        ref = [np.ones_like(y), 2 * y, 4 * y * y - 2, 8 * y ** 3 - 12 * y, 16 * y ** 4 - 48 * y ** 2 + 12]
    else:
        ref = [x ** k for k in range(5)]
    for a in range(5):
        assert np.allclose(poly_values(basis, scale, a, x), ref[a], rtol=1e-13, atol=1e-13)


# ---- single coordinate operator and the harmonic oscillator ---------------------


@pytest.mark.parametrize("N,B,l", [(2, 30, 0), (2, 30, 1), (3, 40, 1), (4, 24, 3)])
def test_single_X_equals_exact_galerkin(N, B, l):
    """X_K^(l) is the exact Galerkin matrix of q_l on the set (Sec. 3.1): the fast
    algorithm for W = x_l equals the dense definition exactly."""
    idx = IndexSet(N, B)
    a = [0] * N
    a[l] = 1
    pot = Potential(N, "mono", 1.0, [(1.0, tuple(a))])
    F = matrix_of(lambda v: fast_apply_W(idx, pot, v), idx.size)
    E = dense_W(idx.k, pot)
    assert np.max(np.abs(F - E)) < 1e-14
    assert np.max(np.abs(F - F.T)) == 0.0


def test_harmonic_potential_gives_diagonal():
    """V = |x|^2 / 2  =>  W = 0  =>  H = D = diag(sum (k_l + 1/2)) (Sec. 1.2)."""
    N, B = 3, 50
    idx = IndexSet(N, B)
    V = Potential(N, "mono", 1.0, [(0.5, (2, 0, 0)), (0.5, (0, 2, 0)), (0.5, (0, 0, 2))])
    W = subtract_harmonic(V)
    assert W.terms == []
    c = complex_normal_by_index(idx.k, 1)
    y = fast_apply_H(idx, W, c)
    D = idx.k.sum(axis=1) + 1.5
    assert np.array_equal(y, D * c)
    Hd = dense_H(idx.k, W)
    assert np.array_equal(np.diag(Hd), D.astype(np.complex128))


def test_x_squared_on_truncated_fibre_closed_form():
    """On a fibre {0..m} the truncated (X^2) has diagonal i + 1/2 except at the top, where
    the missing neighbour leaves m/2; off-diagonals sqrt((i+1)(i+2))/2."""
    N, B = 1, 9  # one fibre 0..8
    idx = IndexSet(N, B)
    pot = Potential(1, "mono", 1.0, [(1.0, (2,))])
    F = matrix_of(lambda v: fast_apply_W(idx, pot, v), idx.size).real
    m = B - 1
    for i in range(m + 1):
        assert F[i, i] == pytest.approx(i + 0.5 if i < m else m / 2.0, abs=1e-14)
        if i + 2 <= m:
            assert F[i, i + 2] == pytest.approx(math.sqrt((i + 1) * (i + 2)) / 2.0, abs=1e-14)


# ---- padded exactness, interior rows, Lemma 1 -----------------------------------


@pytest.mark.parametrize("N,B", [(2, 20), (3, 16)])
def test_fast_on_padded_box_equals_exact(N, B):
    """On a box {0..B-1+deg}^N no path from the set is truncated, so the fast algorithm
    restricted to the set equals the exact Galerkin product (independent code paths:
    sequential direct operations vs. padded 1-D matrices and tensor assembly)."""
    idx = IndexSet(N, B)
    W = hh_W(N, lam=0.2)
    deg = 3
    box = BoxIndex(N, B - 1 + deg)
    c = complex_normal_by_index(idx.k, 5)
    from oracle.operators import extend_zero, restrict_full
    yb = restrict_full(box, idx.k, fast_apply_W(box, W, extend_zero(box, idx.k, c)))
    ye = dense_W(idx.k, W) @ c
    assert np.max(np.abs(yb - ye)) / np.max(np.abs(ye)) < 1e-13


def test_interior_rows_have_no_error():
    """Rows j with j + a_t in K for every term: every path stays in the set, so the
    fast row equals the exact Galerkin row (remark after Theorem 2)."""
    N, B = 2, 60
    idx = IndexSet(N, B)
    W = hh_W(N)
    F = matrix_of(lambda v: fast_apply_W(idx, W, v), idx.size)
    E = dense_W(idx.k, W)
    k = idx.k.astype(np.int64)
    interior = np.ones(idx.size, dtype=bool)
    for _, a in W.terms:
        interior &= np.prod(1 + k + np.array(a), axis=1) <= B
    assert interior.sum() > 20
    assert np.max(np.abs(F[interior] - E[interior])) < 1e-12
    # and the truncation does matter somewhere else
    assert np.max(np.abs(F[~interior] - E[~interior])) > 1e-3


@pytest.mark.parametrize("N,Kmax", [(2, 9), (3, 5)])
def test_lemma1_full_box_equals_gauss_hermite(N, Kmax):
    """Lemma 1: on the full set the insertion equals product Gauss-Hermite quadrature
    with Kmax + 1 nodes per axis (Sec. 4.2)."""
    box = BoxIndex(N, Kmax)
    W = hh_W(N, lam=0.3)
    F = matrix_of(lambda v: fast_apply_W(box, W, v), box.size)
    G = gh_W(box.k, W, Kmax)
    assert np.max(np.abs(F - G)) < 1e-12
    # with too few nodes the identity fails (the pin is not vacuous)
    G2 = gh_W(box.k, W, Kmax - 2)
    assert np.max(np.abs(F - G2)) > 1e-3


def test_gh_nodes_are_jacobi_eigenvalues():
    """X_full = U^T Xi U (Sec. 4.2): the Gauss-Hermite nodes are the eigenvalues of the
    (M+1) x (M+1) Jacobi matrix (Golub-Welsch), and the weights come from the first
    components of the eigenvectors."""
    from oracle.operators import gh_nodes_weights
    M = 14
    xi, w = gh_nodes_weights(M)
    lam, U = np.linalg.eigh(jacobi_matrix(M))
    assert np.allclose(np.sort(xi), lam, atol=1e-12)
    assert np.allclose(w[np.argsort(xi)], math.sqrt(math.pi) * U[0] ** 2, rtol=1e-10)
    # the 1-D GH matrix of x with M = Kmax reproduces the Jacobi matrix
    assert np.allclose(gh_1d("mono", 1.0, 1, M, M), jacobi_matrix(M), atol=1e-12)


# ---- symmetry and axis order ----------------------------------------------------


def test_adjoint_identity_and_hermiticity():
    """On a reduced set the X_K^(l) do not commute, so the fast operator F with axis N
    applied first satisfies F^T = F_rev (axis 1 first): <u, F v> = <F_rev u, v>.
    Exact Hermiticity holds for the dense definition, for F on a full box and for
    potentials whose terms touch one axis."""
    N, B = 2, 40
    idx = IndexSet(N, B)
    W = hh_W(N, lam=0.25)
    u = complex_normal_by_index(idx.k, 11)
    v = complex_normal_by_index(idx.k, 12)
    lhs = np.vdot(u, fast_apply_W(idx, W, v))
    rhs = np.vdot(fast_apply_W(idx, W, u, axis_order="rev"), v)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # the mixed term really breaks symmetry on the hyperbolic set
    F = matrix_of(lambda x: fast_apply_W(idx, W, x), idx.size)
    assert np.max(np.abs(F - F.T)) > 1e-2
    # dense definition: Hermitian
    Hd = dense_H(idx.k, W)
    assert np.max(np.abs(Hd - Hd.conj().T)) < 1e-12
    # single-axis potential on the hyperbolic set: symmetric
    Ws = Potential(N, "mono", 1.0, [(0.3, (3, 0)), (-0.2, (0, 4))])
    Fs = matrix_of(lambda x: fast_apply_W(idx, Ws, x), idx.size)
    assert np.max(np.abs(Fs - Fs.T)) < 1e-12
    # full box: symmetric even with the coupling term
    box = BoxIndex(N, 8)
    Fb = matrix_of(lambda x: fast_apply_W(box, W, x), box.size)
    assert np.max(np.abs(Fb - Fb.T)) < 1e-12


def test_same_operator_in_three_bases():
    """x^2 = (L^2/2)(T_2(x/L) + 1), x^3 = L^3 (T_3 + 3 T_1)/4, x^2 = (H_2 + 2)/4,
    x^3 = (H_3 + 6 H_1)/8: a per-axis basis change leaves the operator unchanged
    (p(X) is linear in the polynomial)."""
    N, B = 3, 80
    idx = IndexSet(N, B)
    L = 5.0
    mono = Potential(N, "mono", 1.0, [(0.7, (2, 1, 0)), (-0.4, (0, 0, 3))])
    cheb = Potential(N, "cheb", L, [
        (0.7 * L ** 2 / 2 * L, (2, 1, 0)), (0.7 * L ** 2 / 2 * L, (0, 1, 0)),
        (-0.4 * L ** 3 / 4, (0, 0, 3)), (-0.4 * L ** 3 * 3 / 4, (0, 0, 1))])
    herm = Potential(N, "herm", 1.0, [
        (0.7 / 4 / 2, (2, 1, 0)), (0.7 * 2 / 4 / 2, (0, 1, 0)),
        (-0.4 / 8, (0, 0, 3)), (-0.4 * 6 / 8, (0, 0, 1))])
    c = complex_normal_by_index(idx.k, 2)
    y0 = fast_apply_W(idx, mono, c)
    for p in (cheb, herm):
        y = fast_apply_W(idx, p, c)
        assert np.max(np.abs(y - y0)) <= 1e-12 * np.max(np.abs(y0))


def test_row_evaluation_matches_sequential_passes():
    """The layered-tree row evaluation (windows per layer) equals the sequential direct
    operations of the fast algorithm."""
    N, B = 4, 300
    idx = IndexSet(N, B)
    W = hh_W(N, lam=0.15, laser=0.05, t=0.3)
    c = complex_normal_by_index(idx.k, 9)
    y = fast_apply_H(idx, W, c)
    rng = np.random.default_rng(0)
    rows = rng.choice(idx.size, 60, replace=False)
    lookup = lambda m: c[idx.rank(np.array(m))[0]]  # noqa: E731
    yr = fast_H_rows(N, B, W, lookup, idx.k[rows])
    assert np.max(np.abs(yr - y[rows])) <= 1e-12 * np.max(np.abs(y))


def test_direct_op_boundary_cases():
    """j_l = 0 has no lower neighbour; a missing upper neighbour contributes zero even
    below the per-axis maximum (reduced set)."""
    idx = IndexSet(2, 12)
    v = np.zeros(idx.size, dtype=np.complex128)
    j = idx.rank(np.array([[2, 3]]))[0]  # (1+2)(1+3) = 12: top of both fibres
    v[j] = 1.0
    y = direct_op(idx, 0, v)
    lo = idx.rank(np.array([[1, 3]]))[0]
    assert y[lo] == pytest.approx(math.sqrt(2 / 2.0))
    assert np.count_nonzero(y) == 1


# ---- the printed error table (Fig. 9) --------------------------------------------


def load_fig9():
    rows = []
    with open(os.path.join(GOLDEN, "fig9_local_errors.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            q, K, N, val = line.split()
            rows.append((q, int(K), int(N), float(val)))
    return rows


def _fig9_case(N, Kp):
    idx = IndexSet(N, Kp + 1)
    box = BoxIndex(N, Kp)
    pot = torsional_potential(N)
    v = decay_vector(idx.k, 5.0)
    v /= np.linalg.norm(v)
    eq, er = error_split(idx, box, pot, v, exact_W_separable(idx, pot, v))
    return np.max(np.abs(eq)), np.max(np.abs(er))


@pytest.mark.parametrize("N,Kp", [(2, 25), (2, 50), (2, 75), (3, 25), (3, 50), (3, 75), (4, 25)])
def test_fig9_local_error_table(N, Kp):
    """E^quad v and E^red(v) reproduce the printed infinity norms to the printed digits
    (within one unit of the last digit)."""
    table = {(q, K, n): val for q, K, n, val in load_fig9()}
    eq, er = _fig9_case(N, Kp)
    assert eq == pytest.approx(table[("Equad", Kp, N)], rel=2e-3)
    assert er == pytest.approx(table[("Ered", Kp, N)], rel=2e-3)


def test_exact_separable_matches_dense():
    N, B = 3, 30
    idx = IndexSet(N, B)
    pot = torsional_potential(N, L=4.0, R=5)
    v = complex_normal_by_index(idx.k, 4)
    assert np.allclose(exact_W_separable(idx, pot, v), dense_W(idx.k, pot) @ v, atol=1e-12)


@pytest.mark.parametrize("N,B,w", [(2, 24, 3), (3, 12, 3), (2, 24, 4)])
def test_padded_cross_gives_the_exact_galerkin_product(N, B, w):
    """On a hyperbolic cross K, the fast algorithm on the cross widened by w >= the largest
    per-axis degree, applied to v extended by zero and restricted to K, is the exact
    Galerkin product (D + W_K) v of the densely assembled exact matrix: every intermediate
    index of a product between two rows of K differs from its start by at most the term's
    degree in each axis.  Without the widening (w = 0) the two differ (the gap that
    hs_error_split reports at scale)."""
    from oracle.index import PaddedIndex
    tt = henon_heiles_chain(N, 0.111, 0.05)
    W = subtract_harmonic(Potential(N, "mono", 1.0, [(x.coef(0.3), x.degrees) for x in tt]))
    ix = IndexSet(N, B)
    v = complex_normal_by_index(ix.k, 3)
    exact = dense_H(ix.k, W) @ v
    for ww in (w, 0):
        P = PaddedIndex(N, B, ww)
        rows = P.rank(ix.k)
        x = np.zeros(P.size, dtype=np.complex128)
        x[rows] = v
        got = fast_apply_H(P, W, x)[rows]
        err = np.linalg.norm(got - exact) / np.linalg.norm(exact)
        if ww:
            assert err <= 1e-13
        else:
            assert err > 1e-6


def test_exact_rows_match_the_dense_galerkin_matrix():
    """exact_H_rows restates the Galerkin matrix row by row; on a tiny set it must agree
    with the dense assembly, and differ from the fast algorithm at rows that reach the
    boundary of K (the reduced set truncates the nested products there)."""
    import numpy as np
    from oracle.index import IndexSet
    from oracle.operators import Potential, dense_H, exact_H_rows, fast_H_rows
    N, B = 3, 40
    ix = IndexSet(N, B)
    rng = np.random.default_rng(5)
    v = rng.normal(size=ix.size) + 1j * rng.normal(size=ix.size)
    pos = {tuple(int(x) for x in k): i for i, k in enumerate(ix.k)}
    look = lambda m: v[pos[tuple(m)]]  # noqa: E731
    for basis, scale in (("mono", 1.0), ("herm", 1.3)):
        pot = Potential(N, basis, scale, [(0.2, (2, 1, 0)), (-0.1, (0, 0, 3)), (0.05, (1, 1, 1))])
        ref = dense_H(ix.k, pot) @ v
        got = exact_H_rows(N, B, pot, look, ix.k)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
        fast = fast_H_rows(N, B, pot, look, ix.k)
        assert np.max(np.abs(fast - ref)) > 1e-6 * np.max(np.abs(ref))
