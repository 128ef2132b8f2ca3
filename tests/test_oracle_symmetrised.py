"""Pins of the oracle's symmetrised fast operator (D + (F + F_rev)/2): exact symmetry on
a reduced set, agreement with products of independently built truncated coordinate
matrices, agreement with F where the factors commute (single-axis terms, the full box),
and the Lanczos exponential being exact for it."""
import numpy as np

from oracle.index import BoxIndex, IndexSet
from oracle.operators import Potential, fast_apply_H, jacobi_matrix, subtract_harmonic, sym_apply_H
from oracle.propagate import lanczos_expm
from synth import coherent_state, complex_normal_by_index, henon_heiles_chain


def _matrix(op, n):
    return np.stack([op(np.eye(n, dtype=np.complex128)[:, i]) for i in range(n)], axis=1)


def _hh(N, lam=0.25):
    V = Potential(N, "mono", 1.0, [(tt.coef(0.0), tt.degrees) for tt in henon_heiles_chain(N, lam)])
    return subtract_harmonic(V)


def _coordinate_matrices(k, P):
    """X^(l)_K as dense matrices, entry by entry from the 1-D Jacobi matrix: rows j and
    columns k of the set, (X^(l))_{jk} = J[j_l, k_l] when j and k agree off axis l."""
    n, N = k.shape
    J = jacobi_matrix(P)
    pos = {tuple(int(x) for x in row): i for i, row in enumerate(k)}
    mats = []
    for l in range(N):
        X = np.zeros((n, n))
        for i, row in enumerate(k):
            for d in (-1, 1):
                m = list(int(x) for x in row)
                m[l] += d
                if m[l] < 0 or tuple(m) not in pos:
                    continue
                X[i, pos[tuple(m)]] = J[row[l], m[l]]
        mats.append(X)
    return mats


def test_symmetric_on_reduced_set_and_differs_from_F():
    N, B = 3, 30
    ix = IndexSet(N, B)
    W = _hh(N)
    S = _matrix(lambda v: sym_apply_H(ix, W, v), ix.size)
    F = _matrix(lambda v: fast_apply_H(ix, W, v), ix.size)
    assert np.max(np.abs(S - S.T)) < 1e-13
    assert np.max(np.abs(S - F)) > 1e-3                 # the coupling terms do not commute here
    assert np.max(np.abs(S - 0.5 * (F + F.T))) < 1e-13  # the symmetric part of F


def test_matches_products_of_truncated_coordinate_matrices():
    """Terms x_1^2 x_2 and x_2 x_3^3 on a hyperbolic set: the symmetrised term is
    (X_1^2 X_2 + X_2 X_1^2)/2 with the truncated matrices built independently."""
    N, B = 3, 24
    ix = IndexSet(N, B)
    W = Potential(N, "mono", 1.0, [(0.7, (2, 1, 0)), (-0.3, (0, 1, 3))])
    X1, X2, X3 = _coordinate_matrices(ix.k.astype(np.int64), B + 4)
    Dg = np.diag(np.sum(ix.k, axis=1) + 0.5 * N)
    ref = Dg + 0.7 * 0.5 * (X1 @ X1 @ X2 + X2 @ X1 @ X1) \
        - 0.3 * 0.5 * (X2 @ X3 @ X3 @ X3 + X3 @ X3 @ X3 @ X2)
    S = _matrix(lambda v: sym_apply_H(ix, W, v), ix.size)
    assert np.max(np.abs(S - ref)) < 1e-12


def test_agrees_with_F_where_factors_commute():
    N, B = 2, 40
    ix = IndexSet(N, B)
    Ws = Potential(N, "mono", 1.0, [(0.3, (3, 0)), (-0.2, (0, 4)), (0.1, (1, 0))])
    c = complex_normal_by_index(ix.k, 5)
    assert np.max(np.abs(sym_apply_H(ix, Ws, c) - fast_apply_H(ix, Ws, c))) < 1e-12
    box = BoxIndex(N, 9)
    W = _hh(N)
    cb = complex_normal_by_index(box.k, 6)
    assert np.max(np.abs(sym_apply_H(box, W, cb) - fast_apply_H(box, W, cb))) < 1e-11


def test_lanczos_is_the_exponential_of_the_symmetric_operator():
    """The Hermitian Lanczos process is exact for S: at full Krylov dimension it returns
    exp(-i h S) c to rounding.  For F (not symmetric on the reduced set) the same process
    with alpha = Re <v, F v> differs from exp(-i h F) c by far more."""
    from scipy.linalg import expm
    N, B = 2, 24
    ix = IndexSet(N, B)
    W = _hh(N, 0.4)
    c = coherent_state(ix.k, [1.2, -0.8])
    c /= np.linalg.norm(c)
    h, n = 0.1, ix.size
    S = _matrix(lambda v: sym_apply_H(ix, W, v), n)
    F = _matrix(lambda v: fast_apply_H(ix, W, v), n)
    ys = lanczos_expm(lambda v: sym_apply_H(ix, W, v), c, h, n)[0]
    yf = lanczos_expm(lambda v: fast_apply_H(ix, W, v), c, h, n)[0]
    assert np.linalg.norm(ys - expm(-1j * h * S) @ c) < 1e-12
    assert np.linalg.norm(yf - expm(-1j * h * F) @ c) > 1e-6
