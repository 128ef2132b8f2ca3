"""Pins of the oracle's Chebyshev interpolation of a potential on [-L, L]^N (Sec. 1.3):
exact reproduction of polynomials (against numpy's power-to-Chebyshev conversion), the
interpolation property at the grid nodes (against numpy's Chebyshev evaluator),
exponential convergence for the Gaussian wells, and the fast operator built from the
coefficients against the one built from the monomials."""
import itertools
import math

import numpy as np
from numpy.polynomial import chebyshev as Ch

from oracle.index import IndexSet
from oracle.operators import Potential, fast_apply_H
from oracle.surrogate import cheb_interpolate, circle_centres, gaussian_sum_W, total_degree_list
from synth import complex_normal_by_index, surrogate_geometry


def _hh(x, L):
    y = x / L
    return y[:, 0] ** 2 * y[:, 1] - y[:, 1] ** 3 / 3.0 - 0.3 * y[:, 2] + 0.2 * y[:, 0] * y[:, 2] ** 2


def test_reproduces_polynomials():
    """W = y1^2 y2 - y2^3/3 - 0.3 y3 + 0.2 y1 y3^2 (y = x/L) has per-axis degree <= 3: its
    interpolant on any grid with R >= 3 is W itself, so the coefficients equal the tensor
    Chebyshev expansion from numpy's poly2cheb (and vanish elsewhere)."""
    N, R, L = 3, 5, 4.0
    rset = list(itertools.product(range(R + 1), repeat=N))
    got = dict(zip(rset, cheb_interpolate(lambda x: _hh(x, L), N, R, L, rset)))
    want = {}
    for coef, degs in [(1.0, (2, 1, 0)), (-1.0 / 3.0, (0, 3, 0)), (-0.3, (0, 0, 1)), (0.2, (1, 0, 2))]:
        per = [Ch.poly2cheb([0.0] * d + [1.0]) for d in degs]
        for js in itertools.product(*[range(len(p)) for p in per]):
            want[js] = want.get(js, 0.0) + coef * np.prod([per[l][j] for l, j in enumerate(js)])
    for r in rset:
        assert abs(got[r] - want.get(r, 0.0)) < 1e-14, r


def _wells(N, t=0.7):
    g = surrogate_geometry(N, 3, 7)
    c = circle_centres(t, 0.6, 1.3, g["base"], g["u"], g["w"], g["phase"])
    return lambda x: gaussian_sum_W(x, [1.2, 0.8, 1.5], 1.1, c)


def test_interpolates_at_the_grid_nodes():
    """The full-grid interpolant equals W at every grid node (numpy's chebval2d-style
    evaluation of the tensor series at a sample of nodes)."""
    N, R, L = 2, 9, 3.0
    f = _wells(N)
    rset = list(itertools.product(range(R + 1), repeat=N))
    a = cheb_interpolate(f, N, R, L, rset)
    A = np.zeros((R + 1, R + 1))
    for coef, r in zip(a, rset):
        A[r] = coef
    theta = (2 * np.arange(R + 1) + 1) * np.pi / (2 * (R + 1))
    y = np.cos(theta)
    for i, j in [(0, 0), (3, 7), (9, 2), (5, 5)]:
        val = Ch.chebval2d(y[i], y[j], A)
        assert abs(val - f(np.array([[L * y[i], L * y[j]]]))[0]) < 1e-13


def test_converges_for_gaussian_wells():
    """Uniform error on random points of the cube falls quickly with R."""
    N, L = 3, 3.0
    f = _wells(N)
    rng = np.random.default_rng(4)
    pts = rng.uniform(-L, L, size=(200, N))
    errs = []
    for R in (6, 12, 18):
        rset = list(itertools.product(range(R + 1), repeat=N))
        a = cheb_interpolate(f, N, R, L, rset)
        vals = np.zeros(len(pts))
        for coef, r in zip(a, rset):
            vals += coef * np.prod([np.cos(r[l] * np.arccos(pts[:, l] / L)) for l in range(N)], axis=0)
        errs.append(np.max(np.abs(vals - f(pts))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6 and errs[2] < 1e-3 * errs[0]


def test_fast_operator_from_coefficients():
    """The Chebyshev-basis fast operator built from the interpolated coefficients of a
    polynomial W equals the one built from its monomials (a basis change leaves the
    operator unchanged)."""
    N, B, R, L = 3, 60, 3, 4.0
    rset = [r for r in itertools.product(range(R + 1), repeat=N)]
    a = cheb_interpolate(lambda x: _hh(x, L), N, R, L, rset)
    cheb = Potential(N, "cheb", L, [(c, r) for c, r in zip(a, rset) if abs(c) > 1e-15])
    mono = Potential(N, "mono", 1.0, [(1.0 / L ** 3, (2, 1, 0)), (-1.0 / (3 * L ** 3), (0, 3, 0)),
                                      (-0.3 / L, (0, 0, 1)), (0.2 / L ** 3, (1, 0, 2))])
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 9)
    y1, y2 = fast_apply_H(ix, cheb, c), fast_apply_H(ix, mono, c)
    assert np.linalg.norm(y1 - y2) < 1e-12 * np.linalg.norm(y2)


def test_total_degree_truncation_order():
    """Coefficients come back in the order of the requested set."""
    N, R, L = 2, 4, 2.0
    f = _wells(N)
    full = list(itertools.product(range(R + 1), repeat=N))
    a_full = dict(zip(full, cheb_interpolate(f, N, R, L, full)))
    td = total_degree_list(N, 4)
    a_td = cheb_interpolate(f, N, R, L, td)
    assert np.array_equal(a_td, np.array([a_full[tuple(r)] for r in td]))
    assert math.isfinite(float(np.sum(a_td)))


def test_compare_with_gauss_hermite_projection():
    """For the Gaussian wells and a packet near the origin, the Hermite projection
    (weight exp(-|x|^2)) gives a more accurate Galerkin action than the Chebyshev
    interpolant on a cube at the same total degree: the interpolant spends its accuracy
    uniformly over [-L, L]^N.  Reference: the exact Galerkin action by a 220-point product
    Gauss-Hermite rule on the Hermite functions."""
    from numpy.polynomial.hermite import hermgauss

    from oracle.operators import fast_apply_W, hermite_functions_scaled
    from oracle.surrogate import gh_project
    from synth import coherent_state
    N, B, D = 2, 32, 6
    f = _wells(N)
    ix = IndexSet(N, B)
    c = coherent_state(ix.k, [0.5, -0.3])
    c /= np.linalg.norm(c)
    x, w = hermgauss(220)
    psi = hermite_functions_scaled(int(ix.k.max()), x)
    X, Y = np.meshgrid(x, x, indexing="ij")
    Gw = f(np.stack([X.ravel(), Y.ravel()], -1)).reshape(x.size, x.size) * w[:, None] * w[None, :]
    A, Bm = psi[ix.k[:, 0]], psi[ix.k[:, 1]]
    y_ex = np.einsum("im,in,mn->i", A, Bm, Gw * np.einsum("jm,jn,j->mn", A, Bm, c))
    td = total_degree_list(N, D)
    herm = Potential(N, "herm", 1.0, list(zip(gh_project(f, N, D, 24), td)))
    e_gh = np.linalg.norm(fast_apply_W(ix, herm, c) - y_ex) / np.linalg.norm(y_ex)
    errs = {}
    for L in (3.0, 5.0):
        cheb = Potential(N, "cheb", L, list(zip(cheb_interpolate(f, N, D, L, td), td)))
        errs[L] = np.linalg.norm(fast_apply_W(ix, cheb, c) - y_ex) / np.linalg.norm(y_ex)
    print(f"relative error of W c: GH projection {e_gh:.2e}, Chebyshev L=3 {errs[3.0]:.2e}, L=5 {errs[5.0]:.2e}")
    assert e_gh < 0.05
    assert e_gh < errs[3.0] < errs[5.0] < 0.5
