"""Pins of the oracle's fourth-order two-stage Gauss-Legendre Magnus step (Sec. 2.1, eq.
2stageMagnus): it reduces to the midpoint step for a time-independent operator, is
exact with an exact exponential of a constant matrix, shows order four against an
independent ODE solution, and reproduces the time-discretisation entries of the paper's
time-integration table (Sec. 6.3, Fig. 13)."""
import math
import os

import numpy as np
from scipy.integrate import solve_ivp

from oracle.index import IndexSet
from oracle.operators import Potential, dense_H, fast_apply_H
from oracle.propagate import (GL2_NODES, dense_expm_apply, lanczos_expm, magnus4_operator,
                              magnus4_step, magnus_midpoint_step, propagate)
from synth import complex_normal_by_index, decay_vector, stretched_hh_cw_laser

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig13_time_errors.txt")


def _pot_at(N, tt):
    return lambda t: Potential(N, "mono", 1.0, [(x.coef(t), x.degrees) for x in tt])


def test_nodes_are_gauss_legendre():
    """c_{1,2} are the roots of the degree-2 Legendre polynomial moved to [0, 1]."""
    x, _ = np.polynomial.legendre.leggauss(2)
    assert np.allclose(sorted(GL2_NODES), 0.5 * (x + 1.0), atol=1e-15, rtol=0)


def test_time_independent_operator_reduces_to_midpoint_step():
    """A_1 = A_2: the commutator is exactly zero and M v = (A v + A v)/2 = A v bit for
    bit, so the step equals the midpoint step exactly."""
    N, B = 3, 40
    ix = IndexSet(N, B)
    W = Potential(N, "mono", 1.0, [(0.02, (2, 1, 0)), (-0.01, (0, 0, 3)), (0.05, (1, 0, 0))])
    c = complex_normal_by_index(ix.k, 11)
    c /= np.linalg.norm(c)
    fac = lambda pot: (lambda v: fast_apply_H(ix, pot, v))  # noqa: E731
    a, *_ = magnus4_step(ix, lambda t: W, fac, c, 0.3, 0.05, 9)
    b, *_ = magnus_midpoint_step(ix, lambda t: W, fac, c, 0.3, 0.05, 9)
    assert np.array_equal(a, b)


def test_exact_exponential_of_constant_matrix():
    """Full Krylov dimension on a 24 x 24 Hermitian matrix: exp(-i h A) c to rounding."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((24, 24)) + 1j * rng.standard_normal((24, 24))
    A = 0.5 * (X + X.conj().T)
    c = rng.standard_normal(24) + 1j * rng.standard_normal(24)
    M = magnus4_operator(lambda v: A @ v, lambda v: A @ v, 0.1)
    y, m_eff, _, _ = lanczos_expm(M, c, 0.1, 24)
    assert m_eff == 24
    assert np.linalg.norm(y - dense_expm_apply(A, c, 0.1)) < 1e-12 * np.linalg.norm(c)


def _dense_family(n, seed):
    rng = np.random.default_rng(seed)
    mats = []
    for _ in range(3):
        X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        mats.append(0.5 * (X + X.conj().T) / math.sqrt(n))
    H0, H1, H2 = mats
    return lambda t: H0 + math.sin(3.0 * t) * H1 + math.cos(t) * H2


def _order_errors(scheme, n=12, T=1.0):
    A = _dense_family(n, 9)
    rng = np.random.default_rng(10)
    c0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    c0 /= np.linalg.norm(c0)
    ref = solve_ivp(lambda t, y: -1j * (A(t) @ y), (0.0, T), c0, method="DOP853",
                    rtol=1e-13, atol=1e-15).y[:, -1]
    errs = []
    for nsteps in (8, 16, 32, 64):
        h = T / nsteps
        # full Krylov dimension with reorthogonalisation: the exponential is exact to
        # rounding, so only the Magnus scheme's own error remains
        c, _ = propagate(None, A, lambda M: (lambda v: M @ v), c0, 0.0, h, nsteps, n,
                         reorth=True, scheme=scheme)
        errs.append(np.linalg.norm(c - ref))
    return np.array(errs)


def test_order_four_against_ode_solution():
    """Observed orders log2(e(h)/e(h/2)) of the two-stage scheme approach 4 on a smooth
    time-dependent Hermitian family; the midpoint rule shows 2.  A dropped or
    sign-flipped commutator, or nodes other than the Gauss-Legendre pair, fall to
    order 2 and fail."""
    e4 = _order_errors(4)
    e2 = _order_errors(2)
    p4 = np.log2(e4[:-1] / e4[1:])
    p2 = np.log2(e2[:-1] / e2[1:])
    assert np.all(np.abs(p2 - 2.0) < 0.15), p2
    assert np.all(p4[1:] > 3.8) and np.all(p4 < 4.4), p4
    assert e4[-1] < 1e-7


def _load_golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        sch, N, m, K, inv_h, val, rtol = line.split()
        rows.append((int(sch), int(N), int(m), int(K), int(inv_h), float(val), float(rtol)))
    return rows


def test_fig13_time_discretisation_entries():
    """The time-integration table's entries dominated by the time-discretisation error:
    the oracle's fast-operator Lanczos propagation against the exact Galerkin solution
    (DOP853 on the dense matrices of the exact coordinate operators)."""
    rows = _load_golden()
    assert rows
    refs = {}
    for sch, N, m, K, inv_h, val, rtol in rows:
        ix = IndexSet(N, K + 1)
        tt = stretched_hh_cw_laser(N)
        pot_at = _pot_at(N, tt)
        c0 = decay_vector(ix.k, 3.0)
        c0 /= np.linalg.norm(c0)
        if (N, K) not in refs:
            H0 = dense_H(ix.k, pot_at(0.0))            # sin^2(0) = 0: no laser
            H1 = dense_H(ix.k, pot_at(0.5 * math.pi)) - H0   # the x_1 term at full strength
            f = lambda t, y: -1j * ((H0 + math.sin(t) ** 2 * H1) @ y)  # noqa: E731
            refs[(N, K)] = solve_ivp(f, (0.0, 1.0), c0, method="DOP853", rtol=1e-13,
                                     atol=1e-15).y[:, -1]
        c, _ = propagate(ix, pot_at, lambda pot: (lambda v: fast_apply_H(ix, pot, v)), c0, 0.0,
                         1.0 / inv_h, inv_h, m, reorth=False, scheme=sch)
        err = float(np.max(np.abs(c - refs[(N, K)])))
        print(f"scheme {sch} N={N} m={m} K={K} h=1/{inv_h}: {err:.3e} (paper {val:.3e})")
        assert abs(err - val) <= rtol * val
