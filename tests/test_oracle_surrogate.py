"""Pins of the surrogate oracle: Gauss-Hermite projection against polynomial exactness
and closed-form Gaussian moments, and the float64 MLP against finite differences."""
import math

import numpy as np
import pytest

from oracle.operators import poly_values
from oracle.surrogate import (adam_step, circle_centres, gaussian_hermite_moment_1d,
                              gaussian_sum_W, gaussian_sum_coeffs_exact, gh_project,
                              mlp_backward, mlp_forward, mlp_init, mse_loss,
                              total_degree_list)
from synth import surrogate_geometry


def test_total_degree_count():
    assert len(total_degree_list(4, 6)) == math.comb(10, 4) == 210
    assert len(total_degree_list(3, 2)) == 10


def test_projection_exact_for_polynomials():
    """A polynomial of total degree <= 6 in the Hermite basis is recovered exactly by a
    product rule with Q >= 7 nodes (the integrand has degree <= 12 per axis... <= 2Q-1)."""
    N, D = 3, 6
    alist = total_degree_list(N, D)
    rng = np.random.default_rng(1)
    coef = rng.standard_normal(len(alist))

    def Wf(x):
        out = np.zeros(x.shape[0])
        for c, a in zip(coef, alist):
            term = np.full(x.shape[0], c)
            for l in range(N):
                term *= poly_values("herm", 1.0, a[l], x[:, l])
            out += term
        return out

    got = gh_project(Wf, N, D, 7)
    assert np.allclose(got, coef, atol=1e-11)
    # with too few nodes it is not exact
    assert np.max(np.abs(gh_project(Wf, N, D, 5) - coef)) > 1e-3


def test_gaussian_moment_closed_form_vs_quadrature():
    """The generating-function moments agree with a fine Gauss-Hermite quadrature."""
    x, w = np.polynomial.hermite.hermgauss(120)
    for n in range(7):
        for c, s in ((0.3, 0.9), (-0.7, 1.4)):
            ref = np.sum(w * np.exp(-(x - c) ** 2 / (2 * s * s)) * poly_values("herm", 1.0, n, x))
            assert gaussian_hermite_moment_1d(n, c, s) == pytest.approx(ref, rel=1e-11, abs=1e-13)


def test_projection_of_gaussian_sum_converges():
    N, D = 4, 6
    geo = surrogate_geometry(N)
    amps, sigma = [1.2, 0.7, 1.9], 1.1
    cen = circle_centres(0.4, 0.6, 1.3, geo["base"], geo["u"], geo["w"], geo["phase"])
    exact = gaussian_sum_coeffs_exact(N, D, amps, sigma, cen)
    fine = gh_project(lambda x: gaussian_sum_W(x, amps, sigma, cen), N, D, 30)
    assert np.max(np.abs(fine - exact)) < 1e-12
    q16 = gh_project(lambda x: gaussian_sum_W(x, amps, sigma, cen), N, D, 16)
    assert np.max(np.abs(q16 - exact)) < 1e-6


def test_mlp_backward_matches_finite_differences():
    sizes = [7, 16, 16, 5]
    params = mlp_init(sizes, 0)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((9, 7))
    T = rng.standard_normal((9, 5))
    y, cache = mlp_forward(params, X)
    g = mlp_backward(params, cache, y, T)
    eps = 1e-6
    for name in params:
        P = params[name]
        flat = P.reshape(-1)
        for i in rng.choice(flat.size, min(6, flat.size), replace=False):
            old = flat[i]
            flat[i] = old + eps
            lp = mse_loss(mlp_forward(params, X)[0], T)
            flat[i] = old - eps
            lm = mse_loss(mlp_forward(params, X)[0], T)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            assert g[name].reshape(-1)[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_adam_first_step_closed_form():
    """First Adam step with bias correction moves each weight by -lr g / (|g| + eps)."""
    params = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -0.01, 0.0])}
    out = adam_step(dict(params), g, {}, lr=0.1)
    ref = params["w"] - 0.1 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(out["w"], ref, atol=1e-12)
