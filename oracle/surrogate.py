"""Oracle: Gauss-Hermite projection of a smooth potential onto Hermite polynomials of
bounded total degree, Chebyshev interpolation of it on a cube, and a float64 multilayer
perceptron with manual backward and Adam.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Projection: for W(x) with the weight exp(-|x|^2) the L2-best coefficients on the
orthogonal family H_a(x) = prod_l H_{a_l}(x_l) are
    alpha_a = <W, H_a> / <H_a, H_a>,  <H_n, H_n> = sqrt(pi) 2^n n! (per axis),
and the inner product is evaluated with the product Gauss-Hermite rule of Sec. 4.1
(Q nodes per axis, the zeros of H_Q).

Potential family (the learned-coefficient workload):
    W(x, t) = - sum_i a_i exp(-|x - c_i(t)|^2 / (2 sigma^2)),
with c_i(t) on circles (centre, orthonormal plane vectors u_i, w_i, radius rho,
angular speed omega, phase phi_i).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .operators import gh_nodes_weights, poly_values


def total_degree_list(N: int, D: int):
    """All a in N_0^N with |a| <= D in lexicographic order."""
    return [a for a in itertools.product(range(D + 1), repeat=N) if sum(a) <= D]


def gaussian_sum_W(x: np.ndarray, amps, sigma: float, centres: np.ndarray) -> np.ndarray:
    """W(x) = -sum_i a_i exp(-|x - c_i|^2 / (2 sigma^2)) at points x (..., N)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape[:-1])
    for a, c in zip(amps, centres):
        d2 = np.sum((x - c) ** 2, axis=-1)
        out -= a * np.exp(-d2 / (2.0 * sigma * sigma))
    return out


def circle_centres(t: float, rho: float, omega: float, base, u, w, phase) -> np.ndarray:
    """c_i(t) = base_i + rho (cos(omega t + phi_i) u_i + sin(omega t + phi_i) w_i)."""
    base, u, w = (np.asarray(z, dtype=np.float64) for z in (base, u, w))
    ang = omega * t + np.asarray(phase, dtype=np.float64)
    return base + rho * (np.cos(ang)[:, None] * u + np.sin(ang)[:, None] * w)


def gh_project(Wvals_fn, N: int, D: int, Q: int) -> np.ndarray:
    """alpha_a for |a| <= D (order of total_degree_list) from a Q^N Gauss-Hermite grid.

    Wvals_fn(points) evaluates W at an array of points (Q^N, N).  The tensor grid sum is
    done axis by axis with a library contraction (tensordot); no other reordering."""
    xi, wt = gh_nodes_weights(Q - 1)
    grid = np.stack(np.meshgrid(*([xi] * N), indexing="ij"), axis=-1).reshape(-1, N)
    F = Wvals_fn(grid).reshape((Q,) * N)
    # 1-D factors  wt_m H_n(xi_m) / (sqrt(pi) 2^n n!)
    P = np.stack([wt * poly_values("herm", 1.0, n, xi) /
                  (math.sqrt(math.pi) * 2.0 ** n * math.factorial(n)) for n in range(D + 1)])
    T = F
    for _ in range(N):
        # contract the leading grid axis, append the degree axis at the end
        T = np.tensordot(T, P, axes=([0], [1]))
    return np.array([T[a] for a in total_degree_list(N, D)])


def cheb_interpolate(Wvals_fn, N: int, R: int, L: float, rset) -> np.ndarray:
    """Chebyshev interpolation of W on [-L, L]^N (Sec. 1.3): the tensor interpolant on the
    full grid of (R + 1)^N first-kind Chebyshev points x = L cos(theta_k),
    theta_k = (2k + 1) pi / (2 (R + 1)), in the basis T_r(x / L):
        alpha_r = prod_l (2 - [r_l = 0]) / (R + 1) * sum_k W(x_k) prod_l cos(r_l theta_{k_l}),
    returned for the multi-indices r in rset (r_l <= R).  Wvals_fn(points) evaluates W at
    an array of points (M, N).  The transform is taken axis by axis with a library
    contraction (tensordot)."""
    theta = (2 * np.arange(R + 1) + 1) * np.pi / (2 * (R + 1))
    x = L * np.cos(theta)
    grid = np.stack(np.meshgrid(*([x] * N), indexing="ij"), axis=-1).reshape(-1, N)
    F = Wvals_fn(grid).reshape((R + 1,) * N)
    C = np.stack([np.cos(r * theta) * ((1.0 if r == 0 else 2.0) / (R + 1)) for r in range(R + 1)])
    T = F
    for _ in range(N):
        T = np.tensordot(T, C, axes=([0], [1]))
    return np.array([T[tuple(r)] for r in rset])


def gaussian_hermite_moment_1d(n: int, c: float, s: float) -> float:
    """Closed form of int exp(-(x-c)^2/(2 s^2)) H_n(x) exp(-x^2) dx.

    From the generating function sum_n H_n(x) t^n / n! = exp(2 x t - t^2): the integral
    against it is a Gaussian integral equal to K0 exp(b t + d t^2) with
    p = 1 + 1/(2 s^2), b = c / (s^2 p), d = 1/p - 1,
    K0 = sqrt(pi/p) exp(c^2 / (4 s^4 p) - c^2 / (2 s^2)); the moment is n! [t^n]."""
    p = 1.0 + 1.0 / (2.0 * s * s)
    b = c / (s * s * p)
    d = 1.0 / p - 1.0
    K0 = math.sqrt(math.pi / p) * math.exp(c * c / (4.0 * s ** 4 * p) - c * c / (2.0 * s * s))
    acc = 0.0
    for j in range(n // 2 + 1):
        acc += b ** (n - 2 * j) / math.factorial(n - 2 * j) * d ** j / math.factorial(j)
    return K0 * math.factorial(n) * acc


def gaussian_sum_coeffs_exact(N: int, D: int, amps, sigma: float, centres) -> np.ndarray:
    """Exact Hermite coefficients of the Gaussian-sum W (closed form, no quadrature)."""
    out = []
    for a in total_degree_list(N, D):
        val = 0.0
        for amp, c in zip(amps, centres):
            prod = 1.0
            for l in range(N):
                prod *= gaussian_hermite_moment_1d(a[l], float(c[l]), sigma) / (
                    math.sqrt(math.pi) * 2.0 ** a[l] * math.factorial(a[l]))
            val -= amp * prod
        out.append(val)
    return np.array(out)


# ----------------------------------------------------------------------------------
# float64 MLP: in -> H -> H -> out with SiLU, MSE loss, Adam
# ----------------------------------------------------------------------------------


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def mlp_init(sizes, seed: int):
    """Weights W_i (out x in) ~ U(-1/sqrt(in), 1/sqrt(in)), biases 0."""
    rng = np.random.default_rng(seed)
    params = {}
    for i in range(len(sizes) - 1):
        bound = 1.0 / math.sqrt(sizes[i])
        params[f"W{i+1}"] = rng.uniform(-bound, bound, size=(sizes[i + 1], sizes[i]))
        params[f"b{i+1}"] = np.zeros(sizes[i + 1])
    return params


def mlp_forward(params, X):
    """Returns (output, cache).  X is (batch, in)."""
    z1 = X @ params["W1"].T + params["b1"]
    h1 = silu(z1)
    z2 = h1 @ params["W2"].T + params["b2"]
    h2 = silu(z2)
    y = h2 @ params["W3"].T + params["b3"]
    return y, (X, z1, h1, z2, h2)


def mse_loss(y, target):
    return float(np.mean((y - target) ** 2))


def mlp_backward(params, cache, y, target):
    """Gradients of mean((y - target)^2) over batch x outputs."""
    X, z1, h1, z2, h2 = cache
    n = y.size
    dy = 2.0 * (y - target) / n
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ params["W3"]
    dz2 = dh2 * silu_grad(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ params["W2"]
    dz1 = dh1 * silu_grad(z1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params
