"""Workload descriptions and seeded random inputs.

Every random draw is made in the canonical lexicographic order of the multi-indices
that the caller passes in, so the same seed gives the same value at the same
multi-index on both sides, whatever order a side stores its vector in.

Potentials are written as term lists of the physical potential V in the monomial basis:
a list of (coef, degrees) pairs plus optional time dependence
    coef(t) = base + amp * sin(freq * t + phase).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "TimeTerm", "henon_heiles_chain", "stretched_hh_cw_laser", "torsional_series", "lex_order",
    "random_downward_set",
    "complex_normal_by_index", "coherent_state", "decay_vector",
    "batch_instances", "surrogate_geometry", "surrogate_param_box",
    "draw_surrogate_params", "mlp_initial_weights",
]


class TimeTerm(tuple):
    """(base, amp, freq, phase, degrees) of a term base + amp sin(freq t + phase)."""

    def __new__(cls, base, degrees, amp=0.0, freq=0.0, phase=0.0):
        return super().__new__(cls, (float(base), float(amp), float(freq), float(phase),
                                     tuple(int(d) for d in degrees)))

    @property
    def degrees(self):
        return self[4]

    def coef(self, t: float) -> float:
        base, amp, freq, phase, _ = self
        return base + amp * math.sin(freq * t + phase)


def _deg(N, pairs):
    a = [0] * N
    for l, p in pairs:
        a[l] += p
    return tuple(a)


def henon_heiles_chain(N: int, lam: float = 0.111, laser: float = 0.0,
                       laser_freq: float = 2.0, harmonic: bool = True):
    """V = 1/2 |x|^2 + lam sum_{l<N} (x_l^2 x_{l+1} - x_{l+1}^3 / 3)
           + laser sin(laser_freq t) sum_d x_d   (laser term omitted when laser == 0).

    N = 2 gives the classical Henon-Heiles potential."""
    terms = []
    if harmonic:
        for l in range(N):
            terms.append(TimeTerm(0.5, _deg(N, [(l, 2)])))
    for l in range(N - 1):
        terms.append(TimeTerm(lam, _deg(N, [(l, 2), (l + 1, 1)])))
        terms.append(TimeTerm(-lam / 3.0, _deg(N, [(l + 1, 3)])))
    if laser != 0.0:
        for d in range(N):
            terms.append(TimeTerm(0.0, _deg(N, [(d, 1)]), amp=laser, freq=laser_freq))
    return terms


def stretched_hh_cw_laser(N: int, L: float = 16.0):
    """The potential of the paper's time-integration study (Sec. 6, eq.
    HenonHeilesExperiments), in the reading that reproduces its error table:
        W(x, t) = sum_{l<N} [(x_l/L)^2 (x_{l+1}/L) - (x_{l+1}/L)^3 / 3] - sin^2(t) x_1 / L,
    with no harmonic term (W is the potential beyond the oscillator).  The laser factor
    -sin^2(t) / L is written as -1/(2L) + 1/(2L) sin(2t + pi/2)."""
    terms = []
    for l in range(N - 1):
        terms.append(TimeTerm(1.0 / L ** 3, _deg(N, [(l, 2), (l + 1, 1)])))
        terms.append(TimeTerm(-1.0 / (3.0 * L ** 3), _deg(N, [(l + 1, 3)])))
    terms.append(TimeTerm(-0.5 / L, _deg(N, [(0, 1)]), amp=0.5 / L, freq=2.0, phase=0.5 * math.pi))
    return terms


def torsional_series(N: int, L: float = 16.0, R: int = 8):
    """The torsional potential W = sum_l (1 - cos(x_l / L)) written in the Chebyshev basis
    T_r(x_l / L) up to degree R, with the closed-form (Jacobi-Anger) coefficients
        1 - cos(y) = 1 - J_0(1) - 2 sum_{k >= 1} (-1)^k J_{2k}(1) T_{2k}(y)
    truncated at degree R (the neglected tail is below |J_{R+2}(1)|, 2.6e-10 for R = 8).
    Returns (coef, degrees) pairs; the N constant terms are merged."""
    from scipy.special import jv
    terms = [(N * (1.0 - jv(0, 1.0)), (0,) * N)]
    for l in range(N):
        for r in range(2, R + 1, 2):
            a = [0] * N
            a[l] = r
            terms.append((-2.0 * (-1.0) ** (r // 2) * jv(r, 1.0), tuple(a)))
    return terms


def random_downward_set(N: int, npoints: int, maxc: int, seed: int) -> np.ndarray:
    """A seeded downward-closed set: the union of the boxes below npoints random corners
    (coordinates uniform in 0..maxc), rows in lexicographic order, shape (n, N)."""
    rng = np.random.default_rng(seed)
    corners = rng.integers(0, maxc + 1, size=(npoints, N))
    rows = set()
    for c in corners:
        for k in np.ndindex(*(int(x) + 1 for x in c)):
            rows.add(k)
    out = np.array(sorted(rows), dtype=np.int64).reshape(-1, N)
    return out


def lex_order(k: np.ndarray) -> np.ndarray:
    """Permutation that sorts multi-index rows lexicographically (k_1 slowest)."""
    k = np.asarray(k)
    return np.lexsort(k.T[::-1])


def complex_normal_by_index(k: np.ndarray, seed: int) -> np.ndarray:
    """c_k with independent N(0,1) real and imaginary parts, drawn in lex order of k
    (numpy default_rng(seed), reals first then imaginaries) and placed by multi-index."""
    k = np.asarray(k)
    order = lex_order(k)
    rng = np.random.default_rng(seed)
    n = k.shape[0]
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    out = np.empty(n, dtype=np.complex128)
    out[order] = re + 1j * im
    return out


def coherent_state(k: np.ndarray, x0) -> np.ndarray:
    """Hermite coefficients of the displaced harmonic-oscillator ground state
    pi^(-N/4) exp(-|x - x0|^2 / 2): c_k = prod_l exp(-x0_l^2/4) (x0_l/sqrt 2)^k_l / sqrt(k_l!)
    (unnormalised on a truncated set)."""
    k = np.asarray(k, dtype=np.int64)
    N = k.shape[1]
    x0 = np.broadcast_to(np.asarray(x0, dtype=np.float64), (N,))
    logc = np.zeros(k.shape[0])
    sign = np.ones(k.shape[0])
    from scipy.special import gammaln
    for l in range(N):
        kl = k[:, l]
        logc += -x0[l] ** 2 / 4.0 - 0.5 * gammaln(kl + 1.0)
        if x0[l] != 0.0:
            logc += kl * math.log(abs(x0[l]) / math.sqrt(2.0))
            if x0[l] < 0:
                sign *= np.where(kl % 2 == 1, -1.0, 1.0)
        else:
            logc = np.where(kl > 0, -np.inf, logc)
    return (sign * np.exp(logc)).astype(np.complex128)


def decay_vector(k: np.ndarray, beta: float) -> np.ndarray:
    """v_k = prod_l max(k_l, 1)^(-beta) (decay model of the paper's local-error study)."""
    k = np.asarray(k, dtype=np.float64)
    return np.prod(np.maximum(k, 1.0) ** (-beta), axis=1).astype(np.complex128)


def batch_instances(n: int, seed: int, nmin: int = 3, nmax: int = 8,
                    log2_bmin: float = 8.0, log2_bmax: float = 14.0,
                    lam_lo: float = 0.05, lam_hi: float = 0.15, accept=None):
    """Instance draws of the batched workload: N ~ U{nmin..nmax},
    B = floor(2^U(log2_bmin, log2_bmax)), lambda ~ U[lam_lo, lam_hi].

    accept(N, B) -> bool, if given, is a size rule: an instance it rejects is drawn
    again (all three values, from the same stream) until one is accepted."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        while True:
            N = int(rng.integers(nmin, nmax + 1))
            B = int(math.floor(2.0 ** rng.uniform(log2_bmin, log2_bmax)))
            lam = float(rng.uniform(lam_lo, lam_hi))
            if accept is None or accept(N, B):
                break
        out.append({"N": N, "B": B, "lam": lam, "seed": 1000 + i})
    return out


def surrogate_geometry(N: int = 4, n_gauss: int = 3, seed: int = 7):
    """Fixed circle geometry of the Gaussian wells: centres in [-0.5, 0.5]^N, a random
    orthonormal plane (u_i, w_i) per well and a phase per well."""
    rng = np.random.default_rng(seed)
    base = rng.uniform(-0.5, 0.5, size=(n_gauss, N))
    u = np.empty((n_gauss, N))
    w = np.empty((n_gauss, N))
    for i in range(n_gauss):
        q, _ = np.linalg.qr(rng.standard_normal((N, 2)))
        u[i], w[i] = q[:, 0], q[:, 1]
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_gauss)
    return {"base": base, "u": u, "w": w, "phase": phase}


def surrogate_param_box():
    """Box of the 7 inputs (t, a1, a2, a3, sigma, rho, omega)."""
    lo = np.array([0.0, 0.5, 0.5, 0.5, 0.8, 0.2, 0.5])
    hi = np.array([2.0 * math.pi, 2.0, 2.0, 2.0, 1.5, 1.0, 2.0])
    return lo, hi


def draw_surrogate_params(n: int, seed: int) -> np.ndarray:
    """n uniform draws from the parameter box, shape (n, 7)."""
    lo, hi = surrogate_param_box()
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.uniform(size=(n, 7))


def mlp_initial_weights(sizes, seed: int):
    """Seeded initial weights of a dense network: W_i (fan_out x fan_in) uniform in
    +-1/sqrt(fan_in), biases zero (keys W1, b1, W2, ...)."""
    rng = np.random.default_rng(seed)
    out = {}
    for i in range(len(sizes) - 1):
        bound = 1.0 / math.sqrt(sizes[i])
        out[f"W{i + 1}"] = rng.uniform(-bound, bound, size=(sizes[i + 1], sizes[i]))
        out[f"b{i + 1}"] = np.zeros(sizes[i + 1])
    return out
