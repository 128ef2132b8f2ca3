"""Oracle: Magnus steps with an m-step Lanczos approximation of the matrix exponential:
the exponential midpoint rule (Sec. 2.1 eq. expMPR) and the fourth-order two-stage
Gauss-Legendre Magnus scheme (Sec. 2.1 eq. 2stageMagnus); Sec. 2.2; Fig. 4
time_propagation.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings of points the paper leaves open (each is listed in the design doc):
  * the start vector is scaled by beta_0 = ||c^n|| instead of being assumed unit norm;
  * alpha_k := Re <v_k, w>: on a reduced set with coupling terms the fast operator is not
    exactly Hermitian, the tridiagonal T_m is kept real symmetric so exp(-i h T_m) is
    unitary;
  * one classical Gram-Schmidt pass against all previous Lanczos vectors (complex
    coefficients) after the three-term update, switchable off;
  * breakdown: stop at step k when beta_k <= 1e-12 * max(1, ||T_k||_inf) and use T_k.
"""
from __future__ import annotations

import numpy as np


def lanczos_expm(applyH, c: np.ndarray, h: float, m: int, reorth: bool = True,
                 breakdown_tol: float = 1e-12):
    """c_new ~= exp(-i h A) c with A applied through applyH (Sec. 2.2):
    V_m exp(-i h T_m) e_1 scaled by ||c||.  Returns (c_new, m_eff, alpha, beta)."""
    c = np.asarray(c, dtype=np.complex128)
    beta0 = np.linalg.norm(c)
    if beta0 == 0.0:
        return c.copy(), 0, np.zeros(0), np.zeros(0)
    V = [c / beta0]
    alpha, beta = [], []
    m_eff = m
    for k in range(m):
        w = applyH(V[k])
        if k > 0:
            w = w - beta[k - 1] * V[k - 1]
        a = np.real(np.vdot(V[k], w))
        alpha.append(a)
        w = w - a * V[k]
        if reorth:
            h_coef = [np.vdot(V[i], w) for i in range(k + 1)]
            for i in range(k + 1):
                w = w - h_coef[i] * V[i]
        b = np.linalg.norm(w)
        if k == m - 1:
            break
        # ||T_{k+1}||_inf with the coefficients found so far (row sums of |T|)
        rows = [abs(alpha[i]) + (beta[i - 1] if i >= 1 else 0.0) + (beta[i] if i < len(beta) else 0.0)
                for i in range(len(alpha))]
        if b <= breakdown_tol * max(1.0, max(rows)):
            m_eff = k + 1
            break
        beta.append(b)
        V.append(w / b)
    n = len(alpha)
    T = np.diag(alpha) + np.diag(beta[: n - 1], 1) + np.diag(beta[: n - 1], -1)
    lam, Q = np.linalg.eigh(T)
    y = beta0 * (Q @ (np.exp(-1j * h * lam) * Q[0, :]))
    out = np.zeros_like(c)
    for i in range(n):
        out += y[i] * V[i]
    return out, m_eff, np.array(alpha), np.array(beta[: n - 1])


def magnus_midpoint_step(idx, pot_at, applyH_factory, c, t, h, m, reorth=True):
    """One step of the exponential midpoint rule Omega^n = -i h A(t_n + h/2)
    (Sec. 2.1, eq. expMPR) with the Lanczos exponential.  pot_at(t) returns the
    potential at time t; applyH_factory(pot) returns a function v -> A v."""
    A = applyH_factory(pot_at(t + 0.5 * h))
    return lanczos_expm(A, c, h, m, reorth)


# Gauss-Legendre nodes of the two-stage scheme (Sec. 2.1 eq. 2stageMagnus)
GL2_NODES = (0.5 - np.sqrt(3.0) / 6.0, 0.5 + np.sqrt(3.0) / 6.0)


def magnus4_operator(applyA1, applyA2, h):
    """The Hermitian M with Omega^n = -i h M for the two-stage scheme (Sec. 2.1, eq.
    2stageMagnus).  Omega^n = -(i/2) h (A_1 + A_2) - (sqrt(3)/12) h^2 [A_2, A_1]; dividing
    by -i h gives M = (A_1 + A_2)/2 - i (sqrt(3) h / 12) (A_2 A_1 - A_1 A_2), applied to a
    vector with four operator products (A_1 v, A_2 v, A_2 A_1 v, A_1 A_2 v)."""
    g = np.sqrt(3.0) * h / 12.0

    def M(v):
        u1 = applyA1(v)
        u2 = applyA2(v)
        comm = applyA2(u1) - applyA1(u2)
        return 0.5 * (u1 + u2) - 1j * g * comm

    return M


def magnus4_step(idx, pot_at, applyH_factory, c, t, h, m, reorth=True):
    """One step of the two-stage Gauss-Legendre Magnus scheme (Sec. 2.1, eq.
    2stageMagnus): A_j = A(t_n + c_j h) with c_{1,2} = 1/2 -+ sqrt(3)/6, and
    exp(-i h M) c by the Lanczos method of Sec. 2.2."""
    A1 = applyH_factory(pot_at(t + GL2_NODES[0] * h))
    A2 = applyH_factory(pot_at(t + GL2_NODES[1] * h))
    return lanczos_expm(magnus4_operator(A1, A2, h), c, h, m, reorth)


def propagate(idx, pot_at, applyH_factory, c0, t0, h, nsteps, m, reorth=True, scheme=2):
    """time_propagation of Fig. 4: nsteps Magnus-Lanczos steps of the exponential
    midpoint rule (scheme 2) or of the two-stage Gauss-Legendre scheme (scheme 4)."""
    if scheme not in (2, 4):
        raise ValueError("scheme must be 2 or 4")
    one = magnus_midpoint_step if scheme == 2 else magnus4_step
    c = np.asarray(c0, dtype=np.complex128).copy()
    t = t0
    m_effs = []
    for _ in range(nsteps):
        c, me, _, _ = one(idx, pot_at, applyH_factory, c, t, h, m, reorth)
        m_effs.append(me)
        t += h
    return c, m_effs


def dense_expm_apply(H: np.ndarray, c: np.ndarray, h: float) -> np.ndarray:
    """exp(-i h H) c for a Hermitian dense matrix via its eigendecomposition (tiny sets)."""
    Hs = 0.5 * (H + H.conj().T)
    lam, U = np.linalg.eigh(Hs)
    return U @ (np.exp(-1j * h * lam) * (U.conj().T @ c))
