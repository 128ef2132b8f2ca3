"""Oracle: exponential-midpoint Magnus step with an m-step Lanczos approximation of the
matrix exponential (Sec. 2.1 eq. expMPR, Sec. 2.2, Fig. 4 time_propagation).

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


def propagate(idx, pot_at, applyH_factory, c0, t0, h, nsteps, m, reorth=True):
    """time_propagation of Fig. 4: nsteps exponential-midpoint Lanczos steps."""
    c = np.asarray(c0, dtype=np.complex128).copy()
    t = t0
    m_effs = []
    for _ in range(nsteps):
        c, me, _, _ = magnus_midpoint_step(idx, pot_at, applyH_factory, c, t, h, m, reorth)
        m_effs.append(me)
        t += h
    return c, m_effs


def dense_expm_apply(H: np.ndarray, c: np.ndarray, h: float) -> np.ndarray:
    """exp(-i h H) c for a Hermitian dense matrix via its eigendecomposition (tiny sets)."""
    Hs = 0.5 * (H + H.conj().T)
    lam, U = np.linalg.eigh(Hs)
    return U @ (np.exp(-1j * h * lam) * (U.conj().T @ c))
