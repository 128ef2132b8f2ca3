"""Oracle: coordinate operators, the fast algorithm, the exact Galerkin matrix, product
Gauss-Hermite quadrature and the quadrature / index-reduction error split.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Notation follows the paper: phi_k are the Hermite functions (Sec. 1.1), X^(l) the
coordinate matrices over an index set (Sec. 3.1), D the harmonic-oscillator diagonal
and W = V - |x|^2 / 2 the remaining potential (Sec. 1.2), W^pol its polynomial
approximation written in a per-axis three-term-recurrence basis (Sec. 1.3).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------------
# Potentials
# ----------------------------------------------------------------------------------

BASES = ("mono", "cheb", "herm")


@dataclass
class Potential:
    """W^pol = sum_t coef_t prod_l p_{a_{t,l}}(x_l) in one per-axis polynomial family.

    basis 'mono': p_a(x) = x^a.
    basis 'cheb': p_a(x) = T_a(x / scale), Chebyshev polynomials of the first kind
                  (Sec. 1.3, eq. ChebyshevRecurrence, scale = L).
    basis 'herm': p_a(x) = H_a(x / scale), physicists' Hermite polynomials.
    terms: list of (coef, degrees) with degrees a tuple of N non-negative ints.
    """

    N: int
    basis: str = "mono"
    scale: float = 1.0
    terms: list = field(default_factory=list)

    def __post_init__(self):
        if self.basis not in BASES:
            raise ValueError(self.basis)
        for c, a in self.terms:
            if len(a) != self.N:
                raise ValueError("degree tuple length != N")

    def max_degree(self) -> int:
        return max((max(a) for _, a in self.terms), default=0)


def recurrence_coeffs(basis: str, scale: float, k: int):
    """(A_k, B_k, C_k) of p_{k+1}(x) = (A_k x + B_k) p_k(x) - C_k p_{k-1}(x), p_0 = 1.

    Chebyshev: T_1 = y, T_{k+1} = 2 y T_k - T_{k-1} with y = x / L (Sec. 1.3).
    Hermite (physicists'): H_1 = 2 y, H_{k+1} = 2 y H_k - 2 k H_{k-1}.
    Monomials: x^{k+1} = x * x^k."""
    if basis == "mono":
        return 1.0, 0.0, 0.0
    if basis == "cheb":
        return (1.0 / scale if k == 0 else 2.0 / scale), 0.0, (0.0 if k == 0 else 1.0)
    if basis == "herm":
        return 2.0 / scale, 0.0, 2.0 * k
    raise ValueError(basis)


def poly_values(basis: str, scale: float, a: int, x: np.ndarray) -> np.ndarray:
    """p_a(x) by the same recurrence, for scalar arguments."""
    x = np.asarray(x, dtype=np.float64)
    pm, p = np.zeros_like(x), np.ones_like(x)
    for k in range(a):
        A, Bc, C = recurrence_coeffs(basis, scale, k)
        pm, p = p, (A * x + Bc) * p - C * pm
    return p


def subtract_harmonic(pot: Potential) -> Potential:
    """W = V - (1/2) sum_l x_l^2 (Sec. 1.2, definition of W).

    Only for a monomial-basis V: the coefficient of each x_l^2 monomial drops by 1/2
    (a missing x_l^2 term is added with coefficient -1/2)."""
    if pot.basis != "mono":
        raise ValueError("subtract_harmonic expects a monomial-basis potential")
    terms = {}
    for c, a in pot.terms:
        terms[tuple(a)] = terms.get(tuple(a), 0.0) + c
    for l in range(pot.N):
        a = [0] * pot.N
        a[l] = 2
        terms[tuple(a)] = terms.get(tuple(a), 0.0) - 0.5
    return Potential(pot.N, "mono", 1.0, [(c, a) for a, c in terms.items() if c != 0])


# ----------------------------------------------------------------------------------
# Direct operation with X^(l) and the fast algorithm (Sec. 3, Fig. 3)
# ----------------------------------------------------------------------------------


def direct_op(idx, l: int, v: np.ndarray) -> np.ndarray:
    """(X^(l) v)_j = sqrt(j_l / 2) v_{j - e_l} + sqrt((j_l + 1) / 2) v_{j + e_l}.

    Sec. 3.1, eq. DirectOperationWithX.  A neighbour outside the index set contributes
    nothing (Galerkin truncation: X^(l) is indexed over the set only)."""
    jl = idx.k[:, l].astype(np.float64)
    out = np.zeros_like(v)
    m = idx.nbr_minus[l]
    p = idx.nbr_plus[l]
    hm = m >= 0
    hp = p >= 0
    out[hm] += np.sqrt(jl[hm] / 2.0) * v[m[hm]]
    out[hp] += np.sqrt((jl[hp] + 1.0) / 2.0) * v[p[hp]]
    return out


def apply_axis_poly(idx, l: int, basis: str, scale: float, a: int, v: np.ndarray) -> np.ndarray:
    """p_a(X^(l)) v by the three-term recurrence with the direct operation in place of x.

    For the Chebyshev basis this is exactly the inner loop of the fast algorithm of
    Fig. 3: w_- = v, w_+ = (1/L) X v, then w_+ <- (2/L) X w_+ - w_-."""
    if a == 0:
        return v.copy()
    wm = v
    A, Bc, C = recurrence_coeffs(basis, scale, 0)
    wp = A * direct_op(idx, l, v) + Bc * v
    for k in range(1, a):
        A, Bc, C = recurrence_coeffs(basis, scale, k)
        nxt = A * direct_op(idx, l, wp) + Bc * wp - C * wm
        wm, wp = wp, nxt
    return wp


def fast_apply_W(idx, pot: Potential, v: np.ndarray, axis_order: str = "eq") -> np.ndarray:
    """W^pol(X_K) v by formal insertion of the coordinate matrices (Sec. 3.2, eq. Horner).

    Each term restarts from the input vector.  axis_order 'eq' applies axis N first and
    axis 1 last, as the nested product of eq. Horner is written; 'rev' applies axis 1
    first (the adjoint identity, and the symmetrised operator sym_apply_H)."""
    v = np.asarray(v, dtype=np.complex128)
    res = np.zeros_like(v)
    axes = range(pot.N - 1, -1, -1) if axis_order == "eq" else range(pot.N)
    for coef, a in pot.terms:
        u = v
        for l in axes:
            if a[l] > 0:
                u = apply_axis_poly(idx, l, pot.basis, pot.scale, a[l], u)
        res += coef * u
    return res


def diag_D(idx) -> np.ndarray:
    """D_jj = sum_l (j_l + 1/2), the harmonic-oscillator part (Sec. 1.1, eq.
    HermiteEigenfunctions1D / EigenfunctionRelation)."""
    return np.sum(idx.k.astype(np.float64), axis=1) + 0.5 * idx.k.shape[1]


def fast_apply_H(idx, pot: Potential, v: np.ndarray, axis_order: str = "eq") -> np.ndarray:
    """(D + W^pol(X_K)) v, the action used in each Lanczos step (Fig. 4, step (2))."""
    v = np.asarray(v, dtype=np.complex128)
    return diag_D(idx) * v + fast_apply_W(idx, pot, v, axis_order)


def sym_apply_H(idx, pot: Potential, v: np.ndarray) -> np.ndarray:
    """(D + (F + F_rev)/2) v: the Hermitian part of the fast operator.

    On a reduced set the truncated coordinate matrices do not commute, so the order of
    the factors in eq. Horner matters there (Sec. 4.2, discussion after Lemma 1; on the
    full set it does not).  Each X^(l)_K is real symmetric, so the transpose of a term
    p(X^(1))...p(X^(N)) (axis N applied first) is the same product applied in the reverse
    order: F^T = F_rev, and (F + F_rev)/2 is the symmetric part of F.  It agrees with F
    on every term that touches a single axis, and on a full box."""
    v = np.asarray(v, dtype=np.complex128)
    return diag_D(idx) * v + 0.5 * (fast_apply_W(idx, pot, v, "eq") + fast_apply_W(idx, pot, v, "rev"))


# ----------------------------------------------------------------------------------
# Exact Galerkin matrix on tiny sets (the plain definition)
# ----------------------------------------------------------------------------------


def jacobi_matrix(P: int) -> np.ndarray:
    """(P+1) x (P+1) matrix of x in the basis phi_0..phi_P: entries sqrt((i+1)/2) on the
    first off-diagonals, from the recurrence x phi_k = sqrt((k+1)/2) phi_{k+1} +
    sqrt(k/2) phi_{k-1} (Sec. 1.1, eq. Recurrence1D)."""
    off = np.sqrt(np.arange(1, P + 1) / 2.0)
    return np.diag(off, 1) + np.diag(off, -1)


def exact_1d(basis: str, scale: float, a: int, kmax: int) -> np.ndarray:
    """Q[i, k] = (phi_i, p_a(x) phi_k) for 0 <= i, k <= kmax, exactly (up to rounding).

    p_a of a Jacobi matrix padded to size kmax + a + 1: a path of length a between two
    indices <= kmax never leaves [0, kmax + a], so the padding makes the entries exact."""
    P = kmax + a + 1
    J = jacobi_matrix(P)
    pm, p = np.zeros_like(J), np.eye(P + 1)
    for k in range(a):
        A, Bc, C = recurrence_coeffs(basis, scale, k)
        pm, p = p, A * (J @ p) + Bc * p - C * pm
    return p[: kmax + 1, : kmax + 1]


def assemble_from_1d(k: np.ndarray, pot: Potential, one_d) -> np.ndarray:
    """M_jk = sum_t coef_t prod_l G^{(l, a_tl)}[j_l, k_l] over rows j, columns k of the
    multi-index array k.  Tensor-product orthonormality (Sec. 1.1) makes this the
    Galerkin matrix when G are the exact 1-D matrices."""
    k = k.astype(np.int64)
    n = k.shape[0]
    M = np.zeros((n, n), dtype=np.complex128)
    cache = {}
    for coef, a in pot.terms:
        T = np.ones((n, n), dtype=np.float64)
        for l in range(pot.N):
            key = a[l]
            if key not in cache:
                cache[key] = one_d(a[l])
            G = cache[key]
            T *= G[np.ix_(k[:, l], k[:, l])]
        M += coef * T
    return M


def dense_W(k: np.ndarray, pot: Potential) -> np.ndarray:
    """The exact Galerkin matrix (phi_j, W^pol phi_k) over the rows of k (tiny sets)."""
    kmax = int(k.max()) if k.size else 0
    return assemble_from_1d(k, pot, lambda a: exact_1d(pot.basis, pot.scale, a, kmax))


def dense_H(k: np.ndarray, pot: Potential) -> np.ndarray:
    """D + (phi_j, W^pol phi_k): the Galerkin matrix of -Delta/2 + V (Sec. 1.2)."""
    D = np.sum(k.astype(np.float64), axis=1) + 0.5 * k.shape[1]
    return np.diag(D).astype(np.complex128) + dense_W(k, pot)


# ----------------------------------------------------------------------------------
# Product Gauss-Hermite quadrature (Sec. 4.1) and the error split (Sec. 5.1)
# ----------------------------------------------------------------------------------


def gh_nodes_weights(M: int):
    """Zeros xi_m of H_{M+1} and weights w_m for the weight exp(-x^2) (Sec. 4.1).
    The library routine numpy.polynomial.hermite.hermgauss serves as this step."""
    return np.polynomial.hermite.hermgauss(M + 1)


def hermite_functions_scaled(kmax: int, x: np.ndarray) -> np.ndarray:
    """psi_k(x) = phi_k(x) exp(x^2 / 2) for k = 0..kmax, by the recurrence of Sec. 1.1
    started from psi_0 = pi^(-1/4).  Shape (kmax + 1, len(x))."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((kmax + 1, x.size))
    out[0] = np.pi ** -0.25
    if kmax >= 1:
        out[1] = x * out[0] / np.sqrt(0.5)
    for k in range(1, kmax):
        out[k + 1] = (x * out[k] - np.sqrt(k / 2.0) * out[k - 1]) / np.sqrt((k + 1) / 2.0)
    return out


def gh_1d(basis: str, scale: float, a: int, kmax: int, M: int) -> np.ndarray:
    """G[i, k] = sum_m omega_m phi_i(xi_m) p_a(xi_m) phi_k(xi_m), omega_m = w_m e^{xi_m^2}
    (Sec. 4.1, eq. GHQuad_full, the starred 1-D factor)."""
    xi, w = gh_nodes_weights(M)
    psi = hermite_functions_scaled(kmax, xi)
    pa = poly_values(basis, scale, a, xi)
    return (psi * (w * pa)) @ psi.T


def gh_W(k: np.ndarray, pot: Potential, M: int) -> np.ndarray:
    """Assembled W^{GH(M)} over the rows of k (Sec. 4.1)."""
    kmax = int(k.max()) if k.size else 0
    return assemble_from_1d(k, pot, lambda a: gh_1d(pot.basis, pot.scale, a, kmax, M))


def restrict_full(box_idx, set_k: np.ndarray, w_box: np.ndarray) -> np.ndarray:
    """Omega: entries of a box vector at the indices of the reduced set (Sec. 5.1)."""
    return w_box[box_idx.rank(set_k.astype(np.int64))]


def extend_zero(box_idx, set_k: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Omega_+: blow a reduced-set vector up to the box with zeros (Sec. 5.1)."""
    out = np.zeros(box_idx.size, dtype=np.complex128)
    out[box_idx.rank(set_k.astype(np.int64))] = v
    return out


def error_split(idx, box_idx, pot: Potential, v: np.ndarray, exact_Wv: np.ndarray):
    """(E^quad v, E^red(v)) as defined in Sec. 5.1 (eqs. ErrorQuadratureDef,
    ErrorGridReductionDef), with W^{GH(K)} on the set obtained through Lemma 1 as the
    restriction of the fast algorithm on the full box.

    exact_Wv is W_{K,pol} v, the exact Galerkin product."""
    gh_v = restrict_full(box_idx, idx.k, fast_apply_W(box_idx, pot, extend_zero(box_idx, idx.k, v)))
    fast_v = fast_apply_W(idx, pot, v)
    return exact_Wv - gh_v, fast_v - gh_v


def exact_W_separable(idx, pot: Potential, v: np.ndarray) -> np.ndarray:
    """W_{K,pol} v for a potential whose every term involves one axis at most, without
    assembling the matrix: along each axis-l fibre of the set the exact 1-D matrix
    (phi_i, p_a phi_k) acts on the fibre's entries (tensor-product orthonormality)."""
    v = np.asarray(v, dtype=np.complex128)
    out = np.zeros_like(v)
    kmax = int(idx.k.max())
    for coef, a in pot.terms:
        ax = [l for l in range(pot.N) if a[l] > 0]
        if len(ax) > 1:
            raise ValueError("exact_W_separable: term couples several axes")
        if not ax:
            out += coef * v
            continue
        l = ax[0]
        Q = exact_1d(pot.basis, pot.scale, a[l], kmax)
        acc = np.zeros_like(v)
        jl = idx.k[:, l].astype(np.int64)
        # walk along the fibre in both directions
        for direction, nbr in ((1, idx.nbr_plus[l]), (-1, idx.nbr_minus[l])):
            cur = np.arange(idx.size)
            steps = 0
            if direction == 1:
                acc += Q[jl, jl] * v
            while True:
                steps += 1
                nxt = np.where(cur >= 0, nbr[np.maximum(cur, 0)], -1)
                ok = nxt >= 0
                if not ok.any() or steps > a[l]:
                    break
                acc[ok] += Q[jl[ok], jl[ok] + direction * steps] * v[nxt[ok]]
                cur = nxt
        out += coef * acc
    return out


# ----------------------------------------------------------------------------------
# Row-wise evaluation for sampled rows of very large sets (layered trees, Sec. 5.3)
# ----------------------------------------------------------------------------------


def _fibre_top(m: tuple, l: int, B: int) -> int:
    rest = 1
    for i, mi in enumerate(m):
        if i != l:
            rest *= 1 + mi
    return B // rest - 1


def fast_H_rows(N: int, B: int, pot: Potential, lookup, rows) -> np.ndarray:
    """(D c + W^pol(X_K) c)_j for the multi-indices j in rows, one row at a time.

    The value of a term at j is expanded as the layered tree of Sec. 5.3 (Figs. 7, 8):
    axis 1 at the root, axis N at the leaves.  At layer l the axis-l polynomial acts
    on a window of radius a_l around j_l inside the fibre [0, top], using the Jacobi
    matrix restricted to that fibre, so truncation at the fibre top is honoured exactly
    as in the direct operation.  lookup(multi_index_tuple) returns c at that index.
    """

    def term_value(m, l, a):
        if l == N:
            return lookup(m)
        al = a[l]
        if al == 0:
            return term_value(m, l + 1, a)
        top = _fibre_top(m, l, B)
        lo = max(0, m[l] - al)
        hi = min(top, m[l] + al)
        pos = list(range(lo, hi + 1))
        u = np.array([term_value(m[:l] + (p,) + m[l + 1:], l + 1, a) for p in pos],
                     dtype=np.complex128)
        n = len(pos)
        J = np.zeros((n, n))
        for i in range(n - 1):
            J[i, i + 1] = J[i + 1, i] = np.sqrt(pos[i + 1] / 2.0)
        wm, wp = np.zeros_like(u), u
        for k in range(al):
            A, Bc, C = recurrence_coeffs(pot.basis, pot.scale, k)
            wm, wp = wp, A * (J @ wp) + Bc * wp - C * wm
        return wp[m[l] - lo]

    out = np.zeros(len(rows), dtype=np.complex128)
    for r, j in enumerate(rows):
        j = tuple(int(x) for x in j)
        acc = (sum(j) + 0.5 * N) * lookup(j)
        for coef, a in pot.terms:
            acc += coef * term_value(j, 0, a)
        out[r] = acc
    return out


# ----------------------------------------------------------------------------------
# Chebyshev interpolation of the torsional potential (Sec. 3.4, eq. TorsionalPotential)
# ----------------------------------------------------------------------------------


def exact_H_rows(N: int, B: int, pot: Potential, lookup, rows) -> np.ndarray:
    """((D + W_K) c)_j, the exact Galerkin product, for the multi-indices j in rows of the
    set K_N(B), one row at a time (the plain definition of Sec. 1.2, restricted to rows).

    W_K is the Galerkin matrix (phi_j, W^pol phi_m) over K.  By tensor-product
    orthonormality (Sec. 1.1) its entry is sum_t coef_t prod_l Q^(a_tl)[j_l, m_l] with Q^(a)
    the exact 1-D matrix of p_a (exact_1d), which vanishes unless |j_l - m_l| <= a_l; m runs
    over that box, and c(m) = lookup(m) for m in K, 0 outside."""
    rows = [tuple(int(x) for x in j) for j in rows]
    kmax = max((max(j) for j in rows), default=0) + max((max(a) for _, a in pot.terms), default=0)
    Q = {}

    def q(a):
        if a not in Q:
            Q[a] = exact_1d(pot.basis, pot.scale, a, kmax)
        return Q[a]

    out = np.zeros(len(rows), dtype=np.complex128)
    for r, j in enumerate(rows):
        acc = (sum(j) + 0.5 * N) * lookup(j)
        for coef, a in pot.terms:
            ranges = [range(max(0, j[l] - a[l]), j[l] + a[l] + 1) for l in range(N)]
            tot = 0.0 + 0.0j
            for m in itertools.product(*ranges):
                if np.prod([1 + x for x in m]) > B:
                    continue
                w = 1.0
                for l in range(N):
                    w *= q(a[l])[j[l], m[l]]
                    if w == 0.0:
                        break
                if w != 0.0:
                    tot += w * lookup(m)
            acc += coef * tot
        out[r] = acc
    return out


def chebyshev_interpolant_1d(f, R: int) -> np.ndarray:
    """Coefficients c_0..c_R of the degree-R polynomial interpolating f(y), y in [-1, 1],
    at the R + 1 Chebyshev points of the first kind, in the basis T_r(y)
    (discrete Chebyshev transform)."""
    theta = (2 * np.arange(R + 1) + 1) * np.pi / (2 * (R + 1))
    fy = f(np.cos(theta))
    c = np.array([(2.0 / (R + 1)) * np.sum(fy * np.cos(k * theta)) for k in range(R + 1)])
    c[0] *= 0.5
    return c


def torsional_potential(N: int, L: float = 16.0, R: int = 8) -> Potential:
    """W(x) = sum_l (1 - cos(x_l / L)) on [-L, L]^N, Chebyshev-interpolated per axis with
    degree R in the basis T_r(x_l / L) (Sec. 3.4).  The N constant terms are merged."""
    c = chebyshev_interpolant_1d(lambda y: 1.0 - np.cos(y), R)
    terms = [(N * c[0], (0,) * N)]
    for l in range(N):
        for r in range(1, R + 1):
            a = [0] * N
            a[l] = r
            terms.append((c[r], tuple(a)))
    return Potential(N, "cheb", L, terms)
