"""Oracle: the hyperbolically reduced index set and its neighbour structure.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Paper, Sec. 1.2 ("Galerkin ansatz with reduced index set"): the reduced set is
    K = { k in N_0^N : prod_l (1 + k_l) <= K_paper + 1 }.
This code takes the product bound B directly (B = K_paper + 1), so the per-axis maximum
index is B - 1.  The paper also requires downward closedness (k in K, k_l > 0 implies
k - e_l in K), which the product rule satisfies.

The canonical order of the oracle is lexicographic in (k_1, ..., k_N), k_N fastest.
"""
from __future__ import annotations

import functools

import numpy as np


@functools.lru_cache(maxsize=None)
def count(N: int, B: int) -> int:
    """|K_N(B)| by splitting on the first coordinate: a = 1 + k_1 ranges over 1..B and the
    rest is K_{N-1}(floor(B / a)).  (Definition of the set, Sec. 1.2.)"""
    if B < 1:
        return 0
    if N == 0:
        return 1
    return sum(count(N - 1, B // a) for a in range(1, B + 1))


def enumerate_lex(N: int, B: int) -> np.ndarray:
    """All k in K_N(B) as a (|K|, N) uint16 array in lexicographic order.

    Built axis by axis: a prefix with remaining bound b admits k_l = 0..b-1 and leaves
    the bound b // (1 + k_l) for the remaining axes (Sec. 1.2)."""
    if N < 1 or B < 1:
        raise ValueError("need N >= 1 and B >= 1")
    if B > 65536:
        raise ValueError("B > 65536 not supported by the uint16 multi-index store")
    pref = np.zeros((1, 0), dtype=np.uint16)
    bnd = np.array([B], dtype=np.int64)
    for _ in range(N):
        cnt = bnd
        tot = int(cnt.sum())
        rep = np.repeat(np.arange(len(bnd)), cnt)
        first = np.cumsum(cnt) - cnt
        a = np.arange(tot, dtype=np.int64) - np.repeat(first, cnt)
        pref = np.concatenate([pref[rep], a.astype(np.uint16)[:, None]], axis=1)
        bnd = bnd[rep] // (1 + a)
    return pref


def in_set(k: np.ndarray, B: int) -> np.ndarray:
    """Membership test prod(1 + k_l) <= B, k_l >= 0 (rows of an integer array)."""
    k = np.asarray(k, dtype=np.int64)
    return np.all(k >= 0, axis=-1) & (np.prod(1 + k, axis=-1) <= B)


class LexRanker:
    """Position of a multi-index in the lexicographic enumeration of K_N(B).

    rank(k) = sum_l #{ k' in K : k'_1..k'_{l-1} = k_1..k_{l-1}, k'_l < k_l }
            = sum_l sum_{a < k_l} |K_{N-l}(floor(B_l / (1 + a)))|,
    with B_1 = B and B_{l+1} = floor(B_l / (1 + k_l)).  A direct count over the set
    definition (Sec. 1.2)."""

    def __init__(self, N: int, B: int):
        self.N, self.B = N, B
        self.tables = []
        for l in range(N):
            n_rest = N - 1 - l
            offs = np.full(B + 1, -1, dtype=np.int64)
            chunks, pos = [], 0
            for b in sorted({B // q for q in range(1, B + 1)}):
                sizes = np.array([count(n_rest, b // (1 + a)) for a in range(b)], dtype=np.int64)
                cs = np.concatenate([[0], np.cumsum(sizes)])
                offs[b] = pos
                chunks.append(cs)
                pos += len(cs)
            self.tables.append((offs, np.concatenate(chunks)))

    def rank(self, k: np.ndarray) -> np.ndarray:
        k = np.asarray(k, dtype=np.int64)
        if k.ndim == 1:
            k = k[None, :]
        r = np.zeros(k.shape[0], dtype=np.int64)
        b = np.full(k.shape[0], self.B, dtype=np.int64)
        for l in range(self.N):
            offs, flat = self.tables[l]
            r += flat[offs[b] + k[:, l]]
            b = b // (1 + k[:, l])
        return r


class IndexSet:
    """K_N(B) in lex order with the neighbour maps k -> k +- e_l (-1 where absent)."""

    def __init__(self, N: int, B: int, with_neighbours: bool = True):
        self.N, self.B = N, B
        self.k = enumerate_lex(N, B)
        self.size = self.k.shape[0]
        self.ranker = LexRanker(N, B)
        self.nbr_plus = None
        self.nbr_minus = None
        if with_neighbours:
            self.nbr_plus = np.empty((N, self.size), dtype=np.int64)
            self.nbr_minus = np.empty((N, self.size), dtype=np.int64)
            k64 = self.k.astype(np.int64)
            prod = np.prod(1 + k64, axis=1)
            for l in range(N):
                kl = k64[:, l]
                # k + e_l is in K iff prod / (1 + k_l) * (2 + k_l) <= B
                ok = (prod // (1 + kl)) * (2 + kl) <= B
                kp = k64.copy()
                kp[:, l] += 1
                out = np.full(self.size, -1, dtype=np.int64)
                out[ok] = self.ranker.rank(kp[ok])
                self.nbr_plus[l] = out
                okm = kl > 0
                km = k64.copy()
                km[:, l] -= 1
                outm = np.full(self.size, -1, dtype=np.int64)
                outm[okm] = self.ranker.rank(km[okm])
                self.nbr_minus[l] = outm

    def rank(self, k: np.ndarray) -> np.ndarray:
        return self.ranker.rank(k)


def full_box(N: int, Kmax: int) -> np.ndarray:
    """The full tensor set {0..Kmax}^N in lex order (Sec. 1.2, K_full)."""
    g = np.indices((Kmax + 1,) * N).reshape(N, -1).T
    return g.astype(np.uint16)


class BoxIndex:
    """Full box {0..Kmax}^N with neighbour maps, same interface as IndexSet."""

    def __init__(self, N: int, Kmax: int):
        self.N, self.Kmax = N, Kmax
        self.k = full_box(N, Kmax)
        self.size = self.k.shape[0]
        n1 = Kmax + 1
        strides = [n1 ** (N - 1 - l) for l in range(N)]
        idx = np.arange(self.size, dtype=np.int64)
        self.nbr_plus = np.empty((N, self.size), dtype=np.int64)
        self.nbr_minus = np.empty((N, self.size), dtype=np.int64)
        for l in range(N):
            kl = self.k[:, l].astype(np.int64)
            self.nbr_plus[l] = np.where(kl < Kmax, idx + strides[l], -1)
            self.nbr_minus[l] = np.where(kl > 0, idx - strides[l], -1)

    def rank(self, k: np.ndarray) -> np.ndarray:
        k = np.asarray(k, dtype=np.int64)
        n1 = self.Kmax + 1
        r = np.zeros(k.shape[0], dtype=np.int64)
        for l in range(self.N):
            r = r * n1 + k[:, l]
        return r


class TotalDegreeIndex:
    """The total-degree set {k in N_0^N : |k|_1 <= D} (a downward-closed set other than
    the hyperbolic cross, Sec. 1.2) in lex order, with neighbour maps and rank, same
    interface as IndexSet.  Enumerated by brute force over the box {0..D}^N."""

    def __init__(self, N: int, D: int):
        self.N, self.D = N, D
        grid = np.indices((D + 1,) * N).reshape(N, -1).T
        self.k = grid[grid.sum(axis=1) <= D].astype(np.uint16)   # lex order (last axis fastest)
        self.size = self.k.shape[0]
        self._pos = {tuple(int(x) for x in row): i for i, row in enumerate(self.k)}
        self.nbr_plus = np.full((N, self.size), -1, dtype=np.int64)
        self.nbr_minus = np.full((N, self.size), -1, dtype=np.int64)
        for i, row in enumerate(self.k):
            for l in range(N):
                m = [int(x) for x in row]
                m[l] += 1
                self.nbr_plus[l, i] = self._pos.get(tuple(m), -1)
                m[l] -= 2
                if m[l] >= 0:
                    self.nbr_minus[l, i] = self._pos[tuple(m)]

    def rank(self, k: np.ndarray) -> np.ndarray:
        return np.array([self._pos[tuple(int(x) for x in row)] for row in np.atleast_2d(k)], dtype=np.int64)


class PaddedIndex:
    """The padded cross {k : prod(1 + max(k_l - w, 0)) <= B} (the hyperbolic cross of Sec. 1.2
    widened by w in every axis: it holds every k + d with k in K_N(B) and |d_l| <= w) in
    lex order, with neighbour maps and rank, same interface as IndexSet.  Enumerated by
    brute force over the box {0..B-1+w}^N, so for small sets only."""

    def __init__(self, N: int, B: int, w: int):
        self.N, self.B, self.w = N, B, w
        grid = np.indices((B + w,) * N).reshape(N, -1).T
        cost = np.prod(1 + np.maximum(grid - w, 0), axis=1)
        self.k = grid[cost <= B].astype(np.uint16)   # lex order (last axis fastest)
        self.size = self.k.shape[0]
        self._pos = {tuple(int(x) for x in row): i for i, row in enumerate(self.k)}
        self.nbr_plus = np.full((N, self.size), -1, dtype=np.int64)
        self.nbr_minus = np.full((N, self.size), -1, dtype=np.int64)
        for i, row in enumerate(self.k):
            for l in range(N):
                m = [int(x) for x in row]
                m[l] += 1
                self.nbr_plus[l, i] = self._pos.get(tuple(m), -1)
                m[l] -= 2
                if m[l] >= 0:
                    self.nbr_minus[l, i] = self._pos[tuple(m)]

    def rank(self, k: np.ndarray) -> np.ndarray:
        return np.array([self._pos[tuple(int(x) for x in row)] for row in np.atleast_2d(k)], dtype=np.int64)


class ListIndex:
    """An explicit downward-closed set given by its rows (sorted lexicographically here),
    with neighbour maps and rank, same interface as IndexSet."""

    def __init__(self, rows: np.ndarray):
        rows = np.asarray(rows, dtype=np.int64)
        order = np.lexsort(rows.T[::-1])
        self.k = rows[order].astype(np.uint16)
        self.size, self.N = self.k.shape
        self._pos = {tuple(int(x) for x in row): i for i, row in enumerate(self.k)}
        self.nbr_plus = np.full((self.N, self.size), -1, dtype=np.int64)
        self.nbr_minus = np.full((self.N, self.size), -1, dtype=np.int64)
        for i, row in enumerate(self.k):
            for l in range(self.N):
                m = [int(x) for x in row]
                m[l] += 1
                self.nbr_plus[l, i] = self._pos.get(tuple(m), -1)
                m[l] -= 2
                if m[l] >= 0:
                    self.nbr_minus[l, i] = self._pos.get(tuple(m), -1)

    def rank(self, k: np.ndarray) -> np.ndarray:
        return np.array([self._pos[tuple(int(x) for x in row)] for row in np.atleast_2d(k)], dtype=np.int64)
