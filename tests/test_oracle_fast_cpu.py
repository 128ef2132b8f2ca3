"""Pins of the compiled CPU oracle (oracle/fast_cpu.c): its enumeration against the
NumPy oracle's lexicographic one and the known set sizes (Sec. 1.2), its H application
against operators.fast_apply_H (Sec. 3.2, eq. Horner; Fig. 3) in all three bases and with
the harmonic part alone (H = D exactly, Sec. 1.1), and independence of the thread count."""
import numpy as np
import pytest

from oracle import fast_cpu
from oracle.index import IndexSet, count, enumerate_lex
from oracle.operators import Potential, fast_apply_H, subtract_harmonic


@pytest.mark.parametrize("N,B", [(1, 30), (2, 64), (3, 200), (4, 300), (6, 64)])
def test_enumeration_matches(N, B):
    S = fast_cpu.FastSet(N, B)
    assert S.size == count(N, B)
    assert np.array_equal(S.multi_indices(), enumerate_lex(N, B))


@pytest.mark.parametrize("N,B", [(1, 20), (2, 64), (3, 200), (4, 300), (5, 120)])
@pytest.mark.parametrize("basis,scale", [("mono", 1.0), ("cheb", 3.0), ("herm", 1.5)])
def test_apply_h_matches_numpy_oracle(N, B, basis, scale):
    rng = np.random.default_rng(N * 100 + B)
    S = fast_cpu.FastSet(N, B)
    ix = IndexSet(N, B)
    v = rng.normal(size=S.size) + 1j * rng.normal(size=S.size)
    terms = [(float(rng.normal()), tuple(int(a) for a in rng.integers(0, 4, N))) for _ in range(6)]
    pot = Potential(N, basis, scale, terms)
    y = S.apply_H(pot, v, 1)
    ref = fast_apply_H(ix, pot, v)
    assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref)
    assert np.max(np.abs(y - ref)) <= 1e-14 * np.max(np.abs(ref))
    # every row is computed on its own: the thread count does not change a bit
    assert np.array_equal(y, S.apply_H(pot, v, 3))


def test_harmonic_part_alone_is_the_diagonal():
    N, B = 3, 150
    S = fast_cpu.FastSet(N, B)
    V = Potential(N, "mono", 1.0, [(0.5, tuple(2 if i == l else 0 for i in range(N))) for l in range(N)])
    W = subtract_harmonic(V)
    assert W.terms == []
    v = np.random.default_rng(1).normal(size=S.size) + 0j
    y = S.apply_H(W, v)
    k = S.multi_indices().astype(np.float64)
    assert np.array_equal(y, (k.sum(axis=1) + 0.5 * N) * v)


def test_refuses_out_of_range():
    with pytest.raises(ValueError):
        fast_cpu.FastSet(0, 10)
    with pytest.raises(ValueError):
        fast_cpu.FastSet(2, 100000)
