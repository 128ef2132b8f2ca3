"""Pins of the oracle's index set (hyperbolic cross, Sec. 1.2) against brute force and
independent counts."""
import itertools

import numpy as np
import pytest

from oracle.index import BoxIndex, IndexSet, LexRanker, count, enumerate_lex, in_set


def brute(N, B):
    """Filter the box {0..B-1}^N by the defining product rule."""
    pts = [k for k in itertools.product(range(B), repeat=N) if np.prod([1 + x for x in k]) <= B]
    return np.array(sorted(pts), dtype=np.int64)


@pytest.mark.parametrize("N,B", [(1, 7), (2, 1), (2, 12), (3, 20), (4, 30), (2, 64), (5, 9)])
def test_enumeration_matches_brute_force(N, B):
    k = enumerate_lex(N, B).astype(np.int64)
    ref = brute(N, B)
    assert k.shape == ref.shape
    assert np.array_equal(k, ref)  # same set and lexicographic order
    assert count(N, B) == len(ref)


def test_known_sizes():
    # |K_1(B)| = B; divisor-sum values for the workload configurations
    assert count(1, 4096) == 4096
    assert count(2, 64) == 280
    assert count(6, 4096) == 4883360
    assert count(4, 8192) == 1510397
    assert count(10, 4096) == 103495890
    # K_2(B) = sum_{a<=B} floor(B/a) (divisor summatory function), independent formula
    for B in (1, 2, 10, 100, 1000):
        assert count(2, B) == sum(B // a for a in range(1, B + 1))


def test_size_formula_recursion():
    # |K_N(B)| = sum_{a=1}^{B} |K_{N-1}(floor(B/a))|
    for N in range(2, 6):
        for B in (5, 17, 64):
            assert count(N, B) == sum(count(N - 1, B // a) for a in range(1, B + 1))


@pytest.mark.parametrize("N,B", [(2, 40), (3, 64), (4, 100), (6, 256)])
def test_neighbour_tables(N, B):
    idx = IndexSet(N, B)
    k = idx.k.astype(np.int64)
    assert np.array_equal(idx.rank(k), np.arange(idx.size))
    for l in range(N):
        p, m = idx.nbr_plus[l], idx.nbr_minus[l]
        # downward closure: every k with k_l > 0 has k - e_l in the set
        assert np.all((m >= 0) == (k[:, l] > 0))
        # k - e_l and k + e_l are what they claim to be
        hm = m >= 0
        d = k[m[hm]] - k[hm]
        assert np.all(d[:, l] == -1) and np.all(np.delete(d, l, axis=1) == 0)
        hp = p >= 0
        d = k[p[hp]] - k[hp]
        assert np.all(d[:, l] == 1) and np.all(np.delete(d, l, axis=1) == 0)
        # absent + neighbours are exactly those that violate the product rule
        kp = k.copy()
        kp[:, l] += 1
        assert np.array_equal(hp, in_set(kp, B))
        # + then - is the identity
        assert np.all(m[p[hp]] == np.nonzero(hp)[0])


def test_box_index():
    box = BoxIndex(3, 4)
    assert box.size == 125
    k = box.k.astype(np.int64)
    assert np.array_equal(box.rank(k), np.arange(125))
    for l in range(3):
        hp = box.nbr_plus[l] >= 0
        assert np.all(hp == (k[:, l] < 4))
        d = k[box.nbr_plus[l][hp]] - k[hp]
        assert np.all(d[:, l] == 1)


def test_ranker_on_random_members():
    rng = np.random.default_rng(3)
    N, B = 6, 4096
    r = LexRanker(N, B)
    # draw random members by rejection and compare the rank to a direct count over
    # the lex enumeration of a small sub-problem: rank differences of consecutive
    # members of one axis-N fibre are 1
    for _ in range(50):
        while True:
            k = rng.integers(0, 8, size=N)
            if np.prod(1 + k) <= B:
                break
        if np.prod(1 + k[:-1]) * (k[-1] + 2) <= B:
            k2 = k.copy()
            k2[-1] += 1
            assert r.rank(k2)[0] - r.rank(k)[0] == 1


def test_total_degree_index():
    """|{|k|_1 <= D}| = C(N + D, N); downward closed; neighbour maps consistent."""
    import math
    from oracle.index import TotalDegreeIndex
    for N, D in [(1, 5), (2, 7), (3, 6), (4, 4)]:
        ix = TotalDegreeIndex(N, D)
        assert ix.size == math.comb(N + D, N)
        k = ix.k.astype(np.int64)
        assert np.all(k.sum(axis=1) <= D)
        for l in range(N):
            p = ix.nbr_plus[l]
            ok = p >= 0
            assert np.array_equal(ok, k.sum(axis=1) < D)
            assert np.all(k[p[ok], l] == k[ok, l] + 1)
            m = ix.nbr_minus[l]
            assert np.array_equal(m >= 0, k[:, l] > 0)
        assert np.array_equal(ix.rank(k), np.arange(ix.size))


@pytest.mark.parametrize("N,B,w", [(1, 10, 2), (2, 20, 3), (3, 12, 1), (3, 8, 3)])
def test_padded_index(N, B, w):
    """The padded cross prod(1 + max(k_l - w, 0)) <= B: w = 0 gives the hyperbolic cross;
    it contains every k + d with k in K_N(B) and |d_l| <= w; it is downward closed; its
    size follows the recursion in the first coordinate (values 0..w cost 1, value w + a
    costs 1 + a); the neighbour maps are those of brute force."""
    from oracle.index import PaddedIndex
    P = PaddedIndex(N, B, w)
    assert sorted(map(tuple, PaddedIndex(N, B, 0).k)) == sorted(map(tuple, enumerate_lex(N, B)))
    members = set(map(tuple, P.k.astype(int)))
    for k in enumerate_lex(N, B).astype(int):
        for d in itertools.product(range(-w, w + 1), repeat=N):
            m = tuple(int(a + b) for a, b in zip(k, d))
            if min(m) >= 0:
                assert m in members
    for m in members:
        for l in range(N):
            if m[l] > 0:
                assert tuple(m[i] - (i == l) for i in range(N)) in members

    def cnt(n, b):
        if b < 1:
            return 0
        if n == 0:
            return 1
        return (w + 1) * cnt(n - 1, b) + sum(cnt(n - 1, b // (1 + a)) for a in range(1, b))
    assert P.size == cnt(N, B)
    for l in range(N):
        for i, m in enumerate(P.k.astype(int)):
            up = tuple(m[j] + (j == l) for j in range(N))
            assert (P.nbr_plus[l, i] >= 0) == (up in members)


@pytest.mark.parametrize("N,B", [(2, 30), (3, 40), (4, 24)])
def test_list_index(N, B):
    """ListIndex built from the rows of a hyperbolic cross (shuffled) is that set, with the
    same lexicographic order and neighbour maps as IndexSet; on a random downward-closed set
    its neighbour maps and ranks agree with brute force."""
    from oracle.index import ListIndex
    from synth import random_downward_set
    ref = IndexSet(N, B)
    rows = ref.k.astype(np.int64)
    L = ListIndex(rows[np.random.default_rng(1).permutation(len(rows))])
    assert np.array_equal(L.k, ref.k)
    assert np.array_equal(L.nbr_plus, ref.nbr_plus) and np.array_equal(L.nbr_minus, ref.nbr_minus)
    assert np.array_equal(L.rank(rows), np.arange(len(rows)))
    R = random_downward_set(N, 5, 6, seed=N)
    L2 = ListIndex(R)
    members = {tuple(r) for r in R.tolist()}
    assert len(members) == L2.size
    for i, row in enumerate(L2.k.astype(int).tolist()):
        assert L2.rank(np.array([row]))[0] == i
        for l in range(N):
            up = tuple(row[j] + (j == l) for j in range(N))
            dn = tuple(row[j] - (j == l) for j in range(N))
            assert (L2.nbr_plus[l, i] >= 0) == (up in members)
            assert (L2.nbr_minus[l, i] >= 0) == (row[l] > 0)
            if row[l] > 0:
                assert tuple(L2.k[L2.nbr_minus[l, i]].astype(int)) == dn
