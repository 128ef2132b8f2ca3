"""Host-side checks of the C-ABI library: it loads, exports every function that
include/hs.h declares, builds index sets that agree with the oracle's enumeration
(paper Sec. 1.2), classifies potentials, and reports invalid arguments as status codes.
No call here touches a GPU."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from oracle.index import count, enumerate_lex

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hs():
    from paper_1403_3511_amd import hs as _hs
    return _hs


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hs_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported(hs):
    names = declared_functions()
    assert len(names) >= 35
    for n in names:
        assert hasattr(hs._lib, n), n          # dlsym through ctypes
    assert sorted(hs.EXPORTED) == names        # the binding wraps exactly the header
    assert "gfx950" in hs.hs_version()


@pytest.mark.parametrize("N,B,d", [(1, 50, 0), (2, 64, 0), (3, 500, 1), (3, 500, 2), (4, 700, 0),
                                   (4, 700, 4), (6, 300, 0), (10, 64, 0)])
def test_host_index_matches_oracle(hs, N, B, d):
    idx = hs.Index(N, B, d, upload=False)
    assert idx.size == count(N, B)
    k = idx.multi_indices().astype(np.int64)
    # every row is a member, and the rows are exactly the oracle's set
    assert np.all(np.prod(1 + k, axis=1) <= B)
    ref = enumerate_lex(N, B).astype(np.int64)
    assert sorted(map(tuple, k)) == sorted(map(tuple, ref))
    # tiles: rows sharing the prefix are contiguous, and within a tile the suffixes run in
    # graded order (prod(1 + s), lex)
    dd = idx.tile_dim
    assert 1 <= dd <= N
    pre, suf = k[:, :N - dd], k[:, N - dd:]
    keys = [tuple(p) for p in pre]
    starts = [0] + [i for i in range(1, len(keys)) if keys[i] != keys[i - 1]]
    assert len(set(keys)) == len(starts) == idx.ntiles
    for a, b in zip(starts, starts[1:] + [len(keys)]):
        g = [(int(np.prod(1 + s)), tuple(s)) for s in suf[a:b]]
        assert g == sorted(g)


@pytest.mark.parametrize("N,K,d", [(1, 7, 0), (2, 9, 0), (3, 5, 1), (3, 5, 3), (4, 4, 0), (4, 4, 2)])
def test_box_index_matches_full_box(hs, N, K, d):
    """Box sets: the rows are exactly {0..K}^N; tiles share prefixes and every tile holds
    the whole suffix list in lexicographic order."""
    from oracle.index import full_box
    idx = hs.Index(N, K, d, upload=False, box=True)
    assert idx.size == (K + 1) ** N
    k = idx.multi_indices().astype(np.int64)
    assert sorted(map(tuple, k)) == sorted(map(tuple, full_box(N, K).astype(np.int64)))
    dd = idx.tile_dim
    assert idx.ntiles == (K + 1) ** (N - dd)
    tile = (K + 1) ** dd
    for t in range(idx.ntiles):
        blk = k[t * tile:(t + 1) * tile]
        assert len({tuple(p) for p in blk[:, :N - dd]}) == 1
        assert [tuple(s) for s in blk[:, N - dd:]] == sorted(tuple(s) for s in blk[:, N - dd:])


@pytest.mark.parametrize("N,D,d", [(1, 9, 0), (2, 12, 0), (3, 8, 1), (3, 8, 2), (4, 7, 0), (4, 7, 4), (6, 6, 0)])
def test_total_degree_index_matches_oracle(hs, N, D, d):
    """Total-degree sets: the rows are exactly {|k|_1 <= D}; tiles share prefixes; a tile
    with prefix p holds the first C(d + D - |p|, d) suffixes of the list graded by
    (|s|_1, lex)."""
    import math
    from oracle.index import TotalDegreeIndex
    idx = hs.Index(N, D, d, upload=False, total_degree=True)
    ref = TotalDegreeIndex(N, D)
    assert idx.size == ref.size == math.comb(N + D, N)
    k = idx.multi_indices().astype(np.int64)
    assert sorted(map(tuple, k)) == sorted(map(tuple, ref.k.astype(np.int64)))
    dd = idx.tile_dim
    pre = [tuple(p) for p in k[:, :N - dd]]
    glob = sorted({(int(s.sum()), tuple(s)) for s in k[:, N - dd:]})
    i = 0
    while i < len(pre):
        j = i
        while j < len(pre) and pre[j] == pre[i]:
            j += 1
        n = math.comb(dd + D - sum(pre[i]), dd)
        assert j - i == n
        assert [tuple(s) for s in k[i:j, N - dd:]] == [g[1] for g in glob[:n]]
        i = j


def test_explicit_downward_closed_sets(hs):
    """hs_index_create_from_list: the rows come back in lexicographic order; for N >= 3 the
    tiles are the distinct prefixes (first N - 1 coordinates) with the last axis as the
    suffix, for N = 2 one row per tile; a repeated row or a set that is not downward
    closed is refused."""
    from synth import random_downward_set
    k = random_downward_set(4, 6, 7, seed=3)
    rng = np.random.default_rng(0)
    shuffled = k[rng.permutation(len(k))]
    idx = hs.Index(4, rows=shuffled, upload=False)
    assert idx.size == len(k)
    assert idx.tile_dim == 1 and idx.ntiles == len({tuple(r[:3]) for r in k})
    assert idx.nsuffix == k[:, 3].max() + 1
    assert np.array_equal(idx.multi_indices().astype(np.int64), k)
    k2 = random_downward_set(2, 5, 9, seed=4)
    idx2 = hs.Index(2, rows=k2, upload=False)
    assert idx2.tile_dim == 0 and idx2.ntiles == idx2.size == len(k2)
    assert np.array_equal(idx2.multi_indices().astype(np.int64), k2)
    k1 = np.arange(7).reshape(-1, 1)
    idx1 = hs.Index(1, rows=k1, upload=False)
    assert idx1.tile_dim == 1 and idx1.ntiles == 1
    assert np.array_equal(idx1.multi_indices().astype(np.int64), k1)
    with pytest.raises(hs.HSError) as e:
        hs.Index(4, rows=np.vstack([k, k[:1]]), upload=False)
    assert e.value.code == -1
    with pytest.raises(hs.HSError) as e:
        hs.Index(2, rows=[[0, 0], [0, 2]], upload=False)   # (0, 1) missing
    assert e.value.code == -1


def test_embedding_into_a_box(hs):
    """hs_index_embed: each row of a hyperbolic set maps to the box row with the same
    multi-index, or to -1 outside a smaller box."""
    sub = hs.Index(3, 30, upload=False)
    ks = sub.multi_indices().astype(np.int64)
    for K, d in ((29, 0), (5, 1), (5, 3)):
        box = hs.Index(3, K, d, upload=False, box=True)
        kb = box.multi_indices().astype(np.int64)
        m = sub.embed_map(box)
        inside = np.all(ks <= K, axis=1)
        assert np.array_equal(m >= 0, inside)
        assert np.array_equal(kb[m[inside]], ks[inside])

def test_embedding_between_any_set_kinds(hs):
    """hs_index_embed into a hyperbolic cross, a total-degree set and a set given as a
    list: each row maps to the target row with the same multi-index, or -1 outside."""
    sub = hs.Index(3, 60, upload=False)
    ks = sub.multi_indices().astype(np.int64)
    targets = [(hs.Index(3, 20, upload=False), lambda k: np.prod(1 + k, axis=1) <= 20),
               (hs.Index(3, 8, upload=False, total_degree=True), lambda k: k.sum(axis=1) <= 8),
               (hs.Index(3, 90, upload=False), lambda k: np.prod(1 + k, axis=1) <= 90)]
    lst = hs.Index(3, 20, upload=False).multi_indices()
    targets.append((hs.Index(3, rows=lst, upload=False), lambda k: np.prod(1 + k, axis=1) <= 20))
    for tgt, member in targets:
        kt = tgt.multi_indices().astype(np.int64)
        m = sub.embed_map(tgt)
        inside = member(ks)
        assert np.array_equal(m >= 0, inside)
        assert np.array_equal(kt[m[inside]], ks[inside])


def test_error_split_argument_checks(hs):
    """Containment and padding are checked on the host before anything runs."""
    fake = (C.c_double * 64)()
    fp = C.cast(fake, C.c_void_p)
    sub = hs.Index(2, 30, upload=False)
    small = hs.Index(2, 10, upload=False, box=True)
    box = hs.Index(2, 29, upload=False, box=True)
    pad2 = hs.Index(2, 31, upload=False, box=True)
    pot = hs.Pot(2, [(0.1, (8, 0)), (0.2, (0, 2))], basis="cheb", scale=16.0, upload=False)
    for b, p in ((small, None), (box, pad2)):   # box too small; pad by 2 < 8 / 2
        with pytest.raises(hs.HSError) as e:
            hs.hs_error_split(sub.h, fp, b.h, fp, fp, p.h if p else None, fp if p else None,
                              fp if p else None, pot.h, fp, fp, fp, fp, fp, None)
        assert e.value.code == -1


def test_prefix_tiles_are_initial_segments(hs):
    """A tile with remaining bound b holds the first |K_d(b)| suffixes of the global list."""
    N, B = 5, 400
    idx = hs.Index(N, B, 2, upload=False)
    k = idx.multi_indices().astype(np.int64)
    suf = k[:, 3:]
    glob = sorted({(int(np.prod(1 + s)), tuple(s)) for s in suf})
    pre = [tuple(p) for p in k[:, :3]]
    i = 0
    while i < len(pre):
        j = i
        while j < len(pre) and pre[j] == pre[i]:
            j += 1
        rem = B // int(np.prod(1 + np.array(pre[i])))
        assert j - i == count(2, rem)
        assert [tuple(s) for s in suf[i:j]] == [g[1] for g in glob[:j - i]]
        i = j


def test_potential_classification(hs):
    from synth import henon_heiles_chain
    tt = henon_heiles_chain(6, 0.111, 0.05)
    p = hs.Pot(6, [(x[0], x[1], x[2], x[3], x.degrees) for x in tt], subtract_harmonic=True, upload=False)
    assert p.fused
    cheb = hs.Pot(3, [(0.3, (2, 1, 0)), (-0.2, (0, 3, 0))], basis="cheb", scale=6.0, upload=False)
    assert cheb.fused
    herm = hs.Pot(3, [(0.1, (2, 2, 2)), (0.2, (6, 0, 0))], basis="herm", upload=False)
    assert not herm.fused
    # x_1 x_3 couples non-adjacent axes: outside the fused class
    assert not hs.Pot(3, [(1.0, (1, 0, 1))], upload=False).fused


def test_debug_build_is_built_with_its_checks(hs):
    """libhs_debug.so (built by __graft_entry__.build()) exports the same ABI and reports
    its neighbour-index checks; the release library reports none."""
    path = os.path.join(ROOT, "paper_1403_3511_amd", "libhs_debug.so")
    assert os.path.exists(path), "libhs_debug.so not built: run __graft_entry__.build()"
    dbg = C.CDLL(path)
    for name in declared_functions():
        assert hasattr(dbg, name), name
    built = C.c_int32(-1)
    dbg.hs_debug_checks.argtypes = [C.POINTER(C.c_int32)]
    assert dbg.hs_debug_checks(C.byref(built)) == 0 and built.value == 1
    assert hs.debug_checks() is False


def test_exact_operator_argument_checks(hs):
    """hs_apply_exact / hs_step_exact refuse padded sets that do not carry the exact
    Galerkin operator, before anything reaches a device (dummy device pointers)."""
    from synth import henon_heiles_chain
    tt = henon_heiles_chain(3, 0.111, 0.0)
    pot = hs.Pot(3, [(x[0], x[1], x[2], x[3], x.degrees) for x in tt], subtract_harmonic=True, upload=False)
    sub = hs.Index(3, 12, upload=False)
    d = C.c_void_p(256)  # never dereferenced: every case fails its checks first

    def expect(code, pad, p=pot, s=sub):
        with pytest.raises(hs.HSError) as e:
            hs.hs_apply_exact(s.h, pad.h, d, d, p.h, d, d, C.c_void_p(512), d, None)
        assert e.value.code == code, hs.last_error()
        with pytest.raises(hs.HSError) as e:
            hs.hs_step_exact(s.h, pad.h, d, d, p.h, d, 0.0, None, 0.01, 5, 1, d, d, None, None)
        assert e.value.code == code, hs.last_error()

    expect(-1, hs.Index(3, 12, upload=False))                       # not a box or a padded cross
    expect(-1, hs.Index(3, 11 + 1, box=True, upload=False))         # box without the margin (needs 11 + 2)
    expect(-1, hs.Index(3, 12, pad=2, upload=False))                # padded cross narrower than degree 3
    expect(-1, hs.Index(3, 13, pad=3, upload=False))                # padded cross of another bound
    expect(-1, hs.Index(4, 20, box=True, upload=False))             # another dimension
    lst = hs.Index(3, rows=sub.multi_indices(), upload=False)
    expect(-5, hs.Index(3, 16, box=True, upload=False), s=lst)      # sets given as lists
    nb = C.c_int64()
    box = hs.Index(3, 13, box=True, upload=False)  # kept alive across the call
    hs.hs_exact_workspace_bytes(sub.h, box.h, pot.h, 5, C.byref(nb))
    assert nb.value > 0
    with pytest.raises(hs.HSError):
        hs.hs_exact_workspace_bytes(sub.h, sub.h, pot.h, 33, C.byref(nb))


def test_error_paths(hs):
    h = C.c_void_p()
    codes = []

    def expect(code, fn, *args):
        with pytest.raises(hs.HSError) as e:
            fn(*args)
        assert e.value.code == code, (fn, hs.last_error())
        assert hs.last_error()  # a message is left for the caller
        codes.append(code)

    expect(-1, hs.hs_index_create, 0, 10, 0, C.byref(h))          # N < 1
    expect(-1, hs.hs_index_create, 17, 10, 0, C.byref(h))         # N > HS_NMAX
    expect(-1, hs.hs_index_create, 2, 0, 0, C.byref(h))           # B < 1
    expect(-1, hs.hs_index_create, 3, 10, 4, C.byref(h))          # tile_dim > N
    deg = (C.c_uint16 * 2)(1, 0)
    base = (C.c_double * 1)(1.0)
    expect(-1, hs.hs_pot_create, 2, 7, 1.0, 1, deg, base, None, None, None, 0, C.byref(h))   # basis
    expect(-1, hs.hs_pot_create, 2, 0, -1.0, 1, deg, base, None, None, None, 0, C.byref(h))  # scale
    expect(-5, hs.hs_pot_create, 2, 2, 1.0, 1, deg, base, None, None, None, 1, C.byref(h))   # herm + harmonic
    bad = (C.c_double * 1)(float("nan"))
    expect(-7, hs.hs_pot_create, 2, 0, 1.0, 1, deg, bad, None, None, None, 0, C.byref(h))    # non-finite
    big = (C.c_uint16 * 2)(65, 0)
    expect(-5, hs.hs_pot_create, 2, 0, 1.0, 1, big, base, None, None, None, 0, C.byref(h))   # degree > 64
    idx = hs.Index(2, 20, upload=False)
    pot3 = hs.Pot(3, [(1.0, (1, 0, 0))], upload=False)
    nb = C.c_int64()
    expect(-1, hs.hs_workspace_bytes, idx.h, pot3.h, 0, 10, C.byref(nb))      # N mismatch
    pot2 = hs.Pot(2, [(1.0, (1, 0))], upload=False)
    expect(-1, hs.hs_workspace_bytes, idx.h, pot2.h, 0, 33, C.byref(nb))      # m > 32
    expect(-1, hs.hs_workspace_bytes, idx.h, pot2.h, 5, 10, C.byref(nb))      # dtype
    expect(-1, hs.hs_apply_h, idx.h, None, pot2.h, None, 0, None, None, None, None)  # NULL buffers
    fk = (C.c_double * 64)()
    fkp, fkq = C.cast(fk, C.c_void_p), C.cast(C.byref(fk, 256), C.c_void_p)
    expect(-1, hs.hs_apply_x, idx.h, fkp, 2, 0, fkp, fkq, None)                # axis >= N
    expect(-1, hs.hs_apply_x, idx.h, fkp, -1, 0, fkp, fkq, None)               # axis < 0
    expect(-1, hs.hs_apply_x, idx.h, fkp, 0, 4, fkp, fkq, None)                # dtype
    expect(-1, hs.hs_apply_x, idx.h, fkp, 0, 0, fkp, fkp, None)                # in == out
    expect(-1, hs.hs_apply_x, idx.h, None, 0, 0, fkp, fkq, None)               # NULL metadata
    expect(-1, hs.hs_set_small_step_rows, -1)                                 # negative limit
    expect(-1, hs.hs_propagate, idx.h, fkp, pot2.h, fkp, 0, 0.0, None, 0.1, 4, 1, -1, fkp, fkq, None)  # nsteps < 0
    expect(-1, hs.hs_propagate, idx.h, fkp, pot2.h, fkp, 0, 0.0, None, 0.1, 0, 1, 5, fkp, fkq, None)   # m < 1
    expect(-7, hs.hs_propagate, idx.h, fkp, pot2.h, fkp, 0, 0.0, None, float("inf"), 4, 1, 5, fkp, fkq,
           None)                                                                 # h not finite
    expect(-1, hs.hs_pot_set_form, pot2.h, 7)                                 # unknown form
    gz = np.zeros(5 * 3 * 5)
    gp = gz.ctypes.data_as(C.POINTER(C.c_double))
    expect(-1, hs.hs_cheb_interp, 5, 3, 4, 4, 2.0, gp, 0, None, None, None)   # N > 4
    expect(-1, hs.hs_cheb_interp, 2, 3, 4, 16, 2.0, gp, 0, None, None, None)  # R + 1 > 16
    expect(-1, hs.hs_cheb_interp, 2, 3, 4, 4, 0.0, gp, 0, None, None, None)   # L <= 0
    expect(-5, hs.hs_cheb_interp, 4, 3, 4, 15, 2.0, gp, 0, None, None, None)  # 16^4 grid > LDS
    gen = hs.Pot(2, [(1.0, (4, 0))], upload=False)                            # outside the fused class
    assert not gen.fused
    expect(-5, hs.hs_pot_set_form, gen.h, hs.HS_FORM_SYM)
    hs.hs_pot_set_form(gen.h, hs.HS_FORM_PAPER)
    expect(-1, hs.hs_magnus4_workspace_bytes, idx.h, pot3.h, 0, 4, C.byref(nb))   # N mismatch
    expect(-1, hs.hs_magnus4_workspace_bytes, idx.h, pot2.h, 0, -1, C.byref(nb))  # m < 0
    # the two parameter blocks must differ (checked before any device access)
    fake = (C.c_double * 64)()
    fp = C.cast(fake, C.c_void_p)
    expect(-1, hs.hs_step_magnus4, idx.h, fp, pot2.h, fp, fp, 0, 0.0, None, 0.1, 4, 1, fp, fp,
           None, None)
    expect(-1, hs.hs_apply_magnus4, idx.h, fp, pot2.h, fp, fp, 0, 0.1, fp, fp, fp, None)
    expect(-1, hs.hs_step_magnus4, idx.h, fp, pot2.h, None, fp, 0, 0.0, None, 0.1, 4, 1, fp, fp,
           None, None)                                                           # NULL block
    expect(-1, hs.hs_mlp_create, 7, 100, 210, C.byref(h))                    # hidden not a multiple of 64
    expect(-1, hs.hs_mlp_create, 40, 256, 210, C.byref(h))                   # in > 32
    n = C.c_int32()
    expect(-1, hs.hs_gh_ncoef, 0, 6, C.byref(n))
    g = np.zeros(4 * 3 * 5)
    expect(-1, hs.hs_gh_project, 5, 3, 6, 16, g.ctypes.data_as(C.POINTER(C.c_double)), 1, None, None, None)
    assert set(codes) == {-1, -5, -7}


def test_magnus4_workspace_sizes(hs):
    """The fourth-order step needs three vectors beyond the midpoint step's workspace;
    its operator application alone needs three vectors plus the H workspace."""
    for N, B, terms in [(3, 300, [(0.1, (2, 1, 0)), (0.2, (0, 0, 3))]),
                        (2, 100, [(0.1, (4, 0)), (0.2, (1, 1))])]:
        idx = hs.Index(N, B, upload=False)
        pot = hs.Pot(N, terms, upload=False)
        for dt, es in ((hs.HS_C128, 16), (hs.HS_C64, 8)):
            vec = -(-idx.size * es // 256) * 256
            a, b, c0, c4 = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
            hs.hs_workspace_bytes(idx.h, pot.h, dt, 7, C.byref(a))
            hs.hs_magnus4_workspace_bytes(idx.h, pot.h, dt, 7, C.byref(b))
            hs.hs_workspace_bytes(idx.h, pot.h, dt, 0, C.byref(c0))
            hs.hs_magnus4_workspace_bytes(idx.h, pot.h, dt, 0, C.byref(c4))
            assert b.value == a.value + 3 * vec
            assert c4.value == c0.value + 3 * vec


def test_cheb_coefficient_counts(hs):
    import itertools
    for N, D, R in [(1, 10, 15), (2, 15, 15), (3, 8, 12), (4, 6, 6), (4, 5, 8), (3, 20, 6)]:
        want = sum(1 for r in itertools.product(range(R + 1), repeat=N) if sum(r) <= D)
        assert hs.cheb_ncoef(N, D, R) == want == len(hs.cheb_degrees(N, D, R))
    assert hs.cheb_ncoef(4, 6, 6) == math.comb(10, 4)


def test_sizes_and_counts(hs):
    n = C.c_int32()
    hs.hs_gh_ncoef(4, 6, C.byref(n))
    assert n.value == math.comb(10, 4) == 210
    h = C.c_void_p()
    hs.hs_mlp_create(7, 256, 210, C.byref(h))
    nb = C.c_int64()
    hs.hs_mlp_device_bytes(h, 256, C.byref(nb))
    nparam = 256 * 7 + 256 + 256 * 256 + 256 + 210 * 256 + 210
    assert nparam == 121810
    assert nb.value >= 4 * 4 * nparam  # weights, gradients, two Adam moments
    hs.hs_mlp_destroy(h)
    # workspace of the generic program: one vector per extra slot
    idx = hs.Index(3, 200, upload=False)
    herm = hs.Pot(3, [(0.1, (2, 2, 2)), (0.2, (6, 0, 0))], basis="herm", upload=False)
    hs.hs_workspace_bytes(idx.h, herm.h, 0, 0, C.byref(nb))
    assert nb.value >= 16 * idx.size


@pytest.mark.parametrize("N,B", [(1, 1), (1, 50), (2, 64), (3, 500), (5, 97), (8, 30), (16, 3)])
def test_index_count_without_enumeration(hs, N, B):
    assert hs.index_count(N, B) == count(N, B)


def test_index_count_agrees_with_built_sets(hs):
    for N, B in [(6, 4096), (8, 700), (3, 16384)]:
        assert hs.index_count(N, B) == hs.Index(N, B, upload=False).size
    n = C.c_int64()
    assert hs._lib.hs_index_count(0, 10, C.byref(n)) != 0
    assert hs._lib.hs_index_count(3, 0, C.byref(n)) != 0
    assert hs._lib.hs_index_count(3, 65537, C.byref(n)) != 0
    assert hs._lib.hs_index_count(3, 10, None) != 0


def test_batched_draw_size_rule(hs):
    """The batched workload's redraw rule keeps every accepted draw as it was and draws a
    rejected instance again from the same stream."""
    from synth import batch_instances
    cap = 1 << 16
    plain = batch_instances(64, seed=3)
    ruled = batch_instances(64, seed=3, accept=lambda N, B: hs.index_count(N, B) <= cap)
    assert all(hs.index_count(d["N"], d["B"]) <= cap for d in ruled)
    assert [d["seed"] for d in ruled] == [1000 + i for i in range(64)]
    # up to the first rejected draw the two sequences agree
    first = next(i for i, d in enumerate(plain) if hs.index_count(d["N"], d["B"]) > cap)
    assert ruled[:first] == plain[:first]
    assert ruled[first] != plain[first]


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and says why, before
    any device is touched."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("N,B,w,d", [(1, 10, 2, 0), (2, 24, 3, 0), (3, 12, 3, 0), (3, 12, 3, 1), (4, 10, 2, 0),
                                     (4, 10, 1, 4)])
def test_padded_index_matches_oracle(hs, N, B, w, d):
    """The library's padded cross is the oracle's set, with graded tiles, and every row of
    the hyperbolic cross embeds at the padded row holding its multi-index (as do box
    embeddings, through the same ranking)."""
    from oracle.index import PaddedIndex
    P = hs.Index(N, B, d, upload=False, pad=w)
    ref = PaddedIndex(N, B, w)
    k = P.multi_indices().astype(np.int64)
    assert P.size == ref.size
    assert sorted(map(tuple, k)) == sorted(map(tuple, ref.k.astype(np.int64)))
    dd = P.tile_dim
    pre, suf = k[:, :N - dd], k[:, N - dd:]
    keys = [tuple(p) for p in pre]
    starts = [0] + [i for i in range(1, len(keys)) if keys[i] != keys[i - 1]]
    for a, b in zip(starts, starts[1:] + [len(keys)]):
        g = [(int(np.prod(1 + np.maximum(s - w, 0))), tuple(s)) for s in suf[a:b]]
        assert g == sorted(g)
    sub = hs.Index(N, B, upload=False)
    mp = sub.embed_map(P)
    ks = sub.multi_indices().astype(np.int64)
    assert np.all(mp >= 0)
    assert np.array_equal(k[mp], ks)
    box = hs.Index(N, w + 2, upload=False, box=True)
    mb = sub.embed_map(box)
    inside = np.all(ks <= w + 2, axis=1)
    assert np.array_equal(mb >= 0, inside)
    assert np.array_equal(box.multi_indices().astype(np.int64)[mb[inside]], ks[inside])


def test_padded_index_errors(hs):
    h = C.c_void_p()
    for args in ((0, 10, 2, 0), (3, 0, 2, 0), (3, 65535, 2, 0), (3, 10, -1, 0), (3, 10, 17, 0), (3, 10, 2, 4)):
        with pytest.raises(hs.HSError):
            hs.hs_index_create_padded(*args, C.byref(h))
    sub = hs.Index(3, 10, upload=False)
    with pytest.raises(hs.HSError):
        sub.embed_map(hs.Index(4, 10, upload=False))   # the sets differ in N


def test_padded_count_saturates(hs):
    """The padded cross at N = 16, w = 16 has 17^16 > 2^63 members: refused as too large
    (no wrapped count), while the same w at N = 3 builds."""
    h = C.c_void_p()
    with pytest.raises(hs.HSError) as e:
        hs.hs_index_create_padded(16, 1, 16, 0, C.byref(h))
    assert e.value.code == -2
    assert hs.Index(3, 1, upload=False, pad=16).size == 17 ** 3


def test_bench_flop_model():
    """The bench's algorithmic flop count per row of H (8 per distinct partial product of a
    term, axis N first, 4 per term, 4 for the diagonal).  By hand for N = 2 (W = 0.111 x1^2 x2
    - 0.037 x2^3): partial products X2, X2^2, X2^3, X1 X2, X1^2 X2 -> 8*5 + 4*2 + 4 = 52; the
    chains with the laser give 276 at N = 6 and 484 at N = 10."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    from synth import henon_heiles_chain
    for N, laser, want in ((2, 0.0, 52), (6, 0.05, 276), (10, 0.05, 484)):
        deg = bench.w_degrees(henon_heiles_chain(N, 0.111, laser), N)
        assert bench.alg_flops_per_row(N, deg) == want
    # the harmonic part cancels in W: a pure oscillator costs the diagonal only
    assert bench.w_degrees(henon_heiles_chain(3, 0.0, 0.0), 3) == []


def test_fibre_lists_extend_the_device_block(hs):
    """hs_index_build_fibres appends the per-axis fibre lists (a position word, 8 bytes, and
    its two neighbour distances, 4 bytes, per row and axis, halos included) to the device
    block; a second call changes nothing; NULL is refused."""
    for N, B, kw in ((2, 4096, {}), (4, 512, {}), (3, 1500, {"tile_dim": 1}), (3, 40, {"box": True})):
        idx = hs.Index(N, B, upload=False, **kw)
        n0 = C.c_int64()
        hs.hs_index_device_bytes(idx.h, C.byref(n0))
        hs.hs_index_build_fibres(idx.h)
        n1 = C.c_int64()
        hs.hs_index_device_bytes(idx.h, C.byref(n1))
        assert n1.value >= n0.value + 12 * N * idx.size
        # halos add at most 2 * 8 positions per 240 core positions of a fibre; batch starts
        # (one per 256 positions) and padding
        assert n1.value <= n0.value + 12 * N * idx.size * (1 + 16 / 240) + 8 * N * (idx.size / 64 + 2) + 4096
        hs.hs_index_build_fibres(idx.h)
        n2 = C.c_int64()
        hs.hs_index_device_bytes(idx.h, C.byref(n2))
        assert n2.value == n1.value
    with pytest.raises(hs.HSError):
        hs.hs_index_build_fibres(None)
