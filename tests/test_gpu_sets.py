"""Index sets other than the hyperbolic cross on the GPU: total-degree sets
{|k|_1 <= D} in the tiled layout, against the oracle's fast operator on the same set
(fused and generic potentials, every prefix/suffix split), Lanczos steps and the
fourth-order operator on them, and the symmetrised form refused there."""
import math

import numpy as np
import pytest

from oracle.index import TotalDegreeIndex
from oracle.operators import Potential, fast_apply_H, torsional_potential
from oracle.propagate import lanczos_expm, magnus4_operator
from synth import coherent_state, complex_normal_by_index
from tests.hsutil import hh_workload, lib_terms, oracle_W, rel2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


def _setup(hs, N, D, d, kind):
    ix = TotalDegreeIndex(N, D)
    if kind == "hh":
        tt = hh_workload(N, 0.111, 0.05)
        W_at = lambda t: oracle_W(N, tt, t)  # noqa: E731
        pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    else:
        W = torsional_potential(N)
        W_at = lambda t: W  # noqa: E731
        pot = hs.Pot(N, [(float(c), a) for c, a in W.terms], basis="cheb", scale=W.scale)
    idx = hs.Index(N, D, d, total_degree=True)
    pos = ix.rank(idx.multi_indices().astype(np.int64))
    return ix, W_at, pot, idx, pos


@pytest.mark.parametrize("N,D,d,kind", [(2, 60, 0, "hh"), (3, 30, 0, "hh"), (3, 30, 1, "hh"), (4, 16, 3, "hh"),
                                        (4, 16, 4, "hh"), (6, 9, 0, "hh"), (3, 24, 0, "torsional")])
def test_apply_on_total_degree_set(hs, N, D, d, kind):
    import torch
    ix, W_at, pot, idx, pos = _setup(hs, N, D, d, kind)
    assert pot.fused == (kind == "hh")
    pot.set_time(0.3)
    c = complex_normal_by_index(ix.k, 60 + N)
    y_ref = fast_apply_H(ix, W_at(0.3), c)
    cl = torch.from_numpy(np.ascontiguousarray(c[pos])).to("cuda")
    yl = torch.empty_like(cl)
    hs.apply_h(idx, pot, cl, yl)
    torch.cuda.synchronize()
    y = np.empty_like(c)
    y[pos] = yl.cpu().numpy()
    assert rel2(y, y_ref) <= 1e-12


def test_steps_and_magnus4_on_total_degree_set(hs):
    import torch
    N, D, m, h, n = 3, 30, 8, 0.02, 4
    ix, W_at, pot, idx, pos = _setup(hs, N, D, 0, "hh")
    c0 = coherent_state(ix.k, [0.8, -0.4, 0.3])
    c0 /= np.linalg.norm(c0)
    ref = c0.copy()
    t = 0.0
    for _ in range(n):
        W = W_at(t + 0.5 * h)
        ref = lanczos_expm(lambda v: fast_apply_H(ix, W, v), ref, h, m)[0]
        t += h
    c = torch.from_numpy(np.ascontiguousarray(c0[pos])).to("cuda")
    t = 0.0
    for _ in range(n):
        hs.step(idx, pot, c, t, h, m)
        t += h
    torch.cuda.synchronize()
    got = np.empty_like(c0)
    got[pos] = c.cpu().numpy()
    assert rel2(got, ref) <= 1e-11
    # fourth-order operator (fused passes) on the same set
    c1, c2 = 0.5 - math.sqrt(3.0) / 6.0, 0.5 + math.sqrt(3.0) / 6.0
    hh = 0.5
    W1, W2 = W_at(0.4 + c1 * hh), W_at(0.4 + c2 * hh)
    v = complex_normal_by_index(ix.k, 71)
    y_ref = magnus4_operator(lambda x: fast_apply_H(ix, W1, x), lambda x: fast_apply_H(ix, W2, x), hh)(v)
    d1, d2 = pot.blocks2()
    hs.hs_pot_set_time(pot.h, hs.ptr(d1), 0.4 + c1 * hh, None, hs.stream_ptr())
    hs.hs_pot_set_time(pot.h, hs.ptr(d2), 0.4 + c2 * hh, None, hs.stream_ptr())
    vl = torch.from_numpy(np.ascontiguousarray(v[pos])).to("cuda")
    yl = torch.empty_like(vl)
    hs.apply_magnus4(idx, pot, hh, vl, yl)
    torch.cuda.synchronize()
    y = np.empty_like(v)
    y[pos] = yl.cpu().numpy()
    assert rel2(y, y_ref) <= 1e-12


def test_symmetrised_form_refused_off_the_hyperbolic_cross(hs):
    import torch
    idx = hs.Index(3, 10, total_degree=True)
    tt = hh_workload(3, 0.111, 0.05)
    pot = hs.Pot(3, lib_terms(tt), subtract_harmonic=True)
    pot.set_form(hs.HS_FORM_SYM)
    x = torch.zeros(idx.size, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(hs.HSError) as e:
        hs.apply_h(idx, pot, x, y)
    assert e.value.code == -5


@pytest.mark.parametrize("kind,N,n", [("total_degree", 3, 0), ("total_degree", 4, 1), ("box", 2, 0), ("box", 3, 1)])
def test_degenerate_sets(hs, kind, N, n):
    """One-row and (N + 1)-row total-degree sets, the one-point box and the 2^N box: H,
    a Lanczos step and the fourth-order operator against the oracle."""
    import torch
    from oracle.index import BoxIndex
    ix = TotalDegreeIndex(N, n) if kind == "total_degree" else BoxIndex(N, n)
    tt = hh_workload(N, 0.111, 0.05)
    W = oracle_W(N, tt, 0.2)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    pot.set_time(0.2)
    idx = hs.Index(N, n, total_degree=(kind == "total_degree"), box=(kind == "box"))
    assert idx.size == ix.size
    pos = ix.rank(idx.multi_indices().astype(np.int64))
    c = complex_normal_by_index(ix.k, 5)
    cl = torch.from_numpy(np.ascontiguousarray(c[pos])).to("cuda")
    yl = torch.empty_like(cl)
    hs.apply_h(idx, pot, cl, yl)
    hs.step(idx, pot, cl, 0.0, 0.01, 4)
    torch.cuda.synchronize()
    y = np.empty_like(c)
    y[pos] = yl.cpu().numpy()
    assert rel2(y, fast_apply_H(ix, W, c)) <= 1e-12
    ref = lanczos_expm(lambda v: fast_apply_H(ix, oracle_W(N, tt, 0.005), v), c, 0.01, 4)[0]
    got = np.empty_like(c)
    got[pos] = cl.cpu().numpy()
    assert rel2(got, ref) <= 1e-11


@pytest.mark.parametrize("N,npts,maxc,kind", [(2, 5, 40, "hh"), (3, 8, 20, "hh"), (4, 6, 9, "hh"),
                                             (5, 10, 6, "hh"), (6, 12, 5, "hh"), (7, 10, 3, "hh"),
                                             (8, 10, 3, "hh"), (1, 1, 30, "hh"), (3, 8, 20, "torsional")])
def test_explicit_downward_closed_set(hs, N, npts, maxc, kind):
    """A random downward-closed set (union of boxes below random corners) given as a list:
    H against the oracle on the same set, and a Lanczos step."""
    import torch
    from oracle.index import ListIndex
    from synth import random_downward_set
    rows = random_downward_set(N, npts, maxc, seed=40 + N)
    ix = ListIndex(rows)
    if kind == "hh":
        tt = hh_workload(N, 0.111, 0.05)
        W_at = lambda t: oracle_W(N, tt, t)  # noqa: E731
        pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    else:
        W = torsional_potential(N)
        W_at = lambda t: W  # noqa: E731
        pot = hs.Pot(N, [(float(c), a) for c, a in W.terms], basis="cheb", scale=W.scale)
    idx = hs.Index(N, rows=rows)
    pos = ix.rank(idx.multi_indices().astype(np.int64))
    pot.set_time(0.3)
    c = complex_normal_by_index(ix.k, 80 + N)
    cl = torch.from_numpy(np.ascontiguousarray(c[pos])).to("cuda")
    yl = torch.empty_like(cl)
    hs.apply_h(idx, pot, cl, yl)
    torch.cuda.synchronize()
    y = np.empty_like(c)
    y[pos] = yl.cpu().numpy()
    assert rel2(y, fast_apply_H(ix, W_at(0.3), c)) <= 1e-12
    c0 = c / np.linalg.norm(c)
    ref = lanczos_expm(lambda v: fast_apply_H(ix, W_at(0.005), v), c0, 0.01, 6)[0]
    cs = torch.from_numpy(np.ascontiguousarray(c0[pos])).to("cuda")
    hs.step(idx, pot, cs, 0.0, 0.01, 6)
    torch.cuda.synchronize()
    got = np.empty_like(c0)
    got[pos] = cs.cpu().numpy()
    assert rel2(got, ref) <= 1e-11


@pytest.mark.parametrize("N,B,w", [(2, 30, 3), (3, 12, 2)])
def test_steps_on_a_padded_cross(hs, N, B, w):
    """Padded crosses (the hyperbolic cross widened by w) serve H applications and steps
    like any tiled set: 3 steps against the oracle's propagation on the same set, on both
    step paths."""
    import torch
    from oracle.index import PaddedIndex
    tt = hh_workload(N, 0.111, 0.05)
    P = PaddedIndex(N, B, w)
    idx = hs.Index(N, B, pad=w)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    pos = P.rank(idx.multi_indices().astype(np.int64))
    c0 = complex_normal_by_index(P.k, 9)
    c0 /= np.linalg.norm(c0)
    m, h = 10, 0.01
    ref = c0.copy()
    for i in range(3):
        W = oracle_W(N, tt, i * h + 0.5 * h)
        ref, _, _, _ = lanczos_expm(lambda v: fast_apply_H(P, W, v), ref, h, m)
    for limit in (1024, 0):
        old = hs.set_small_step_rows(limit)
        c = torch.from_numpy(np.ascontiguousarray(c0[pos])).to("cuda")
        ws = hs.workspace(idx, pot, 0, m)
        for i in range(3):
            hs.step(idx, pot, c, i * h, h, m, ws=ws)
        torch.cuda.synchronize()
        hs.set_small_step_rows(old)
        got = np.empty_like(c0)
        got[pos] = c.cpu().numpy()
        assert rel2(got, ref) <= 1e-12, limit


@pytest.mark.parametrize("N", [3, 4, 5, 6, 7, 8])
def test_list_with_long_fibres(hs, N):
    """A list whose fibres along the last axis are 64 rows long ({0,1}^(N-1) x {0..63}):
    its tiles take the fused kernel's 64-row wave path (tile dimension 1, N - 1 prefix
    axes); H against the oracle on the same set."""
    import itertools
    import torch
    from oracle.index import ListIndex
    rows = np.array([p + (a,) for p in itertools.product(range(2), repeat=N - 1) for a in range(64)])
    ix = ListIndex(rows)
    tt = hh_workload(N, 0.111, 0.05)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    pot.set_time(0.2)
    idx = hs.Index(N, rows=rows)
    assert idx.tile_dim == 1 and idx.size == len(rows)
    pos = ix.rank(idx.multi_indices().astype(np.int64))
    c = complex_normal_by_index(ix.k, 90 + N)
    cl = torch.from_numpy(np.ascontiguousarray(c[pos])).to("cuda")
    yl = torch.empty_like(cl)
    hs.apply_h(idx, pot, cl, yl)
    torch.cuda.synchronize()
    y = np.empty_like(c)
    y[pos] = yl.cpu().numpy()
    assert rel2(y, fast_apply_H(ix, oracle_W(N, tt, 0.2), c)) <= 1e-12
