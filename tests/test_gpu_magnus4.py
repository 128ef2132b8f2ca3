"""The fourth-order two-stage Gauss-Legendre Magnus scheme on the GPU (paper Sec. 2.1,
eq. 2stageMagnus) against the oracle: the operator M = (A_1 + A_2)/2 - i (sqrt(3) h/12)
[A_2, A_1] applied to a vector, full Lanczos steps, the paper's time-integration
workload (Sec. 6.3, Fig. 13), the FP32 form, and at the benchmark's size sampled rows of
M c plus the exact reduction to the midpoint step for a constant potential."""
import math

import numpy as np
import pytest

from oracle.index import IndexSet
from oracle.operators import Potential, fast_apply_H, fast_H_rows
from oracle.propagate import magnus4_operator, propagate
from synth import coherent_state, complex_normal_by_index, decay_vector, stretched_hh_cw_laser
from tests.hsutil import hh_workload, lib_terms, lib_to_lex, oracle_W, rel2

pytestmark = pytest.mark.gpu

C1 = 0.5 - math.sqrt(3.0) / 6.0
C2 = 0.5 + math.sqrt(3.0) / 6.0


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


def _set_blocks(hs, pot, t1, t2):
    d1, d2 = pot.blocks2()
    hs.hs_pot_set_time(pot.h, hs.ptr(d1), float(t1), None, hs.stream_ptr())
    hs.hs_pot_set_time(pot.h, hs.ptr(d2), float(t2), None, hs.stream_ptr())


def _to_lib(idx, N, B, c_lex):
    import torch
    lexpos = lib_to_lex(idx, N, B)
    return torch.from_numpy(np.ascontiguousarray(c_lex[lexpos])).to("cuda"), lexpos


def _from_lib(t, lexpos):
    out = np.empty(t.shape[0], dtype=np.complex128)
    out[lexpos] = t.cpu().numpy().astype(np.complex128)
    return out


def _drive_terms(N, kind):
    """Fused-class potentials: 'laser' (time-dependent linear terms only, harmonic part
    subtracted), 'cubic' (the cubic coupling itself oscillates), 'x2' (laser, harmonic
    part kept, so x_l^2 coefficients are present)."""
    tt = hh_workload(N, 0.111, 0.05)
    if kind == "cubic":
        from synth import TimeTerm
        tt = [TimeTerm(x[0], x.degrees, amp=0.04, freq=1.3, phase=0.2) if sum(x.degrees) == 3 else x
              for x in tt]
    return tt, kind != "x2"


def _oracle_pot(N, tt, t, harmonic):
    V = Potential(N, "mono", 1.0, [(x.coef(t), x.degrees) for x in tt])
    return oracle_W(N, tt, t) if harmonic else V


@pytest.mark.parametrize("N,B,kind", [(2, 700, "laser"), (3, 300, "laser"), (5, 64, "laser"),
                                      (3, 300, "cubic"), (4, 150, "x2"), (6, 300, "cubic")])
def test_apply_m_fused(hs, N, B, kind):
    """y = M c for fused-class potentials (the two fused passes): several tiles and a
    ragged tail; h = 0.5 so the commutator carries weight."""
    import torch
    tt, harmonic = _drive_terms(N, kind)
    t, h = 0.4, 0.5
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 20 + N)
    W1, W2 = _oracle_pot(N, tt, t + C1 * h, harmonic), _oracle_pot(N, tt, t + C2 * h, harmonic)
    y_ref = magnus4_operator(lambda v: fast_apply_H(ix, W1, v), lambda v: fast_apply_H(ix, W2, v), h)(c)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=harmonic)
    assert pot.fused
    _set_blocks(hs, pot, t + C1 * h, t + C2 * h)
    cl, lexpos = _to_lib(idx, N, B, c)
    yl = torch.empty_like(cl)
    hs.apply_magnus4(idx, pot, h, cl, yl)
    torch.cuda.synchronize()
    y = _from_lib(yl, lexpos)
    assert rel2(y, y_ref) <= 1e-12
    # the commutator's share lies far above the tolerance, so dropping it would fail
    comm = y_ref - 0.5 * (fast_apply_H(ix, W1, c) + fast_apply_H(ix, W2, c))
    assert np.linalg.norm(comm) > 1e4 * 1e-12 * np.linalg.norm(y_ref)


def test_apply_m_generic(hs):
    """A potential outside the fused class, time-dependent through two terms."""
    import torch
    N, B = 3, 200
    degs = [(4, 0, 0), (1, 2, 0), (0, 1, 1), (0, 0, 2), (1, 0, 0)]
    rng = np.random.default_rng(31)
    base = rng.standard_normal(len(degs)) * 0.01
    amp = [0.0, 0.02, 0.0, 0.0, 0.05]
    terms = [(float(b), a, 1.5, 0.3, d) for b, a, d in zip(base, amp, degs)]

    def W_at(t):
        return Potential(N, "mono", 1.0, [(b + a * math.sin(1.5 * t + 0.3), d)
                                           for b, a, d in zip(base, amp, degs)])
    t, h = 0.2, 0.4
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 33)
    W1, W2 = W_at(t + C1 * h), W_at(t + C2 * h)
    y_ref = magnus4_operator(lambda v: fast_apply_H(ix, W1, v), lambda v: fast_apply_H(ix, W2, v), h)(c)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, terms)
    assert not pot.fused
    _set_blocks(hs, pot, t + C1 * h, t + C2 * h)
    cl, lexpos = _to_lib(idx, N, B, c)
    yl = torch.empty_like(cl)
    hs.apply_magnus4(idx, pot, h, cl, yl)
    torch.cuda.synchronize()
    assert rel2(_from_lib(yl, lexpos), y_ref) <= 1e-12


@pytest.mark.parametrize("reorth", [True, False])
def test_steps_against_oracle(hs, reorth):
    import torch
    N, B, m, h, n = 3, 300, 8, 0.02, 5
    tt = hh_workload(N, 0.111, 0.05)
    ix = IndexSet(N, B)
    c0 = coherent_state(ix.k, [0.8, -0.4, 0.3])
    c0 /= np.linalg.norm(c0)
    ref, meffs = propagate(ix, lambda t: oracle_W(N, tt, t), lambda W: (lambda v: fast_apply_H(ix, W, v)),
                           c0, 0.0, h, n, m, reorth=reorth, scheme=4)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    c, lexpos = _to_lib(idx, N, B, c0)
    ws = hs.workspace_magnus4(idx, pot, hs.HS_C128, m)
    diag = torch.zeros(1 + 2 * m, dtype=torch.float64, device="cuda")
    t = 0.0
    for _ in range(n):
        hs.step_magnus4(idx, pot, c, t, h, m, reorth=reorth, ws=ws, diag=diag)
        t += h
    torch.cuda.synchronize()
    assert int(diag[0].item()) == meffs[-1] == m
    assert rel2(_from_lib(c, lexpos), ref) <= 1e-11


def test_graph_replay_matches_eager(hs):
    """A fourth-order step captured in a HIP graph (time read from and advanced on the
    device) gives the eager result on every replay, with eager work and
    synchronisations between the replays."""
    import torch
    N, B, m, h = 2, 500, 6, 0.05
    tt = hh_workload(N, 0.111, 0.05)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    pot.blocks2()
    k = idx.multi_indices()
    c0 = coherent_state(k, 0.7)
    c0 /= np.linalg.norm(c0)
    ce = torch.from_numpy(c0.copy()).to("cuda")
    wse = hs.workspace_magnus4(idx, pot, hs.HS_C128, m)
    te = torch.zeros(1, dtype=torch.float64, device="cuda")
    eager = []
    for _ in range(3):
        hs.step_magnus4(idx, pot, ce, 0.0, h, m, ws=wse, t_dev=te)
        eager.append(ce.cpu().numpy().copy())
    cg = torch.from_numpy(c0.copy()).to("cuda")
    wsg = hs.workspace_magnus4(idx, pot, hs.HS_C128, m)
    tg = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    snapshot = cg.clone()
    with torch.cuda.stream(s2):
        with torch.cuda.graph(g, stream=s2):
            hs.step_magnus4(idx, pot, cg, 0.0, h, m, ws=wsg, t_dev=tg)
    torch.cuda.synchronize()
    cg.copy_(snapshot)
    tg.zero_()
    torch.cuda.synchronize()
    junk = torch.randn(1000, device="cuda")
    for i in range(3):
        g.replay()
        torch.cuda.synchronize()
        junk = junk * 1.0001 + 1.0
        torch.cuda.synchronize()
        assert np.array_equal(cg.cpu().numpy(), eager[i]), f"replay {i} differs from eager"
    assert tg.item() == pytest.approx(3 * h, abs=1e-15)


def test_fig13_workload(hs):
    """The paper's time-integration workload (stretched Henon-Heiles with the CW laser,
    N = 2, K = 40, m = 7, no reorthogonalisation), 10 steps of h = 1/10 to t = 1."""
    import torch
    N, K, m, h = 2, 40, 7, 0.1
    tt = stretched_hh_cw_laser(N)
    ix = IndexSet(N, K + 1)
    c0 = decay_vector(ix.k, 3.0)
    c0 /= np.linalg.norm(c0)
    pot_at = lambda t: Potential(N, "mono", 1.0, [(x.coef(t), x.degrees) for x in tt])  # noqa: E731
    ref, _ = propagate(ix, pot_at, lambda W: (lambda v: fast_apply_H(ix, W, v)), c0, 0.0, h, 10, m,
                       reorth=False, scheme=4)
    idx = hs.Index(N, K + 1)
    pot = hs.Pot(N, lib_terms(tt))
    c, lexpos = _to_lib(idx, N, K + 1, c0)
    t = 0.0
    for _ in range(10):
        hs.step_magnus4(idx, pot, c, t, h, m, reorth=False)
        t += h
    torch.cuda.synchronize()
    got = _from_lib(c, lexpos)
    assert rel2(got, ref) <= 1e-11
    assert np.max(np.abs(got - ref)) <= 1e-12


def test_float32_form(hs):
    """complex64 Krylov vectors and float32 H applications against the float64 path."""
    import torch
    N, B, m, h = 4, 400, 8, 0.02
    tt = hh_workload(N, 0.111, 0.05)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    k = idx.multi_indices()
    c0 = coherent_state(k, 0.5)
    c0 /= np.linalg.norm(c0)
    out = {}
    for dt in (hs.HS_C128, hs.HS_C64):
        c = torch.from_numpy(c0).to("cuda")
        t = 0.0
        for _ in range(5):
            hs.step_magnus4(idx, pot, c, t, h, m, dtype=dt)
            t += h
        torch.cuda.synchronize()
        out[dt] = c.cpu().numpy()
    assert rel2(out[hs.HS_C64], out[hs.HS_C128]) < 1e-5


def _vec(k):
    """Packet plus a deterministic perturbation with integer-residue phases (bit-identical
    however rows are batched)."""
    k = np.atleast_2d(np.asarray(k, dtype=np.int64))
    n = k.shape[1]
    r1 = (k @ np.arange(3, 3 + 2 * n, 2, dtype=np.int64)) % 97
    r2 = ((k * k) @ np.arange(n, 0, -1, dtype=np.int64)) % 89
    return coherent_state(k, 0.5) + 1e-3 * (np.cos(2 * np.pi * r1 / 97.0) + 1j * np.sin(2 * np.pi * r2 / 89.0))


def test_bench_size_sampled_rows(hs):
    """N = 6, product bound 4096 (the benchmark's set): sampled rows of M c against the
    oracle's row-by-row evaluation of A_2 (A_1 c) and A_1 (A_2 c)."""
    import torch
    N, B, t, h = 6, 4096, 0.3, 0.4
    tt = hh_workload(N, 0.111, 0.05)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    k = idx.multi_indices()
    c = torch.from_numpy(np.concatenate([_vec(k[i:i + 4_000_000]) for i in range(0, len(k), 4_000_000)])).to("cuda")
    y = torch.empty_like(c)
    _set_blocks(hs, pot, t + C1 * h, t + C2 * h)
    hs.apply_magnus4(idx, pot, h, c, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    rows = np.concatenate([np.arange(0, 6), rng.choice(idx.size, 10, replace=False), [idx.size - 1]])
    y_lib = y[torch.from_numpy(rows).to("cuda")].cpu().numpy()
    del c, y
    W1, W2 = oracle_W(N, tt, t + C1 * h), oracle_W(N, tt, t + C2 * h)
    vlook = lambda m: _vec(np.array(m))[0]  # noqa: E731
    memo = ({}, {})

    def inner(j, W):
        def look(m):
            if m not in memo[j]:
                memo[j][m] = fast_H_rows(N, B, W, vlook, [m])[0]
            return memo[j][m]
        return look
    kk = k[rows]
    u1 = fast_H_rows(N, B, W1, vlook, kk)
    u2 = fast_H_rows(N, B, W2, vlook, kk)
    z = fast_H_rows(N, B, W2, inner(0, W1), kk)
    w = fast_H_rows(N, B, W1, inner(1, W2), kk)
    y_ref = 0.5 * (u1 + u2) - 1j * (math.sqrt(3.0) * h / 12.0) * (z - w)
    assert rel2(y_lib, y_ref) <= 1e-12


def test_constant_potential_equals_midpoint_step(hs):
    """Without time dependence A_1 = A_2: the GPU's commutator is exactly zero and the
    fourth-order step reproduces the midpoint step (benchmark size) to rounding: the
    fused Magnus passes and the midpoint step's H application evaluate the same rows with
    different row codes (operation order)."""
    import torch
    N, B, m, h = 6, 4096, 6, 0.01
    tt = hh_workload(N, 0.111, 0.0)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    k = idx.multi_indices()
    c0 = torch.from_numpy(np.concatenate([coherent_state(k[i:i + 4_000_000], 0.5)
                                          for i in range(0, len(k), 4_000_000)])).to("cuda")
    c0 /= torch.linalg.norm(c0)
    a = c0.clone()
    b = c0.clone()
    hs.step(idx, pot, a, 0.0, h, m, reorth=True)
    hs.step_magnus4(idx, pot, b, 0.0, h, m, reorth=True)
    torch.cuda.synchronize()
    assert float(torch.linalg.norm(a - b) / torch.linalg.norm(a)) <= 1e-14
    assert float((a - b).abs().max() / a.abs().max()) <= 1e-14


@pytest.mark.parametrize("case", ["m1", "h0", "zero"])
def test_degenerate_steps(hs, case):
    """m = 1 (c <- exp(-i h alpha_0) c), h = 0 (the identity) and the zero vector
    (m_eff = 0, c stays 0) through the fourth-order step, against the oracle."""
    import torch
    N, B = 3, 120
    tt = hh_workload(N, 0.111, 0.05)
    ix = IndexSet(N, B)
    c0 = coherent_state(ix.k, [0.5, 0.2, -0.1])
    c0 /= np.linalg.norm(c0)
    if case == "zero":
        c0 = np.zeros_like(c0)
    m, h = (1, 0.05) if case == "m1" else (6, 0.0 if case == "h0" else 0.05)
    ref, meffs = propagate(ix, lambda t: oracle_W(N, tt, t), lambda W: (lambda v: fast_apply_H(ix, W, v)),
                           c0, 0.0, h, 1, m, scheme=4)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    c, lexpos = _to_lib(idx, N, B, c0)
    diag = torch.full((1 + 2 * m,), -1.0, dtype=torch.float64, device="cuda")
    hs.step_magnus4(idx, pot, c, 0.0, h, m, diag=diag)
    torch.cuda.synchronize()
    got = _from_lib(c, lexpos)
    assert int(diag[0].item()) == meffs[0]
    if case == "zero":
        assert np.max(np.abs(got)) == 0.0
    elif case == "h0":
        assert rel2(got, c0) <= 1e-14
    else:
        assert rel2(got, ref) <= 1e-12
