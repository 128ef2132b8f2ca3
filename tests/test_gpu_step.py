"""GPU parity of the exponential-midpoint Lanczos step (paper Fig. 4) against the oracle's
propagator, through the C ABI."""
import numpy as np
import pytest

from oracle.index import IndexSet
from oracle.operators import fast_apply_H
from oracle.propagate import lanczos_expm
from synth import complex_normal_by_index, coherent_state
from tests.hsutil import hh_workload, lib_terms, lib_to_lex, oracle_W, rel2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


@pytest.fixture(autouse=True, params=["one_workgroup", "general"])
def step_path(request, hs):
    """Every test of this file runs on both step paths: sets up to 1024 rows take the
    one-workgroup step by default, and a row limit of 0 sends them to the general step."""
    old = hs.set_small_step_rows(1024 if request.param == "one_workgroup" else 0)
    yield request.param
    hs.set_small_step_rows(old)


def oracle_steps(N, B, tt, c, t0, h, n, m, reorth=True):
    ix = IndexSet(N, B)
    t = t0
    for _ in range(n):
        W = oracle_W(N, tt, t + 0.5 * h)
        c, _, _, _ = lanczos_expm(lambda v: fast_apply_H(ix, W, v), c, h, m, reorth)
        t += h
    return c


def gpu_steps(hs, N, B, tt, c_lex, t0, h, n, m, dtype=0, reorth=True, use_tdev=False):
    import torch
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    lexpos = lib_to_lex(idx, N, B)
    c = torch.from_numpy(c_lex[lexpos].copy()).to("cuda")
    ws = hs.workspace(idx, pot, dtype, m)
    tdev = torch.tensor([t0], dtype=torch.float64, device="cuda") if use_tdev else None
    diag = torch.zeros(1 + 2 * m, dtype=torch.float64, device="cuda")
    t = t0
    for _ in range(n):
        hs.step(idx, pot, c, t, h, m, dtype=dtype, reorth=reorth, ws=ws, t_dev=tdev, diag=diag)
        t += h
    torch.cuda.synchronize()
    out_lib = c.cpu().numpy()
    out = np.empty_like(out_lib)
    out[lexpos] = out_lib
    return out, diag.cpu().numpy(), (tdev.cpu().numpy() if use_tdev else None)


@pytest.mark.parametrize("nsteps", [1, 100])
def test_small_config_steps(hs, nsteps):
    """N = 2, B = 64, Henon-Heiles, complex normal start (seed 0), m = 10, h = 0.01."""
    N, B = 2, 64
    tt = hh_workload(N)
    ix = IndexSet(N, B)
    c0 = complex_normal_by_index(ix.k, 0)
    ref = oracle_steps(N, B, tt, c0, 0.0, 0.01, nsteps, 10)
    got, diag, _ = gpu_steps(hs, N, B, tt, c0, 0.0, 0.01, nsteps, 10)
    assert int(diag[0]) == 10
    assert rel2(got, ref) <= (1e-12 if nsteps == 1 else 1e-10)
    # norm conservation
    assert abs(np.linalg.norm(got) - np.linalg.norm(c0)) <= 1e-12 * nsteps * np.linalg.norm(c0)


def test_time_dependent_laser_steps(hs):
    N, B = 3, 300
    tt = hh_workload(N, 0.111, 0.05)
    ix = IndexSet(N, B)
    c0 = coherent_state(ix.k, [1.0, 0.5, -0.5])
    c0 /= np.linalg.norm(c0)
    ref = oracle_steps(N, B, tt, c0, 0.1, 0.005, 5, 10)
    got, _, tdev = gpu_steps(hs, N, B, tt, c0, 0.1, 0.005, 5, 10, use_tdev=True)
    assert rel2(got, ref) <= 1e-12
    assert tdev[0] == pytest.approx(0.1 + 5 * 0.005, abs=1e-15)


def test_no_reorth_variant(hs):
    N, B = 2, 200
    tt = hh_workload(N)
    ix = IndexSet(N, B)
    c0 = complex_normal_by_index(ix.k, 5)
    ref = oracle_steps(N, B, tt, c0, 0.0, 0.01, 3, 8, reorth=False)
    got, _, _ = gpu_steps(hs, N, B, tt, c0, 0.0, 0.01, 3, 8, reorth=False)
    assert rel2(got, ref) <= 1e-12


def test_breakdown_on_eigenvector(hs):
    """W = 0 and c = e_0: beta_1 = 0, the step stops at m_eff = 1 and is exact."""
    import torch
    N, B = 3, 50
    tt = [x for x in hh_workload(N, 0.0) if sum(x.degrees) == 2]
    idx = hs.Index(N, B)
    k = idx.multi_indices()
    c_lib = np.zeros(idx.size, dtype=np.complex128)
    c_lib[np.nonzero(k.sum(axis=1) == 0)[0][0]] = 1.0
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    c = torch.from_numpy(c_lib).to("cuda")
    diag = torch.zeros(21, dtype=torch.float64, device="cuda")
    hs.step(idx, pot, c, 0.0, 0.1, 10, diag=diag)
    torch.cuda.synchronize()
    out = c.cpu().numpy()
    assert int(diag[0].item()) == 1
    assert np.allclose(out, c_lib * np.exp(-0.15j), atol=1e-15)


def test_float32_krylov_error_stated(hs):
    N, B = 3, 400
    tt = hh_workload(N, 0.111, 0.05)
    ix = IndexSet(N, B)
    c0 = complex_normal_by_index(ix.k, 9)
    ref = oracle_steps(N, B, tt, c0, 0.0, 0.005, 10, 10)
    got, _, _ = gpu_steps(hs, N, B, tt, c0, 0.0, 0.005, 10, 10, dtype=1)
    err = rel2(got, ref)
    print(f"float32 Krylov form, 10 steps: relative error vs float64 oracle {err:.3e}")
    assert err < 1e-4


def test_graph_replay_matches_eager(hs):
    """A step captured in a HIP graph (time read from and advanced on the device) gives the
    eager result on every replay, with eager work and synchronisations in between."""
    import torch
    N, B, m, h = 3, 300, 10, 0.005
    tt = hh_workload(N, 0.111, 0.05)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    k = idx.multi_indices()
    c0 = coherent_state(k, [1.0, 0.5, -0.5])
    c0 /= np.linalg.norm(c0)
    # eager reference: 4 steps
    ce = torch.from_numpy(c0.copy()).to("cuda")
    wse = hs.workspace(idx, pot, 0, m)
    te = torch.zeros(1, dtype=torch.float64, device="cuda")
    eager = []
    for _ in range(4):
        hs.step(idx, pot, ce, 0.0, h, m, ws=wse, t_dev=te)
        eager.append(ce.cpu().numpy().copy())
    # graph
    cg = torch.from_numpy(c0.copy()).to("cuda")
    wsg = hs.workspace(idx, pot, 0, m)
    tg = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    snapshot = cg.clone()
    with torch.cuda.stream(s2):
        with torch.cuda.graph(g, stream=s2):
            hs.step(idx, pot, cg, 0.0, h, m, ws=wsg, t_dev=tg)
    torch.cuda.synchronize()
    # capture does not execute: restore the start state and time
    cg.copy_(snapshot)
    tg.zero_()
    torch.cuda.synchronize()
    junk = torch.randn(1000, device="cuda")
    for i in range(4):
        g.replay()
        torch.cuda.synchronize()
        junk = junk * 1.0001 + 1.0  # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(cg.cpu().numpy(), eager[i]), f"replay {i} differs from eager"
    assert tg.item() == pytest.approx(4 * h, abs=1e-15)


@pytest.mark.parametrize("use_tdev", [False, True])
def test_propagate_equals_single_steps(hs, use_tdev):
    """hs_propagate (the paper's time_propagation: many steps in one call) gives the result
    of the same number of single steps bit for bit, with the clock on the host or on the
    device, and agrees with the oracle; zero steps leave c unchanged."""
    import torch
    N, B, m, h, n = 3, 300, 10, 0.005, 7
    tt = hh_workload(N, 0.111, 0.05)
    ix = IndexSet(N, B)
    c0 = coherent_state(ix.k, [1.0, 0.5, -0.5])
    c0 /= np.linalg.norm(c0)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    lexpos = lib_to_lex(idx, N, B)
    ws = hs.workspace(idx, pot, 0, m)
    # single steps, step i at 0.1 + i h (as hs_propagate times them)
    cs = torch.from_numpy(c0[lexpos].copy()).to("cuda")
    ts = torch.tensor([0.1], dtype=torch.float64, device="cuda") if use_tdev else None
    for i in range(n):
        hs.step(idx, pot, cs, 0.1 + i * h, h, m, ws=ws, t_dev=ts)
    torch.cuda.synchronize()
    single = np.empty_like(c0)
    single[lexpos] = cs.cpu().numpy()
    c = torch.from_numpy(c0[lexpos].copy()).to("cuda")
    tdev = torch.tensor([0.1], dtype=torch.float64, device="cuda") if use_tdev else None
    hs.propagate(idx, pot, c, 0.1, h, m, 0, ws=ws, t_dev=tdev)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), c0[lexpos])
    hs.propagate(idx, pot, c, 0.1, h, m, n, ws=ws, t_dev=tdev)
    torch.cuda.synchronize()
    got = np.empty_like(c0)
    got[lexpos] = c.cpu().numpy()
    assert np.array_equal(got, single)
    assert rel2(got, oracle_steps(N, B, tt, c0, 0.1, h, n, m)) <= 1e-12
    if use_tdev:
        assert float(tdev[0]) == pytest.approx(0.1 + n * h, abs=1e-14)


def test_propagate_captured_in_one_graph(hs):
    """Ten steps captured as one graph (clock on the device) match ten eager steps on each
    of three replays, with eager work in between."""
    import torch
    N, B, m, h, n = 2, 64, 10, 0.01, 10
    tt = hh_workload(N)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    c0 = complex_normal_by_index(idx.multi_indices(), 0)
    ce = torch.from_numpy(c0.copy()).to("cuda")
    wse = hs.workspace(idx, pot, 0, m)
    te = torch.zeros(1, dtype=torch.float64, device="cuda")
    eager = []
    for _ in range(3):
        hs.propagate(idx, pot, ce, 0.0, h, m, n, ws=wse, t_dev=te)
        eager.append(ce.cpu().numpy().copy())
    cg = torch.from_numpy(c0.copy()).to("cuda")
    wsg = hs.workspace(idx, pot, 0, m)
    tg = torch.zeros(1, dtype=torch.float64, device="cuda")
    snapshot = cg.clone()
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.stream(s2):
        with torch.cuda.graph(g, stream=s2):
            hs.propagate(idx, pot, cg, 0.0, h, m, n, ws=wsg, t_dev=tg)
    torch.cuda.synchronize()
    cg.copy_(snapshot)
    tg.zero_()
    torch.cuda.synchronize()
    junk = torch.randn(1000, device="cuda")
    for i in range(3):
        g.replay()
        torch.cuda.synchronize()
        junk = junk * 1.5 + 1.0
        torch.cuda.synchronize()
        assert np.array_equal(cg.cpu().numpy(), eager[i]), f"replay {i}"
    assert float(tg[0]) == pytest.approx(3 * n * h, abs=1e-13)


SMALL_CASES = [(1, 40), (2, 64), (3, 75), (4, 40), (5, 30), (6, 20), (7, 15), (8, 12)]


@pytest.mark.parametrize("N,B", SMALL_CASES)
def test_one_workgroup_step_agrees_with_general_step(hs, step_path, N, B):
    """Both step paths on small sets of every supported N (HH chain with the laser), FP64
    and FP32 Krylov vectors, with and without the Gram-Schmidt pass: the same m_eff,
    alpha and beta, results within rounding of each other and within 1e-12 of the oracle."""
    import torch
    if step_path != "one_workgroup":
        pytest.skip("compares the two paths itself")
    m, h = 10, 0.01
    tt = hh_workload(N, 0.111, 0.05)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    assert pot.fused and idx.size <= 1024
    ix = IndexSet(N, B)
    lexpos = lib_to_lex(idx, N, B)
    c0 = complex_normal_by_index(ix.k, 70 + N)
    c0 /= np.linalg.norm(c0)
    print("N", N, "B", B, "rows", idx.size, flush=True)
    for dtype, tol in ((0, 1e-13), (1, 1e-6)):
        for reorth in (True, False):
            out, dg = {}, {}
            for limit in (1024, 0):
                hs.set_small_step_rows(limit)
                c = torch.from_numpy(c0[lexpos].copy()).to("cuda")
                ws = hs.workspace(idx, pot, dtype, m)
                diag = torch.zeros(1 + 2 * m, dtype=torch.float64, device="cuda")
                for i in range(3):
                    hs.step(idx, pot, c, 0.2 + i * h, h, m, dtype=dtype, reorth=reorth, ws=ws, diag=diag)
                torch.cuda.synchronize()
                out[limit] = c.cpu().numpy()
                dg[limit] = diag.cpu().numpy()
            hs.set_small_step_rows(1024)
            assert dg[1024][0] == dg[0][0]
            np.testing.assert_allclose(dg[1024][1:], dg[0][1:], rtol=tol, atol=tol)
            assert rel2(out[1024], out[0]) <= tol, (dtype, reorth)
            if dtype == 0:
                got = np.empty_like(c0)
                got[lexpos] = out[1024]
                ref = oracle_steps(N, B, tt, c0, 0.2, h, 3, m, reorth)
                assert rel2(got, ref) <= 1e-12


def test_one_workgroup_step_zero_vector_and_limits(hs, step_path):
    """A zero state stays zero with m_eff = 0; the row limit decides the path (the largest
    set at the limit and the smallest one above it both agree with the oracle)."""
    import torch
    if step_path != "one_workgroup":
        pytest.skip("sets the row limit itself")
    N, B, m, h = 3, 75, 8, 0.01
    tt = hh_workload(N, 0.111, 0.05)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    c = torch.zeros(idx.size, dtype=torch.complex128, device="cuda")
    ws = hs.workspace(idx, pot, 0, m)
    diag = torch.full((1 + 2 * m,), 7.0, dtype=torch.float64, device="cuda")
    hs.step(idx, pot, c, 0.0, h, m, ws=ws, diag=diag)
    torch.cuda.synchronize()
    assert not torch.any(c != 0)
    assert float(diag[0]) == 0.0
    ix = IndexSet(N, B)
    c0 = complex_normal_by_index(ix.k, 3)
    ref = oracle_steps(N, B, tt, c0, 0.0, h, 2, m)
    for limit in (idx.size, idx.size - 1):
        hs.set_small_step_rows(limit)
        got, _, _ = gpu_steps(hs, N, B, tt, c0, 0.0, h, 2, m)
        assert rel2(got, ref) <= 1e-12, limit
    hs.set_small_step_rows(1024)


@pytest.mark.parametrize("m", [1, 2, 32])
def test_one_workgroup_step_krylov_extremes(hs, step_path, m):
    """m = 1 (one vector: the exponential of a 1x1 matrix), m = 2 and the largest m = 32 (four
    chunks of inner products): the two step paths agree and match the oracle."""
    import torch
    if step_path != "one_workgroup":
        pytest.skip("compares the two paths itself")
    N, B, h = 3, 75, 0.01
    tt = hh_workload(N, 0.111, 0.05)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    ix = IndexSet(N, B)
    lexpos = lib_to_lex(idx, N, B)
    c0 = complex_normal_by_index(ix.k, 90 + m)
    c0 /= np.linalg.norm(c0)
    out = {}
    for limit in (1024, 0):
        hs.set_small_step_rows(limit)
        c = torch.from_numpy(c0[lexpos].copy()).to("cuda")
        ws = hs.workspace(idx, pot, 0, m)
        for i in range(2):
            hs.step(idx, pot, c, i * h, h, m, ws=ws)
        torch.cuda.synchronize()
        out[limit] = c.cpu().numpy()
    hs.set_small_step_rows(1024)
    assert rel2(out[1024], out[0]) <= 1e-13
    got = np.empty_like(c0)
    got[lexpos] = out[1024]
    ref = oracle_steps(N, B, tt, c0, 0.0, h, 2, m)
    # m = 1, 2 are poor propagators; the comparison is with the oracle's same poor step
    assert rel2(got, ref) <= 1e-12
