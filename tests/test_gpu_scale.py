"""The FP32 form at scale: N = 10, product bound 4096 (103,495,890 rows), chained
Henon-Heiles lambda = 0.111 plus the laser term, packet at x_d = 0.5.  The float64 H
application is checked on sampled rows against the oracle's row-by-row evaluation
(paper Sec. 5.3 layered tree); the FP32 form (complex64 Krylov vectors and matvec,
float64 reductions) is compared with the float64 path over full steps."""
import numpy as np
import pytest

from oracle.operators import fast_H_rows
from synth import coherent_state
from tests.hsutil import hh_workload, lib_terms, oracle_W, rel2

pytestmark = pytest.mark.gpu

N, B = 10, 4096


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs
    tt = hh_workload(N, 0.111, 0.05)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(tt), subtract_harmonic=True)
    k = idx.multi_indices()
    c0 = coherent_state(k, 0.5)
    c0 /= np.linalg.norm(c0)
    return hs, tt, idx, pot, k, c0


def _vector(k):
    """Coherent packet plus a deterministic perturbation of size 1e-3 on every row, a
    closed-form function of the multi-index (so the oracle evaluates it by index)."""
    k = np.atleast_2d(np.asarray(k, dtype=np.int64))
    w1 = np.arange(1, N + 1) * 0.37
    w2 = np.arange(N, 0, -1) * 0.11
    pert = np.cos(k @ w1) + 1j * np.sin((k * k) @ w2)
    return coherent_state(k, 0.5) + 1e-3 * pert


def test_n10_float64_sampled_rows(setup):
    import torch
    hs, tt, idx, pot, k, c0 = setup
    assert idx.size == 103495890
    c_lib = np.concatenate([_vector(k[i:i + 8_000_000]) for i in range(0, len(k), 8_000_000)])
    pot.set_time(0.3)
    c = torch.from_numpy(c_lib).to("cuda")
    y = torch.empty_like(c)
    hs.apply_h(idx, pot, c, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    head = np.arange(0, 30)
    rand = rng.choice(idx.size, 90, replace=False)
    rows = np.concatenate([head, rand])
    y_lib = y[torch.from_numpy(rows).to("cuda")].cpu().numpy()
    del c, y
    lookup = lambda m: _vector(np.array(m))[0]  # noqa: E731
    y_ref = fast_H_rows(N, B, oracle_W(N, tt, 0.3), lookup, k[rows])
    assert rel2(y_lib[:30], y_ref[:30]) <= 1e-12      # rows carrying the packet
    assert rel2(y_lib[30:], y_ref[30:]) <= 1e-12      # random rows (perturbation only)


def test_n10_float32_form_error(setup):
    """10 steps of h = 0.005, m = 10: complex64 Krylov form against the float64 path
    (itself parity-checked against the oracle at smaller sizes)."""
    import torch
    hs, tt, idx, pot, k, c0 = setup
    out = {}
    for dtype in (hs.HS_C128, hs.HS_C64):
        c = torch.from_numpy(c0).to("cuda")
        ws = hs.workspace(idx, pot, dtype, 10)
        t = 0.0
        for _ in range(10):
            hs.step(idx, pot, c, t, 0.005, 10, dtype=dtype, ws=ws)
            t += 0.005
        torch.cuda.synchronize()
        out[dtype] = c
        del ws
    err = float(torch.linalg.norm(out[hs.HS_C64] - out[hs.HS_C128]) / torch.linalg.norm(out[hs.HS_C128]))
    drift = abs(float(torch.linalg.norm(out[hs.HS_C128])) - 1.0)
    print(f"N=10 B=4096, 10 steps: FP32 form relative error vs FP64 {err:.2e}; FP64 norm drift {drift:.1e}")
    assert err < 1e-5
