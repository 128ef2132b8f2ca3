"""Learned coefficients on the GPU: the Gauss-Hermite projection kernel against the
oracle's projection (paper Sec. 4.1 quadrature), the BF16-MFMA network's forward,
gradients and Adam update against the float64 oracle network, training on quadrature
targets, the quadrature fallback outside the training box, the gain over the
quadrature, and propagation with surrogate coefficients."""
import math
import time

import numpy as np
import pytest

from oracle.index import IndexSet
from oracle.operators import Potential, fast_apply_H
from oracle.propagate import lanczos_expm
from oracle.surrogate import (adam_step, circle_centres, gaussian_sum_W, gh_project, mlp_backward,
                              mlp_forward, mlp_init, mse_loss, total_degree_list)
from synth import coherent_state, draw_surrogate_params, surrogate_geometry, surrogate_param_box
from tests.hsutil import lib_to_lex, rel2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


def oracle_coeffs(geom, prow, N, D, Q):
    G = geom["base"].shape[0]
    t, amps, sigma, rho, omega = prow[0], prow[1:1 + G], prow[G + 1], prow[G + 2], prow[G + 3]
    cen = circle_centres(t, rho, omega, geom["base"], geom["u"], geom["w"], geom["phase"])
    return gh_project(lambda x: gaussian_sum_W(x, amps, sigma, cen), N, D, Q)


def dev64(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float64))).to("cuda")


@pytest.mark.parametrize("N,D,Q,ns", [(4, 6, 16, 3), (4, 6, 7, 2), (3, 4, 10, 2), (2, 6, 12, 3),
                                      (1, 3, 5, 2), (4, 0, 4, 1), (4, 8, 9, 1)])
def test_gh_project_vs_oracle(hs, N, D, Q, ns):
    import torch
    if N == 1:  # circles degenerate to segments on the line
        geom = {"base": np.array([[0.3], [-0.2], [0.0]]), "u": np.ones((3, 1)), "w": np.zeros((3, 1)),
                "phase": np.array([0.1, 2.0, 4.0])}
    else:
        geom = surrogate_geometry(N, 3, seed=7)
    P = draw_surrogate_params(ns, seed=100 + N + D + Q)
    out = hs.gh_project(geom, dev64(P), D, Q)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got.shape == (ns, math.comb(N + D, N))
    for s in range(ns):
        ref = oracle_coeffs(geom, P[s], N, D, Q)
        err = np.max(np.abs(got[s] - ref)) / np.max(np.abs(ref))
        print(f"N={N} D={D} Q={Q} sample {s}: max rel err {err:.2e}")
        assert err < 1e-12


def test_gh_project_empty_and_invalid(hs):
    import torch
    geom = surrogate_geometry(4, 3, seed=7)
    out = torch.empty((0, 210), dtype=torch.float64, device="cuda")
    hs.gh_project(geom, torch.empty((0, 7), dtype=torch.float64, device="cuda"), 6, 16, out=out)
    with pytest.raises(hs.HSError):
        hs.gh_project(geom, dev64(draw_surrogate_params(1, 0)), 6, 33)
    with pytest.raises(hs.HSError):
        hs.gh_project(surrogate_geometry(5, 3, seed=7), dev64(draw_surrogate_params(1, 0)), 2, 4)


def _norms(targets):
    lo, hi = surrogate_param_box()
    mean = targets.mean(axis=0)
    std = targets.std(axis=0) + 1e-3 * np.abs(targets).max()
    return lo, hi, mean, std


def _random_params(seed, sizes):
    p = mlp_init(sizes, seed)
    rng = np.random.default_rng(seed + 1)
    for k in list(p):
        if k.startswith("b"):
            p[k] = rng.uniform(-0.1, 0.1, size=p[k].shape)
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def test_mlp_forward_vs_oracle(hs):
    import torch
    sizes = [7, 256, 256, 210]
    params = _random_params(3, sizes)
    X = draw_surrogate_params(200, seed=5)  # ragged against the 16-row tiles
    lo, hi = surrogate_param_box()
    rng = np.random.default_rng(9)
    mean, std = rng.normal(size=210), rng.uniform(0.5, 2.0, size=210)
    net = hs.MLP(7, 256, 210, max_batch=256)
    net.upload(params, lo, hi, mean, std)
    got = net.predict(dev64(X))
    torch.cuda.synchronize()
    Xn = 2.0 * (X - lo) / (hi - lo) - 1.0
    y, _ = mlp_forward(params, Xn)
    ref = y * std + mean
    yg = (got.cpu().numpy() - mean) / std
    err = rel2(yg, y)
    print(f"forward rel err (normalised outputs) {err:.2e}")
    # BF16 operands (unit roundoff 2^-8), FP32 accumulation over K <= 256
    assert err < 2e-2
    assert np.max(np.abs(got.cpu().numpy() - ref) / std) < 0.1


def test_mlp_gradients_and_adam_vs_oracle(hs):
    import torch
    sizes = [7, 256, 256, 210]
    params = _random_params(4, sizes)
    X = draw_surrogate_params(256, seed=6)
    lo, hi = surrogate_param_box()
    rng = np.random.default_rng(10)
    mean, std = rng.normal(size=210), rng.uniform(0.5, 2.0, size=210)
    T = mean + std * rng.normal(size=(256, 210))
    net = hs.MLP(7, 256, 210, max_batch=256)
    net.upload(params, lo, hi, mean, std)
    grads = torch.zeros(net.nparam, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    Xd, Td = dev64(X), dev64(T)
    lr = 1e-3
    net.train_step(Xd, Td, lr, loss=loss, grads=grads)
    torch.cuda.synchronize()
    g_gpu = net.unflatten(grads.cpu().numpy().astype(np.float64))
    # oracle gradients at the same weights
    Xn = 2.0 * (X - lo) / (hi - lo) - 1.0
    Tn = (T - mean) / std
    y, cache = mlp_forward(params, Xn)
    g_ref = mlp_backward(params, cache, y, Tn)
    assert float(loss.item()) == pytest.approx(mse_loss(y, Tn), rel=2e-2)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        e = rel2(g_gpu[k], g_ref[k])
        print(f"grad {k}: rel err {e:.2e}")
        assert e < 5e-2, k
    # Adam: the oracle's update applied to the GPU's gradients (two steps: bias correction)
    state = {}
    p_ref = adam_step(dict(params), g_gpu, state, lr=lr)
    w1 = net.download()
    for k in p_ref:
        assert np.max(np.abs(w1[k] - p_ref[k])) < 2e-6, k
    net.train_step(Xd, Td, lr, loss=loss, grads=grads)
    torch.cuda.synchronize()
    g2 = net.unflatten(grads.cpu().numpy().astype(np.float64))
    p_ref = adam_step({k: w1[k].astype(np.float64) for k in w1}, g2, state, lr=lr)
    w2 = net.download()
    for k in p_ref:
        assert np.max(np.abs(w2[k] - p_ref[k])) < 2e-6, k


@pytest.fixture(scope="module")
def trained(hs):
    """Network trained on Q = 16 quadrature targets (4096 draws), N = 4, D = 6."""
    import torch
    N, D, Q = 4, 6, 16
    geom = surrogate_geometry(N, 3, seed=7)
    Ptr = draw_surrogate_params(4096, seed=11)
    Pd = dev64(Ptr)
    Td = hs.gh_project(geom, Pd, D, Q)
    torch.cuda.synchronize()
    T = Td.cpu().numpy()
    lo, hi, mean, std = _norms(T)
    net = hs.MLP(7, 256, 210, max_batch=4096)
    net.upload(_random_params(21, [7, 256, 256, 210]), lo, hi, mean, std)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    g = torch.Generator(device="cpu").manual_seed(0)
    losses = []
    nsteps, bs = 12000, 256
    for it in range(nsteps):
        sel = torch.randint(0, 4096, (bs,), generator=g).to("cuda")
        lr = 2e-3 * 0.5 * (1 + math.cos(math.pi * it / nsteps)) + 1e-5
        net.train_step(Pd[sel].contiguous(), Td[sel].contiguous(), lr, loss=loss)
        if it % 500 == 0 or it == nsteps - 1:
            losses.append(float(loss.item()))
    print("training loss", ["%.2e" % v for v in losses])
    return dict(net=net, geom=geom, N=N, D=D, Q=Q, losses=losses, lo=lo, hi=hi)


def test_training_reduces_loss(trained):
    L = trained["losses"]
    assert L[-1] < 3e-2 * L[0]


def test_surrogate_accuracy_and_gain(hs, trained):
    """Held-out error of the network against the quadrature reference, and the time per
    batch of coefficients: the network against the quadrature at the reference's Q and at
    the smallest Q that is as accurate as the network."""
    import torch
    net, geom, D = trained["net"], trained["geom"], trained["D"]
    Pv = dev64(draw_surrogate_params(256, seed=12))
    ref24 = hs.gh_project(geom, Pv, D, 24)
    pred = net.predict(Pv)
    torch.cuda.synchronize()
    J = ref24.cpu().numpy()
    scale = np.linalg.norm(J, axis=1)
    e_mlp = float(np.median(np.linalg.norm(pred.cpu().numpy() - J, axis=1) / scale))
    errs = {}
    for Q in range(2, 17):
        c = hs.gh_project(geom, Pv, D, Q).cpu().numpy()
        errs[Q] = float(np.median(np.linalg.norm(c - J, axis=1) / scale))
    # the cheapest quadrature at least as accurate as the network
    q_match = min([Q for Q in errs if errs[Q] <= e_mlp] or [16])

    def timeit(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    out = torch.empty_like(ref24)
    t_mlp = timeit(lambda: net.predict(Pv, out=out))
    t_q16 = timeit(lambda: hs.gh_project(geom, Pv, D, 16, out=out))
    t_qm = timeit(lambda: hs.gh_project(geom, Pv, D, q_match, out=out))
    print(f"median rel err: network {e_mlp:.2e}; quadrature " +
          " ".join(f"Q={q}:{e:.1e}" for q, e in errs.items()))
    print(f"256 coefficient sets: network {t_mlp*1e6:.1f} us, quadrature Q=16 {t_q16*1e6:.1f} us, "
          f"quadrature Q={q_match} (as accurate as the network) {t_qm*1e6:.1f} us")
    assert e_mlp < 2e-2
    assert errs[16] < 1e-6
    assert q_match > 2  # the network beats the coarsest rule
    # the gain: the network is faster than the quadrature of the same accuracy
    assert t_mlp < t_qm


def test_fallback_outside_box(hs, trained):
    import torch
    net, geom, D, Q = trained["net"], trained["geom"], trained["D"], trained["Q"]
    P = draw_surrogate_params(8, seed=13)
    P[1, 4] = 2.5   # sigma above the box
    P[5, 0] = -1.0  # time below the box
    Pd = dev64(P)
    used = torch.full((8,), -1, dtype=torch.int32, device="cuda")
    c = net.coeffs(geom, Pd, D, Q, used=used)
    ref_q = hs.gh_project(geom, Pd, D, Q)
    ref_n = net.predict(Pd)
    torch.cuda.synchronize()
    u = used.cpu().numpy()
    assert list(u) == [0, 1, 0, 0, 0, 1, 0, 0]
    c, ref_q, ref_n = c.cpu().numpy(), ref_q.cpu().numpy(), ref_n.cpu().numpy()
    for s in range(8):
        assert np.array_equal(c[s], ref_q[s] if u[s] else ref_n[s])


def _learned_pot(hs, N, D):
    return hs.Pot(N, [(0.0, a) for a in total_degree_list(N, D)], basis="herm")


def test_learned_workload_steps(hs, trained):
    """Propagation with device-set coefficients (quadrature or network, recomputed at the
    midpoint of every step) against the oracle's propagator.  The degree-6 expansion makes
    |H| grow quickly with the bound (about 5e3 at B = 64, 5e5 at B = 256), and the
    10-dimensional Krylov step is well conditioned only while h |H| stays near m: B = 64,
    h = 0.002 (a relative 1e-14 change of the coefficients moves the result by about 2e-15
    here, by 1e-4 at B = 256, h = 0.01)."""
    import torch
    net, geom, D, Q = trained["net"], trained["geom"], trained["D"], trained["Q"]
    N, B = 4, 64
    degs = total_degree_list(N, D)
    prow = draw_surrogate_params(1, seed=14)[0]
    h, m, nsteps = 0.002, 10, 10
    ix = IndexSet(N, B)
    c0 = coherent_state(ix.k, np.array([0.5, 0.0, -0.3, 0.2]))

    def run(source):
        idx = hs.Index(N, B)
        pot = _learned_pot(hs, N, D)
        lexpos = lib_to_lex(idx, N, B)
        c = torch.from_numpy(c0[lexpos].copy()).to("cuda")
        ws = hs.workspace(idx, pot, hs.HS_C128, m)
        P = dev64(prow[None, :].copy())
        coef = torch.empty((1, len(degs)), dtype=torch.float64, device="cuda")
        t, used = 0.0, []
        for _ in range(nsteps):
            P[0, 0] = t + 0.5 * h
            if source == "net":
                net.coeffs(geom, P, D, Q, out=coef)
            else:
                hs.gh_project(geom, P, D, Q, out=coef)
            pot.set_coeffs_device(coef[0])
            hs.step(idx, pot, c, t, h, m, ws=ws)
            used.append(coef[0].cpu().numpy().copy())
            t += h
        torch.cuda.synchronize()
        out = np.empty_like(c0)
        out[lexpos] = c.cpu().numpy()
        return out, used

    got, used = run("quad")
    c = c0.copy()
    for k in range(nsteps):
        W = Potential(N, "herm", 1.0, list(zip(used[k], degs)))
        c, _, _, _ = lanczos_expm(lambda v: fast_apply_H(ix, W, v), c, h, m, True)
    assert rel2(got, c) < 1e-12
    cn, _ = run("net")
    d = rel2(cn, got)
    print(f"B={B}, {nsteps} steps of h={h}: network vs quadrature coefficients, rel diff {d:.2e}")
    assert d < 1e-2


def test_learned_workload_matvec_full_size(hs, trained):
    """N = 4, B = 8192 (1,510,397 rows): H c with network coefficients on sampled rows
    against the oracle's row-by-row evaluation, and the change of H c between network and
    quadrature coefficients."""
    import torch
    from oracle.index import LexRanker
    from oracle.operators import fast_H_rows
    net, geom, D, Q = trained["net"], trained["geom"], trained["D"], trained["Q"]
    N, B = 4, 8192
    degs = total_degree_list(N, D)
    idx = hs.Index(N, B)
    k = idx.multi_indices()
    c_lib = coherent_state(k, np.array([0.5, 0.0, -0.3, 0.2]))
    c_lib /= np.linalg.norm(c_lib)
    P = dev64(draw_surrogate_params(1, seed=15))
    cn = net.coeffs(geom, P, D, Q)
    cq = hs.gh_project(geom, P, D, Q)
    c = torch.from_numpy(c_lib).to("cuda")
    out = {}
    for name, cf in (("net", cn), ("quad", cq)):
        pot = _learned_pot(hs, N, D)
        pot.set_coeffs_device(cf[0])
        y = torch.empty_like(c)
        hs.apply_h(idx, pot, c, y)
        torch.cuda.synchronize()
        out[name] = y.cpu().numpy()
    alpha = cn[0].cpu().numpy()
    lexpos = LexRanker(N, B).rank(k.astype(np.int64))
    inv = np.empty_like(lexpos)
    inv[lexpos] = np.arange(lexpos.size)
    ranker = LexRanker(N, B)
    lookup = lambda m: c_lib[inv[ranker.rank(np.array(m))[0]]]  # noqa: E731
    rng = np.random.default_rng(3)
    rows = np.concatenate([np.arange(0, 12), rng.choice(idx.size, 12, replace=False)])
    y_ref = fast_H_rows(N, B, Potential(N, "herm", 1.0, list(zip(alpha, degs))), lookup, k[rows])
    assert rel2(out["net"][rows], y_ref) < 1e-12
    d = rel2(out["net"], out["quad"])
    print(f"B={B}: H c with network vs quadrature coefficients, rel diff {d:.2e}")
    assert d < 5e-2
