"""Chains of recurrence passes run per fibre (hs_index_build_fibres): the generic
program's passes along one axis (paper Sec. 3.2, eq. Horner: the basis's three-term
recurrence applied axis by axis) as one launch over the axis's fibres.  Each chain step
performs the pass's operations in the same order, so the H application and the step
with fibres equal those without bit for bit; the passes themselves are held to the
oracle by test_gpu_generic.py and test_gpu_learned (here: also against the oracle)."""
import numpy as np
import pytest

from oracle.index import IndexSet
from oracle.operators import Potential, fast_apply_H
from synth import complex_normal_by_index
from tests.hsutil import lib_to_lex, rel2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


def total_degree_terms(N, D, seed):
    rng = np.random.default_rng(seed)
    degs = []

    def rec(pre, left):
        if len(pre) == N:
            degs.append(tuple(pre))
            return
        for a in range(left + 1):
            rec(pre + [a], left - a)
    rec([], D)
    return [(float(c), d) for c, d in zip(rng.standard_normal(len(degs)) * 0.01, degs)]


# (N, B, set kind, basis, D): fibres longer than one segment (N = 2, B = 4096 and
# N = 3, B = 2048 reach 4096 and 2048 rows along an axis), boxes, total-degree sets
# N = 3 and 4 with tile dimension 1 (fibres of the last axis are whole tiles, the other
# axes are prefix axes, whose batches are laid out k-major)
CASES = [(2, 4096, "hyperbolic", "herm", 6), (3, 2048, "hyperbolic", "cheb", 5), (4, 512, "hyperbolic", "herm", 6),
         (3, 40, "box", "mono", 4), (4, 24, "total_degree", "herm", 5), (5, 256, "hyperbolic", "herm", 4),
         (3, 1500, "hyperbolic_d1", "herm", 6), (4, 1024, "hyperbolic_d1", "cheb", 6),
         (3, 300, "list", "herm", 5), (3, 200, "padded", "mono", 4)]


def make_index(hs, N, B, kind, fibres):
    if kind == "box":
        return hs.Index(N, B, box=True, fibres=fibres)
    if kind == "total_degree":
        return hs.Index(N, B, total_degree=True, fibres=fibres)
    if kind == "hyperbolic_d1":
        return hs.Index(N, B, tile_dim=1, fibres=fibres)
    if kind == "list":  # the hyperbolic cross given row by row (tile dimension 0)
        return hs.Index(N, rows=hs.Index(N, B, upload=False).multi_indices(), fibres=fibres)
    if kind == "padded":
        return hs.Index(N, B, pad=2, fibres=fibres)
    return hs.Index(N, B, fibres=fibres)


@pytest.mark.parametrize("N,B,kind,basis,D", CASES)
def test_fibre_chains_equal_the_passes(hs, N, B, kind, basis, D):
    import torch
    terms = total_degree_terms(N, D, N * 100 + D)
    scale = float(np.sqrt(2 * B) + 1) if basis == "cheb" else 1.0
    pot = hs.Pot(N, terms, basis=basis, scale=scale)
    assert not pot.fused
    plain = make_index(hs, N, B, kind, False)
    fib = make_index(hs, N, B, kind, True)
    assert fib.size == plain.size
    rng = np.random.default_rng(7)
    c0 = rng.standard_normal(plain.size) + 1j * rng.standard_normal(plain.size)
    for dt, cdt in ((hs.HS_C128, torch.complex128), (hs.HS_C64, torch.complex64)):
        c = torch.from_numpy(c0).to("cuda", cdt)
        y0, y1 = torch.empty_like(c), torch.empty_like(c)
        hs.apply_h(plain, pot, c, y0, dtype=dt)
        hs.apply_h(fib, pot, c, y1, dtype=dt)
        torch.cuda.synchronize()
        assert torch.equal(y0, y1), f"dtype {dt}"
    # a step (ten H applications inside) is the same bit for bit too
    a = torch.from_numpy(c0 / np.linalg.norm(c0)).to("cuda")
    b = a.clone()
    hs.step(plain, pot, a, 0.0, 0.01, 6)
    hs.step(fib, pot, b, 0.0, 0.01, 6)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_fibre_chains_against_the_oracle(hs):
    """The learned workload's form (N = 4, total degree 6, Hermite basis) on K_4(512)."""
    import torch
    N, B = 4, 512
    terms = total_degree_terms(N, 6, 11)
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 31)
    W = Potential(N, "herm", 1.0, [(cf, d) for cf, d in terms])
    y_ref = fast_apply_H(ix, W, c)
    idx = hs.Index(N, B, fibres=True)
    pot = hs.Pot(N, terms, basis="herm")
    lexpos = lib_to_lex(idx, N, B)
    cl = torch.from_numpy(np.ascontiguousarray(c[lexpos])).to("cuda")
    yl = torch.empty_like(cl)
    hs.apply_h(idx, pot, cl, yl)
    torch.cuda.synchronize()
    y = np.empty_like(c)
    y[lexpos] = yl.cpu().numpy()
    assert rel2(y, y_ref) <= 1e-12
    assert np.max(np.abs(y - y_ref)) <= 1e-12 * np.max(np.abs(y_ref))


def test_fibres_built_after_upload_are_not_used(hs):
    """A device block uploaded before the fibres were built lacks them: the H application
    keeps to the passes (same result) until the block is uploaded again."""
    import ctypes
    import torch
    N, B = 3, 256
    pot = hs.Pot(N, total_degree_terms(N, 5, 3), basis="herm")
    idx = hs.Index(N, B)
    n0 = ctypes.c_int64()
    hs.hs_index_device_bytes(idx.h, ctypes.byref(n0))
    hs.hs_index_build_fibres(idx.h)
    hs.hs_index_build_fibres(idx.h)  # idempotent
    n1 = ctypes.c_int64()
    hs.hs_index_device_bytes(idx.h, ctypes.byref(n1))
    assert n1.value > n0.value
    c = torch.randn(idx.size, dtype=torch.complex128, device="cuda")
    y0, y1 = torch.empty_like(c), torch.empty_like(c)
    hs.apply_h(idx, pot, c, y0)          # old block: passes
    dev = hs.dev_buffer(n1.value)
    hs.hs_index_upload(idx.h, hs.ptr(dev), n1.value, hs.stream_ptr())
    idx.dev = dev
    hs.apply_h(idx, pot, c, y1)          # new block: chains
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)


def test_fibre_step_graph_replays_equal_eager(hs):
    """A step on a set with fibres (chains, the fused combination) captured once and
    replayed, with eager work between replays, gives the eager steps bit for bit."""
    import torch
    N, B, m, h = 4, 1024, 8, 0.002
    pot = hs.Pot(N, total_degree_terms(N, 6, 17), basis="herm")
    idx = hs.Index(N, B, tile_dim=1, fibres=True)
    rng = np.random.default_rng(23)
    c0 = rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size)
    c0 /= np.linalg.norm(c0)
    ce = torch.from_numpy(c0.copy()).to("cuda")
    wse = hs.workspace(idx, pot, 0, m)
    te = torch.zeros(1, dtype=torch.float64, device="cuda")
    eager = []
    for _ in range(3):
        hs.step(idx, pot, ce, 0.0, h, m, ws=wse, t_dev=te)
        eager.append(ce.cpu().numpy().copy())
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


def test_fibre_magnus4_step_equals_the_passes(hs):
    """The fourth-order step applies H four times per Krylov vector through the generic
    program: with fibres it is the same bit for bit."""
    import torch
    N, B, m, h = 3, 600, 6, 0.005
    pot = hs.Pot(N, total_degree_terms(N, 5, 29), basis="herm")
    plain = hs.Index(N, B)
    fib = hs.Index(N, B, fibres=True)
    rng = np.random.default_rng(5)
    c0 = rng.standard_normal(plain.size) + 1j * rng.standard_normal(plain.size)
    c0 /= np.linalg.norm(c0)
    a = torch.from_numpy(c0.copy()).to("cuda")
    b = a.clone()
    hs.step_magnus4(plain, pot, a, 0.0, h, m)
    hs.step_magnus4(fib, pot, b, 0.0, h, m)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("seed", range(9))
def test_random_generic_potentials_with_fibres(hs, seed):
    """The random potentials of test_gpu_generic.py (trie and split programs, three bases,
    N = 2..5, terms accumulated into y along the way): with fibres the same bit for bit."""
    import torch
    from tests.test_gpu_generic import random_case
    N, B, basis, scale, degs, coefs = random_case(seed)
    pot = hs.Pot(N, [(float(cf), d) for cf, d in zip(coefs, degs)], basis=basis, scale=scale)
    plain = hs.Index(N, B)
    for td in (0, 1):
        fib = hs.Index(N, B, tile_dim=td, fibres=True)
        if td == 1:
            plain_td = hs.Index(N, B, tile_dim=1)
        else:
            plain_td = plain
        rng = np.random.default_rng(seed)
        c = torch.from_numpy(rng.standard_normal(fib.size) + 1j * rng.standard_normal(fib.size)).to("cuda")
        y0, y1 = torch.empty_like(c), torch.empty_like(c)
        hs.apply_h(plain_td, pot, c, y0)
        hs.apply_h(fib, pot, c, y1)
        torch.cuda.synchronize()
        assert torch.equal(y0, y1), f"seed {seed}, tile dimension {td}"
