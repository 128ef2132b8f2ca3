"""Batched form: one persistent launch over many instances of uneven N and B.  Checked
against the per-instance path (bit for bit: the same row code and the same segment
reductions) and against the oracle, plus autotuning and graph replay."""
import numpy as np
import pytest

from oracle.index import IndexSet
from oracle.operators import fast_apply_H
from oracle.propagate import lanczos_expm
from synth import batch_instances, complex_normal_by_index, henon_heiles_chain
from tests.hsutil import lib_terms, lib_to_lex, oracle_W, rel2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


def make_batch(hs, draws):
    idxs, pots, ks, cs = [], [], [], []
    for d in draws:
        idx = hs.Index(d["N"], d["B"])
        pot = hs.Pot(d["N"], lib_terms(henon_heiles_chain(d["N"], d["lam"])), subtract_harmonic=True)
        k = idx.multi_indices()
        idxs.append(idx)
        pots.append(pot)
        ks.append(k)
        cs.append(complex_normal_by_index(k, d["seed"]))
    return idxs, pots, ks, cs


def pack(b, cs):
    import torch
    x = np.zeros(b.total, dtype=np.complex128)
    for i, c in enumerate(cs):
        x[b.offsets[i]:b.offsets[i] + c.size] = c
    return torch.from_numpy(x).to("cuda")


# a small seeded draw of the batched workload's distribution: N in 3..8, B log-uniform
DRAWS = batch_instances(12, seed=11, log2_bmax=10.5)


def test_batched_apply_equals_per_instance_bitwise(hs):
    import torch
    idxs, pots, ks, cs = make_batch(hs, DRAWS)
    b = hs.Batch(idxs, pots)
    x = pack(b, cs)
    y = torch.zeros_like(x)
    b.apply_h(x, y)
    yb = y.cpu().numpy()
    for i, (idx, pot, c) in enumerate(zip(idxs, pots, cs)):
        ci = torch.from_numpy(c).to("cuda")
        yi = torch.empty_like(ci)
        hs.apply_h(idx, pot, ci, yi)
        torch.cuda.synchronize()
        seg = yb[b.offsets[i]:b.offsets[i] + c.size]
        assert np.array_equal(seg, yi.cpu().numpy()), f"instance {i} (N={idx.N}, B={idx.B}) differs"


def test_batched_apply_vs_oracle(hs):
    import torch
    draws = DRAWS[:6]
    idxs, pots, ks, cs = make_batch(hs, draws)
    b = hs.Batch(idxs, pots)
    x = pack(b, cs)
    y = torch.zeros_like(x)
    b.apply_h(x, y)
    yb = y.cpu().numpy()
    for i, d in enumerate(draws):
        ix = IndexSet(d["N"], d["B"])
        lexpos = lib_to_lex(idxs[i], d["N"], d["B"])
        c_lex = np.empty_like(cs[i])
        c_lex[lexpos] = cs[i]
        ref = fast_apply_H(ix, oracle_W(d["N"], henon_heiles_chain(d["N"], d["lam"]), 0.0), c_lex)
        got = np.empty_like(ref)
        got[lexpos] = yb[b.offsets[i]:b.offsets[i] + cs[i].size]
        assert rel2(got, ref) <= 1e-12


def test_batched_step_equals_per_instance_and_oracle(hs):
    import torch
    m, h = 10, 0.01
    idxs, pots, ks, cs = make_batch(hs, DRAWS)
    b = hs.Batch(idxs, pots)
    x = pack(b, cs)
    ws = b.workspace(m)
    for _ in range(2):
        b.step(x, 0.0, h, m, ws=ws)
    xb = x.cpu().numpy()
    for i, (idx, pot, c) in enumerate(zip(idxs, pots, cs)):
        ci = torch.from_numpy(c.copy()).to("cuda")
        wsi = hs.workspace(idx, pot, 0, m)
        for _ in range(2):
            hs.step(idx, pot, ci, 0.0, h, m, ws=wsi)
        torch.cuda.synchronize()
        seg = xb[b.offsets[i]:b.offsets[i] + c.size]
        ref_i = ci.cpu().numpy()
        assert rel2(seg, ref_i) <= 1e-13, f"instance {i}: batched vs per-instance"
    # two instances against the oracle propagator
    for i in (0, 5):
        d = DRAWS[i]
        ix = IndexSet(d["N"], d["B"])
        lexpos = lib_to_lex(idxs[i], d["N"], d["B"])
        c_lex = np.empty_like(cs[i])
        c_lex[lexpos] = cs[i]
        W = oracle_W(d["N"], henon_heiles_chain(d["N"], d["lam"]), 0.0)
        for _ in range(2):
            c_lex, _, _, _ = lanczos_expm(lambda v: fast_apply_H(ix, W, v), c_lex, h, m)
        got = np.empty_like(c_lex)
        got[lexpos] = xb[b.offsets[i]:b.offsets[i] + cs[i].size]
        assert rel2(got, c_lex) <= 1e-12


def test_autotune_and_graph_replay(hs):
    import torch
    m, h = 8, 0.01
    idxs, pots, ks, cs = make_batch(hs, DRAWS[:8])
    b = hs.Batch(idxs, pots)
    x = pack(b, cs)
    y = torch.zeros_like(x)
    wg, pc = b.autotune(x, y)
    assert wg in (64, 128, 256) and pc in (2, 4, 8, 16)
    order, rows = b.tuning()
    assert order in (0, 1) and rows
    for (_, _, kind, items, w, p, gr) in rows:
        assert kind in (0, 1) and items > 0 and w in (64, 128, 256) and p in (2, 4, 8, 16) and gr in (1, 2, 4)
    b.apply_h(x, y)
    y_ref = y.clone()
    # whatever order and launches the tuning chose, each instance still equals its own
    # single-instance application bit for bit
    yb = y.cpu().numpy()
    for i, (idx, pot, c) in enumerate(zip(idxs, pots, cs)):
        ci = torch.from_numpy(c).to("cuda")
        yi = torch.empty_like(ci)
        hs.apply_h(idx, pot, ci, yi)
        torch.cuda.synchronize()
        assert np.array_equal(yb[b.offsets[i]:b.offsets[i] + c.size], yi.cpu().numpy()), i
    # eager steps
    xe = x.clone()
    ws = b.workspace(m)
    eager = []
    for _ in range(3):
        b.step(xe, 0.0, h, m, ws=ws)
        eager.append(xe.cpu().numpy().copy())
    # captured step replayed
    xg = x.clone()
    wsg = b.workspace(m)
    tg = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    s2 = torch.cuda.Stream()
    s2.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    snap = xg.clone()
    with torch.cuda.stream(s2):
        with torch.cuda.graph(g, stream=s2):
            b.step(xg, 0.0, h, m, ws=wsg, t_dev=tg)
    torch.cuda.synchronize()
    xg.copy_(snap)
    torch.cuda.synchronize()
    for i in range(3):
        g.replay()
        torch.cuda.synchronize()
        b.apply_h(x, y)  # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(xg.cpu().numpy(), eager[i]), f"replay {i}"
    assert torch.equal(y, y_ref)


def test_batch_refuses_other_forms_and_sets(hs):
    """Batches serve the paper's operator form on hyperbolic sets: a symmetrised
    potential or a box set is refused at creation, and a form set after creation is
    refused at the next call instead of being ignored."""
    import torch
    draws = DRAWS[:2]
    idxs, pots, ks, cs = make_batch(hs, draws)
    pots[1].set_form(hs.HS_FORM_SYM)
    with pytest.raises(hs.HSError) as e:
        hs.Batch(idxs, pots)
    assert e.value.code == -5
    pots[1].set_form(hs.HS_FORM_PAPER)
    box = hs.Index(draws[0]["N"], 6, box=True)
    with pytest.raises(hs.HSError):
        hs.Batch([box], pots[:1])
    b = hs.Batch(idxs, pots)
    x = pack(b, cs)
    y = torch.empty_like(x)
    b.apply_h(x, y)
    pots[0].set_form(hs.HS_FORM_SYM)
    with pytest.raises(hs.HSError) as e:
        b.apply_h(x, y)
    assert e.value.code == -5
    pots[0].set_form(hs.HS_FORM_PAPER)
    b.apply_h(x, y)
    torch.cuda.synchronize()


def test_full_range_draw_with_size_rule(hs):
    """B over the whole range 2^8..2^14 with the bench's redraw rule (here at 2^17 rows):
    batched application bit for bit equal to the per-instance path, and batched steps equal
    to per-instance steps that share one workspace."""
    import ctypes
    import torch
    cap = 1 << 17
    draws = batch_instances(16, seed=5, log2_bmax=14.0, accept=lambda N, B: hs.index_count(N, B) <= cap)
    assert max(d["B"] for d in draws) > 2 ** 11
    print("draws", [(d["N"], d["B"]) for d in draws], flush=True)
    idxs, pots, ks, cs = make_batch(hs, draws)
    b = hs.Batch(idxs, pots)
    x = pack(b, cs)
    y = torch.zeros_like(x)
    b.apply_h(x, y)
    yb = y.cpu().numpy()
    for i, (idx, pot, c) in enumerate(zip(idxs, pots, cs)):
        ci = torch.from_numpy(c).to("cuda")
        yi = torch.empty_like(ci)
        hs.apply_h(idx, pot, ci, yi)
        torch.cuda.synchronize()
        assert np.array_equal(yb[b.offsets[i]:b.offsets[i] + c.size], yi.cpu().numpy()), f"instance {i}"
    m, h = 10, 0.005
    ws = b.workspace(m)
    b.step(x, 0.0, h, m, ws=ws)
    xb = x.cpu().numpy()
    nbmax = 0
    for idx, pot in zip(idxs, pots):
        nb = ctypes.c_int64()
        hs.hs_workspace_bytes(idx.h, pot.h, hs.HS_C128, m, ctypes.byref(nb))
        nbmax = max(nbmax, nb.value)
    ws1 = hs.dev_buffer(nbmax)
    singles = [torch.from_numpy(c.copy()).to("cuda") for c in cs]
    for idx, pot, ci in zip(idxs, pots, singles):
        hs.step(idx, pot, ci, 0.0, h, m, ws=ws1)
    torch.cuda.synchronize()
    for i, ci in enumerate(singles):
        seg = xb[b.offsets[i]:b.offsets[i] + cs[i].size]
        assert rel2(seg, ci.cpu().numpy()) <= 1e-13, f"instance {i}: batched vs per-instance"
