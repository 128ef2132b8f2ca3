"""Workloads for the debug build's neighbour-index checks (not collected by pytest; run
by tests/test_gpu_debug_bounds.py, once with libhs_debug.so in a child process and once
with the release library): every H-application kernel family on every set kind, the
direct operation, general and one-workgroup steps, a batch and the exact operator.
run(hs) returns, per case, the 2-norm of the result and the set's debug counters."""
import json
import sys

import numpy as np


def run(hs):
    import torch
    from synth import (complex_normal_by_index, henon_heiles_chain, random_downward_set,
                       torsional_series)

    def hh_pot(N, x2=False):
        tt = henon_heiles_chain(N, 0.111, 0.05)
        terms = [(t[0], t[1], t[2], t[3], t.degrees) for t in tt]
        if x2:  # x_1^2 and x_1 x_2: the row kernel with the X2 monomials
            terms += [(0.03, 0.0, 0.0, 0.0, (2,) + (0,) * (N - 1)), (0.02, 0.0, 0.0, 0.0, (1, 1) + (0,) * (N - 2))]
        p = hs.Pot(N, terms, subtract_harmonic=True)
        p.set_time(0.01)
        return p

    out = {}

    def record(name, idx, y):
        torch.cuda.synchronize()
        out[name] = {"norm": float(torch.linalg.norm(y.to(torch.complex128))), "counts": list(idx.debug_counts())}

    sets = {
        "hyp_N2_B64": hs.Index(2, 64),
        "hyp_N3_B500": hs.Index(3, 500),
        "hyp_N4_B4096": hs.Index(4, 4096),
        "hyp_N6_B4096": hs.Index(6, 4096),
        "hyp_N7_B2048": hs.Index(7, 2048),
        "hyp_N4_B700_d4": hs.Index(4, 700, 4),
        "box_N3_K20": hs.Index(3, 20, box=True),
        "tdeg_N4_D20": hs.Index(4, 20, total_degree=True),
        "list_N3": hs.Index(3, rows=random_downward_set(3, 40, 30, 5)),
        "padded_N3_B100_w3": hs.Index(3, 100, pad=3),
    }
    for name, idx in sets.items():
        N = idx.N
        c = torch.from_numpy(complex_normal_by_index(idx.multi_indices(), 11)).to("cuda")
        y = torch.empty_like(c)
        for pname, pot in (("hh", hh_pot(N)), ("hh_x2", hh_pot(N, True)),
                           ("torsional", hs.Pot(N, torsional_series(N), basis="cheb", scale=16.0))):
            hs.apply_h(idx, pot, c, y)
            record(f"{name}/{pname}/f64", idx, y)
            c32 = c.to(torch.complex64)
            y32 = torch.empty_like(c32)
            hs.apply_h(idx, pot, c32, y32, hs.HS_C64)
            record(f"{name}/{pname}/f32", idx, y32)
        for axis in range(N):
            hs.apply_x(idx, axis, c, y)
        record(f"{name}/xop", idx, y)
        if idx.size <= 200000:
            pot = hh_pot(N)
            s = c / torch.linalg.norm(c)
            hs.step(idx, pot, s, 0.0, 0.005, 6)
            record(f"{name}/step", idx, s)
    # one-workgroup and general step on a small set
    idx = sets["hyp_N2_B64"]
    pot = hh_pot(2)
    for rows in (1024, 0):
        old = hs.set_small_step_rows(rows)
        s = torch.from_numpy(complex_normal_by_index(idx.multi_indices(), 3)).to("cuda")
        hs.step(idx, pot, s, 0.0, 0.01, 10)
        record(f"small_step_rows{rows}", idx, s)
        hs.set_small_step_rows(old)
    # a batch of three instances
    bidx = [hs.Index(3, 300), hs.Index(5, 2000), hs.Index(6, 1024)]
    bpot = [hh_pot(i.N) for i in bidx]
    b = hs.Batch(bidx, bpot)
    total = int(b.offsets[-1])
    cb = torch.randn(total, dtype=torch.complex128, generator=torch.Generator().manual_seed(5)).to("cuda")
    yb = torch.zeros_like(cb)  # the rows between instances (alignment) stay zero
    b.apply_h(cb, yb)
    torch.cuda.synchronize()
    out["batch"] = {"norm": float(torch.linalg.norm(yb)),
                    "counts": [sum(v) for v in zip(*[i.debug_counts() for i in bidx])]}
    # the exact operator through a padded box
    sub = hs.Index(3, 41)
    op = hs.ExactOperator(sub, hs.Index(3, 44, box=True))
    pot = hs.Pot(3, torsional_series(3), basis="cheb", scale=16.0)
    c = torch.from_numpy(complex_normal_by_index(sub.multi_indices(), 2)).to("cuda")
    y = torch.empty_like(c)
    op.apply(pot, c, y)
    torch.cuda.synchronize()
    out["exact"] = {"norm": float(torch.linalg.norm(y)),
                    "counts": [a + b2 for a, b2 in zip(sub.debug_counts(), op.pad.debug_counts())]}
    return out


if __name__ == "__main__":
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch  # noqa: F401  (the HIP runtime comes up through torch first)
    from paper_1403_3511_amd import hs as _hs
    res = run(_hs)
    print(json.dumps({"checks": _hs.debug_checks(), "lib": _hs.LIB_PATH, "cases": res}), flush=True)
    sys.exit(0)
