"""Shared helpers of the GPU tests: workload construction on both sides and the map
between the library's row order and the oracle's lexicographic order."""
from __future__ import annotations

import numpy as np

from oracle.index import IndexSet, LexRanker
from oracle.operators import Potential, subtract_harmonic
from synth import henon_heiles_chain


def lib_terms(timeterms):
    """synth TimeTerms -> (base, amp, freq, phase, degrees) tuples for hs.Pot."""
    return [(tt[0], tt[1], tt[2], tt[3], tt.degrees) for tt in timeterms]


def oracle_W(N, timeterms, t):
    V = Potential(N, "mono", 1.0, [(tt.coef(t), tt.degrees) for tt in timeterms])
    return subtract_harmonic(V)


def lib_to_lex(idx_lib, N, B):
    """perm such that x_lex = x_lib[perm]... returned as (rank_of_lib_row)."""
    k = idx_lib.multi_indices().astype(np.int64)
    r = LexRanker(N, B).rank(k)
    return r  # lex position of each library row


def to_lib(x_lex, lexpos):
    return x_lex[lexpos]


def rel2(a, b):
    """Relative error of a against b in the 2-norm and the infinity norm, the larger of the
    two (parity is stated in both norms; an error confined to a few rows shows in the
    second)."""
    a = np.asarray(a)
    b = np.asarray(b)
    e2 = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    if b.size == 0:
        return e2
    einf = float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
    return max(e2, einf)


def torch_c128(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x.astype(np.complex128))).to("cuda")


def torch_c64(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64))).to("cuda")


def hh_workload(N, lam=0.111, laser=0.0):
    return henon_heiles_chain(N, lam, laser)
