"""Random potentials outside the fused class, through the generic program of recurrence
passes (trie form or split trie/Clenshaw form, as the compiler chooses), against the
oracle's formal insertion (paper Sec. 3.2, eq. Horner; Fig. 3)."""
import numpy as np
import pytest

from oracle.index import IndexSet, count
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


def random_case(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 6))
    basis = ["mono", "cheb", "herm"][seed % 3]
    D = int(rng.integers(4, 7))
    nterms = int(rng.integers(4, 41))
    degs = set()
    # one term of degree >= 4 on one axis keeps the potential outside the fused class
    first = [0] * N
    first[int(rng.integers(0, N))] = int(rng.integers(4, D + 1))
    degs.add(tuple(first))
    while len(degs) < nterms:
        a = rng.multinomial(int(rng.integers(0, D + 1)), [1.0 / N] * N)
        degs.add(tuple(int(x) for x in a))
    degs = sorted(degs)
    B = 16
    while count(N, 2 * B) <= 20000 and B < 4096:
        B *= 2
    scale = {"mono": 1.0, "cheb": float(np.sqrt(2 * B) + 1), "herm": 1.0 + 0.3 * (seed % 2)}[basis]
    coefs = rng.standard_normal(len(degs)) * 0.01
    return N, B, basis, scale, degs, coefs


@pytest.mark.parametrize("seed", range(9))
def test_random_generic_potential(hs, seed):
    import torch
    N, B, basis, scale, degs, coefs = random_case(seed)
    ix = IndexSet(N, B)
    c = complex_normal_by_index(ix.k, 100 + seed)
    W = Potential(N, basis, scale, list(zip(coefs, degs)))
    y_ref = fast_apply_H(ix, W, c)
    idx = hs.Index(N, B)
    pot = hs.Pot(N, [(float(cf), d) for cf, d in zip(coefs, degs)], basis=basis, scale=scale)
    assert not pot.fused
    lexpos = lib_to_lex(idx, N, B)
    cl = torch.from_numpy(np.ascontiguousarray(c[lexpos])).to("cuda")
    yl = torch.empty_like(cl)
    hs.apply_h(idx, pot, cl, yl)
    torch.cuda.synchronize()
    y = np.empty_like(c)
    y[lexpos] = yl.cpu().numpy()
    err = rel2(y, y_ref)
    print(f"seed {seed}: N={N} B={B} |K|={ix.size} {basis} {len(degs)} terms: rel err {err:.1e}")
    assert err <= 1e-12
