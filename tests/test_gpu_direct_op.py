"""The direct operation y = X_K^(l) c (Sec. 3.1, eq. DirectOperationWithX) through the
C-ABI entry point, against the oracle's direct_op on every set kind, both precisions and
every axis; against the one-dimensional Jacobi matrix for N = 1; and on the full N = 6,
bound 4096 set, element by element against the oracle and by the symmetry of X."""
import numpy as np
import pytest

from oracle.index import BoxIndex, IndexSet, ListIndex, TotalDegreeIndex
from oracle.operators import direct_op, jacobi_matrix
from synth import complex_normal_by_index, random_downward_set
from tests.hsutil import rel2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_3511_amd import hs as _hs
    return _hs


def _sets(hs):
    """(name, oracle set, library set) for each set kind, with tiled splits that differ."""
    rows = random_downward_set(4, 12, 7, seed=21)
    return [
        ("hyperbolic N=3 B=200 d=1", IndexSet(3, 200), hs.Index(3, 200, 1)),
        ("hyperbolic N=3 B=200 d=2", IndexSet(3, 200), hs.Index(3, 200, 2)),
        ("hyperbolic N=6 B=300", IndexSet(6, 300), hs.Index(6, 300)),
        ("box N=3 K=6", BoxIndex(3, 6), hs.Index(3, 6, box=True)),
        ("total degree N=4 D=10", TotalDegreeIndex(4, 10), hs.Index(4, 10, total_degree=True)),
        ("list N=4", ListIndex(rows), hs.Index(4, rows=rows)),
    ]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_direct_op_every_set_and_axis(hs, dtype):
    import torch
    code = hs.HS_C128 if dtype == "c128" else hs.HS_C64
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    tol = 1e-15 if dtype == "c128" else 1e-6
    for name, ix, idx in _sets(hs):
        pos = ix.rank(idx.multi_indices().astype(np.int64))   # oracle row of each library row
        c = complex_normal_by_index(ix.k, 5 + ix.N)
        if dtype == "c64":
            c = c.astype(np.complex64).astype(np.complex128)  # the same input on both sides
        cl = torch.from_numpy(np.ascontiguousarray(c[pos])).to("cuda", tdt)
        yl = torch.empty_like(cl)
        for axis in range(ix.N):
            print(name, dtype, "axis", axis, flush=True)
            hs.apply_x(idx, axis, cl, yl, code)
            torch.cuda.synchronize()
            y = np.empty_like(c)
            y[pos] = yl.cpu().numpy().astype(np.complex128)
            assert rel2(y, direct_op(ix, axis, c)) <= tol, (name, axis)


def test_direct_op_one_axis_is_the_jacobi_matrix(hs):
    """N = 1: the set is {0..B-1} and X is the symmetric tridiagonal Jacobi matrix of the
    Hermite recurrence, off-diagonal sqrt(k/2)."""
    import torch
    B = 37
    idx = hs.Index(1, B)
    k = idx.multi_indices()[:, 0].astype(np.int64)
    assert sorted(k) == list(range(B))
    J = jacobi_matrix(B - 1)
    c = complex_normal_by_index(np.arange(B).reshape(-1, 1), 4)
    cl = torch.from_numpy(np.ascontiguousarray(c[k])).to("cuda")
    yl = torch.empty_like(cl)
    hs.apply_x(idx, 0, cl, yl)
    y = np.empty_like(c)
    y[k] = yl.cpu().numpy()
    assert rel2(y, J @ c) <= 1e-15


def test_direct_op_full_size(hs):
    """N = 6, bound 4096 (4,883,360 rows): every axis against the oracle on every row, and
    <u, X v> = <X u, v> (X is real symmetric)."""
    import torch
    N, B = 6, 4096
    ix = IndexSet(N, B)
    idx = hs.Index(N, B)
    pos = ix.rank(idx.multi_indices().astype(np.int64))
    c = complex_normal_by_index(ix.k, 31)
    u = complex_normal_by_index(ix.k, 32)
    cl = torch.from_numpy(np.ascontiguousarray(c[pos])).to("cuda")
    ul = torch.from_numpy(np.ascontiguousarray(u[pos])).to("cuda")
    yl, zl = torch.empty_like(cl), torch.empty_like(cl)
    for axis in (0, 2, 5):
        print("full size axis", axis, flush=True)
        hs.apply_x(idx, axis, cl, yl)
        hs.apply_x(idx, axis, ul, zl)
        torch.cuda.synchronize()
        y = np.empty_like(c)
        y[pos] = yl.cpu().numpy()
        assert rel2(y, direct_op(ix, axis, c)) <= 1e-15
        lhs = complex(torch.vdot(ul, yl))
        rhs = complex(torch.vdot(zl, cl))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_direct_op_argument_checks(hs):
    import torch
    idx = hs.Index(3, 50)
    c = torch.zeros(idx.size, dtype=torch.complex128, device="cuda")
    for args in ((3, c, torch.empty_like(c)), (-1, c, torch.empty_like(c)), (0, c, c)):
        with pytest.raises(hs.HSError):
            hs.apply_x(idx, *args)
