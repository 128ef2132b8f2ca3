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


def _perturbation(k):
    """A deterministic function of the multi-index, of modulus <= sqrt(2).  The phases are
    residues of integer forms, so they are bit-identical however the rows are batched
    (a floating-point phase like k.k * 0.11 would round differently in a vectorised
    product and in a single-row one, and H's large weights amplify that)."""
    k = np.atleast_2d(np.asarray(k, dtype=np.int64))
    n = k.shape[1]
    r1 = (k @ np.arange(3, 3 + 2 * n, 2, dtype=np.int64)) % 97
    r2 = ((k * k) @ np.arange(n, 0, -1, dtype=np.int64)) % 89
    return np.cos(2.0 * np.pi * r1 / 97.0) + 1j * np.sin(2.0 * np.pi * r2 / 89.0)


def _vector(k):
    """Coherent packet plus a perturbation of size 1e-3 on every row, a closed-form
    function of the multi-index (so the oracle evaluates it by index)."""
    return coherent_state(np.atleast_2d(k), 0.5) + 1e-3 * _perturbation(k)


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


def test_above_32bit_buffer_range():
    """N = 6, product bound 65536 (247,147,586 rows): complex128 vectors of 3.95 GB, past
    the 2^31 bytes of a signed 32-bit byte offset.  The fused kernels address vectors by
    element index (times the 16-byte record stride), so both types take them.  Float64
    checked on sampled rows against the oracle, float32 against float64."""
    import torch
    from paper_1403_3511_amd import hs
    N6, B6 = 6, 65536
    tt = hh_workload(N6, 0.111, 0.05)
    idx = hs.Index(N6, B6)
    assert idx.size == 247147586 and idx.size * 16 > 2 ** 31 > idx.size * 8
    pot = hs.Pot(N6, lib_terms(tt), subtract_harmonic=True)
    pot.set_time(0.3)
    k = idx.multi_indices()

    def vec(kk):
        kk = np.atleast_2d(np.asarray(kk, dtype=np.int64))
        return coherent_state(kk, 1.0) + 1e-3 * _perturbation(kk)

    c = torch.empty(idx.size, dtype=torch.complex128, device="cuda")
    step = 8_000_000
    for i in range(0, idx.size, step):
        c[i:i + step] = torch.from_numpy(vec(k[i:i + step]))
    y = torch.empty_like(c)
    hs.apply_h(idx, pot, c, y)
    rng = np.random.default_rng(4)
    rows = np.concatenate([np.arange(0, 20), rng.choice(idx.size, 40, replace=False),
                           np.arange(idx.size - 10, idx.size)])
    rsel = torch.from_numpy(rows).to("cuda")
    y64 = y[rsel].cpu().numpy()
    y_ref = fast_H_rows(N6, B6, oracle_W(N6, tt, 0.3), lambda m: vec(np.array(m))[0], k[rows])
    assert rel2(y64[:20], y_ref[:20]) <= 1e-12
    assert rel2(y64[20:], y_ref[20:]) <= 1e-12
    # float32 form on the same input, just under its 32-bit limit
    c32 = c.to(torch.complex64)
    del c
    y32 = torch.empty_like(c32)
    hs.apply_h(idx, pot, c32, y32, hs.HS_C64)
    err = float(torch.linalg.norm(y32.to(torch.complex128) - y) / torch.linalg.norm(y))
    print(f"N=6 B=65536: float32 H application relative error vs float64 {err:.2e}")
    assert err < 1e-5


def _dyadic(k):
    """An exactly representable complex value per multi-index, (r1 - 48)/64 + i (r2 - 44)/64
    with r1, r2 integer residues of k: numpy here and torch on the device compute the
    same bits (no transcendental functions), in float64 and float32 alike."""
    k = np.atleast_2d(np.asarray(k, dtype=np.int64))
    n = k.shape[1]
    r1 = (k @ np.arange(3, 3 + 2 * n, 2, dtype=np.int64)) % 97
    r2 = ((k * k) @ np.arange(n, 0, -1, dtype=np.int64)) % 89
    return (r1 - 48) / 64.0 + 1j * (r2 - 44) / 64.0


def _dyadic_device(k_chunk, out):
    import torch
    kk = torch.from_numpy(k_chunk).to("cuda").to(torch.int64)
    n = kk.shape[1]
    w1 = torch.arange(3, 3 + 2 * n, 2, dtype=torch.int64, device="cuda")
    w2 = torch.arange(n, 0, -1, dtype=torch.int64, device="cuda")
    r1 = (kk * w1).sum(1) % 97
    r2 = (kk * kk * w2).sum(1) % 89
    out.real.copy_((r1 - 48).to(torch.float64) / 64.0)
    out.imag.copy_((r2 - 44).to(torch.float64) / 64.0)


def test_n10_bound_2e14_beyond_4gib():
    """N = 10, product bound 2^14 (1,064,429,409 rows; Sec. 3.2, eq. Horner at the largest
    single-GPU size): complex128 vectors of 17 GB and complex64 of 8.5 GB, so element
    indices times the record stride pass 2^32 bytes.  The set is too large for per-tile
    records everywhere, so short tiles take the row kernel.  Sampled rows against the
    oracle's row-by-row evaluation: the first rows, random rows, rows past 4 GiB in each
    type, rows of short tiles past 4 GiB, and the last rows; float64 to 1e-12 (2-norm and
    largest row error), float32 to 1e-5."""
    import torch
    from oracle.index import count
    from paper_1403_3511_amd import hs
    N10, B10 = 10, 16384
    tt = hh_workload(N10, 0.111, 0.05)
    idx = hs.Index(N10, B10)
    assert idx.size == 1064429409
    pot = hs.Pot(N10, lib_terms(tt), subtract_harmonic=True)
    pot.set_time(0.2)
    k = idx.multi_indices()
    print(f"N=10 B=16384: {idx.size} rows, tile dimension {idx.tile_dim}", flush=True)
    c = torch.empty(idx.size, dtype=torch.complex128, device="cuda")
    step = 50_000_000
    for i in range(0, idx.size, step):
        _dyadic_device(k[i:i + step], c[i:i + step])
    torch.cuda.synchronize()
    # rows: first, random, past 4 GiB of complex128 (2^28 elements) and of complex64 (2^29),
    # in short tiles (fewer than 32 rows) past 2^29, and the last ones
    rng = np.random.default_rng(10)
    d = idx.tile_dim

    def tile_len(j):
        return count(d, B10 // int(np.prod(1 + j[:N10 - d].astype(np.int64))))

    far = rng.integers(2 ** 29, idx.size, 4000)
    short = [r for r in far if tile_len(k[r]) < 32][:25]
    long_ = [r for r in far if tile_len(k[r]) >= 64][:15]
    assert len(short) >= 10 and len(long_) >= 10
    rows = np.concatenate([np.arange(0, 10), rng.integers(0, idx.size, 25),
                           rng.integers(2 ** 28, 2 ** 29, 15), np.array(short), np.array(long_),
                           np.arange(idx.size - 15, idx.size)]).astype(np.int64)
    y_ref = fast_H_rows(N10, B10, oracle_W(N10, tt, 0.2), lambda m: _dyadic(np.array(m))[0], k[rows])
    rsel = torch.from_numpy(rows).to("cuda")
    y = torch.empty_like(c)
    hs.apply_h(idx, pot, c, y)
    y64 = y[rsel].cpu().numpy()
    del y
    e2 = rel2(y64, y_ref)
    einf = float(np.max(np.abs(y64 - y_ref)) / np.max(np.abs(y_ref)))
    parts = {"first": slice(0, 10), "random": slice(10, 35), "past 4 GiB": slice(35, 50),
             "short tiles": slice(50, 50 + len(short)),
             "long tiles": slice(50 + len(short), 50 + len(short) + len(long_)),
             "last": slice(len(rows) - 15, len(rows))}
    errs = {k: rel2(y64[v], y_ref[v]) for k, v in parts.items()}
    print(f"float64: sampled-row relative error 2-norm {e2:.2e}, inf-norm {einf:.2e}; by kind "
          + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
    assert e2 <= 1e-12 and einf <= 1e-12
    assert all(v <= 1e-12 for v in errs.values())
    c32 = c.to(torch.complex64)
    del c
    y32 = torch.empty_like(c32)
    hs.apply_h(idx, pot, c32, y32, hs.HS_C64)
    y32s = y32[rsel].cpu().numpy().astype(np.complex128)
    e32 = rel2(y32s, y_ref)
    print(f"float32: sampled-row relative error against the float64 oracle {e32:.2e}", flush=True)
    assert e32 <= 1e-5
