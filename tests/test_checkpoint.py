"""Checkpoint and resume of a propagation's state (c^n, t_n, n): the file format and its
error handling on the CPU (host buffers, no GPU), and, on the GPU, that resuming from a
checkpoint reproduces the uninterrupted run bit for bit."""
import ctypes as C
import os
import struct

import numpy as np
import pytest


@pytest.fixture(scope="module")
def hs():
    from paper_1403_3511_amd import hs as _hs
    return _hs


def _save_host(hs, path, header, data):
    buf = np.ascontiguousarray(data)
    return hs.hs_checkpoint_save(os.fsencode(path), header.encode(), buf.ctypes.data_as(C.c_void_p),
                                 buf.nbytes, 0, None)


def _load_host(hs, path, nbytes):
    out = np.zeros(nbytes, dtype=np.uint8)
    hs.hs_checkpoint_load(os.fsencode(path), out.ctypes.data_as(C.c_void_p), nbytes, 0, None)
    return out


def test_host_round_trip_and_framing(hs, tmp_path):
    rng = np.random.default_rng(5)
    data = rng.standard_normal(1000) + 1j * rng.standard_normal(1000)
    path = str(tmp_path / "a.ckpt")
    header = '{"t_hex": "0x1.47ae147ae147bp-7", "n": 3}'
    _save_host(hs, path, header, data)
    raw = open(path, "rb").read()
    # framing: magic, header length, header, data length, checksum, data
    assert raw[:8] == b"HSCKPT01"
    (hl,) = struct.unpack("<Q", raw[8:16])
    assert raw[16:16 + hl].decode() == header
    (dl,) = struct.unpack("<Q", raw[16 + hl:24 + hl])
    assert dl == data.nbytes and len(raw) == 32 + hl + dl
    assert raw[32 + hl:] == data.tobytes()
    # FNV-1a 64 of the data, computed here from its definition
    h = 14695981039346656037
    for b in data.tobytes():
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    assert struct.unpack("<Q", raw[24 + hl:32 + hl])[0] == h
    back = _load_host(hs, path, data.nbytes).view(np.complex128)
    assert np.array_equal(back, data)
    hl2, dl2 = C.c_int64(), C.c_int64()
    buf = C.create_string_buffer(8)
    hs.hs_checkpoint_info(os.fsencode(path), buf, 8, C.byref(hl2), C.byref(dl2))
    assert hl2.value == len(header) and dl2.value == data.nbytes and buf.value == header[:7].encode()
    assert not os.path.exists(path + ".tmp")


def test_empty_state(hs, tmp_path):
    path = str(tmp_path / "e.ckpt")
    hs.hs_checkpoint_save(os.fsencode(path), b"{}", None, 0, 0, None)
    hs.hs_checkpoint_load(os.fsencode(path), None, 0, 0, None)


def test_corrupt_truncated_and_mismatched_files(hs, tmp_path):
    data = np.arange(64, dtype=np.float64)
    path = str(tmp_path / "b.ckpt")
    _save_host(hs, path, "{}", data)
    raw = bytearray(open(path, "rb").read())

    def expect(code, fn, *args):
        with pytest.raises(hs.HSError) as e:
            fn(*args)
        assert e.value.code == code

    # a flipped data byte fails the checksum and leaves the destination untouched
    bad = bytearray(raw)
    bad[-5] ^= 0x40
    p2 = str(tmp_path / "c.ckpt")
    open(p2, "wb").write(bad)
    out = np.full(data.nbytes, 7, dtype=np.uint8)
    expect(-8, hs.hs_checkpoint_load, os.fsencode(p2), out.ctypes.data_as(C.c_void_p), data.nbytes, 0, None)
    assert (out == 7).all()
    # truncated data, truncated header, wrong magic, missing file
    for blob in (raw[:-1], raw[:12], b"NOTACKPT" + raw[8:]):
        open(p2, "wb").write(blob)
        expect(-8, hs.hs_checkpoint_info, os.fsencode(p2), None, 0, None, None)
    expect(-8, hs.hs_checkpoint_info, os.fsencode(str(tmp_path / "missing")), None, 0, None, None)
    # a destination of another size
    out = np.zeros(data.nbytes - 8, dtype=np.uint8)
    expect(-1, hs.hs_checkpoint_load, os.fsencode(path), out.ctypes.data_as(C.c_void_p), out.nbytes, 0, None)
    # NULL arguments and negative sizes
    expect(-1, hs.hs_checkpoint_save, None, b"{}", None, 0, 0, None)
    expect(-1, hs.hs_checkpoint_save, os.fsencode(path), b"{}", None, 16, 0, None)
    expect(-1, hs.hs_checkpoint_load, os.fsencode(path), None, -1, 0, None)
    # a directory that does not exist cannot take the file
    expect(-8, _save_host, hs, str(tmp_path / "no" / "dir.ckpt"), "{}", data)


def test_binding_header_and_set_check(hs, tmp_path):
    """The binding's header describes the set; loading for another set is refused."""
    import torch
    idx = hs.Index(3, 64, upload=False)
    other = hs.Index(3, 65, upload=False)
    c = torch.randn(idx.size, dtype=torch.complex128)
    path = str(tmp_path / "s.ckpt")
    t = 0.1 + 0.2  # not a short decimal: the hexadecimal form keeps it exact
    hs.checkpoint_save(path, idx, c, t, 7, config={"h": 0.005, "m": 10}, seeds={"start": 0})
    head = hs.checkpoint_info(path)
    assert head["set"] == idx.describe() and head["n"] == 7 and head["config"]["m"] == 10
    back, t2, n2, _ = hs.checkpoint_load(path, idx, device="cpu")
    assert torch.equal(back, c) and t2 == t and n2 == 7
    with pytest.raises(hs.HSError):
        hs.checkpoint_load(path, other, device="cpu")


@pytest.mark.gpu
def test_resume_reproduces_the_uninterrupted_run(hs, tmp_path):
    """Propagate 3 steps, checkpoint, propagate 4 more; then resume from the file in a
    fresh state and propagate the same 4 steps: bitwise the same c^{n+k} and t."""
    import torch
    assert torch.cuda.is_available()  # the HIP runtime comes up through torch first
    from synth import coherent_state
    from tests.hsutil import hh_workload, lib_terms
    N, B, h, m = 4, 512, 0.005, 10
    idx = hs.Index(N, B)
    pot = hs.Pot(N, lib_terms(hh_workload(N, 0.111, 0.05)), subtract_harmonic=True)
    c = torch.from_numpy(coherent_state(idx.multi_indices(), 2.0)).to("cuda")
    c /= torch.linalg.norm(c)
    ws = hs.workspace(idx, pot, hs.HS_C128, m)
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):
        hs.step(idx, pot, c, 0.0, h, m, ws=ws, t_dev=t_dev)
    path = str(tmp_path / "run.ckpt")
    hs.checkpoint_save(path, idx, c, float(t_dev.item()), 3, config={"h": h, "m": m})
    for _ in range(4):
        hs.step(idx, pot, c, 0.0, h, m, ws=ws, t_dev=t_dev)
    torch.cuda.synchronize()
    c_ref, t_ref = c.clone(), float(t_dev.item())

    c2, t2, n2, _ = hs.checkpoint_load(path, idx)
    assert n2 == 3
    t_dev2 = torch.tensor([t2], dtype=torch.float64, device="cuda")
    ws2 = hs.workspace(idx, pot, hs.HS_C128, m)
    for _ in range(4):
        hs.step(idx, pot, c2, 0.0, h, m, ws=ws2, t_dev=t_dev2)
    torch.cuda.synchronize()
    assert torch.equal(c2, c_ref)
    assert float(t_dev2.item()) == t_ref
