"""ctypes binding of libhs.so (include/hs.h) -- argument marshalling only.

Every function of the C ABI is exposed under its own name with checked status codes
(HSError on failure).  The helper classes below only allocate device memory through
PyTorch and pass raw pointers and the current HIP stream; every step of the method
runs in the library's kernels.  There is no fallback: if libhs.so is missing the
import fails.
"""
from __future__ import annotations

import ctypes as C
import itertools
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# HS_LIBRARY may name another build of the same library (launch-shape experiments)
LIB_PATH = os.environ.get("HS_LIBRARY") or os.path.join(_HERE, "libhs.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} not built: run __graft_entry__.build() or "
                      "python -m paper_1403_3511_amd.build")
# PyTorch ships its own HIP runtime under the same soname as the system's.  Loading torch
# first makes libhs.so bind to that one copy; loaded the other way round the process would
# hold two runtimes, and the one the library calls would find no device.
try:
    import torch as _torch_first  # noqa: F401
except ImportError:  # host-only use of the library (index sets, checkpoint files)
    _torch_first = None
_lib = C.CDLL(LIB_PATH)

HS_OK, HS_INFO_BREAKDOWN = 0, 1
HS_C128, HS_C64 = 0, 1
HS_BASIS_MONO, HS_BASIS_CHEB, HS_BASIS_HERM = 0, 1, 2
HS_FORM_PAPER, HS_FORM_SYM = 0, 1
HS_SET_HYPERBOLIC, HS_SET_BOX, HS_SET_TOTAL_DEGREE, HS_SET_LIST, HS_SET_PADDED = 0, 1, 2, 3, 4
BASIS = {"mono": HS_BASIS_MONO, "cheb": HS_BASIS_CHEB, "herm": HS_BASIS_HERM}

_vp, _i32, _i64, _f64, _f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float
_pi64, _pi32, _pf64, _pf32, _pu16 = (C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double), C.POINTER(C.c_float),
                                     C.POINTER(C.c_uint16))

_SIGS = {
    "hs_last_error": [C.c_char_p, C.c_size_t],
    "hs_index_create": [_i32, _i64, _i32, C.POINTER(_vp)],
    "hs_index_destroy": [_vp],
    "hs_index_size": [_vp, _pi64],
    "hs_index_count": [_i32, _i64, _pi64],
    "hs_index_info": [_vp, _pi32, _pi64, _pi64],
    "hs_index_multi_indices": [_vp, _pu16],
    "hs_index_device_bytes": [_vp, _pi64],
    "hs_index_upload": [_vp, _vp, _i64, _vp],
    "hs_index_build_fibres": [_vp],
    "hs_index_create_box": [_i32, _i64, _i32, C.POINTER(_vp)],
    "hs_index_embed": [_vp, _vp, _pi32],
    "hs_index_create_total_degree": [_i32, _i64, _i32, C.POINTER(_vp)],
    "hs_index_create_from_list": [_i32, _i64, _pu16, C.POINTER(_vp)],
    "hs_error_split_workspace_bytes": [_vp, _vp, _vp, _vp, _pi64],
    "hs_error_split": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "hs_pot_create": [_i32, _i32, _f64, _i32, _pu16, _pf64, _pf64, _pf64, _pf64, _i32, C.POINTER(_vp)],
    "hs_pot_destroy": [_vp],
    "hs_pot_is_fused": [_vp, _pi32],
    "hs_pot_device_bytes": [_vp, _pi64],
    "hs_pot_upload": [_vp, _vp, _i64, _vp],
    "hs_pot_set_time": [_vp, _vp, _f64, _vp, _vp],
    "hs_pot_set_coeffs_device": [_vp, _vp, _vp, _vp],
    "hs_pot_set_form": [_vp, _i32],
    "hs_apply_x": [_vp, _vp, _i32, _i32, _vp, _vp, _vp],
    "hs_propagate": [_vp, _vp, _vp, _vp, _i32, _f64, _vp, _f64, _i32, _i32, _i64, _vp, _vp, _vp],
    "hs_set_small_step_rows": [_i64],
    "hs_get_small_step_rows": [_pi64],
    "hs_index_create_padded": [_i32, _i64, _i64, _i32, C.POINTER(_vp)],
    "hs_workspace_bytes": [_vp, _vp, _i32, _i32, _pi64],
    "hs_apply_h": [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp],
    "hs_step": [_vp, _vp, _vp, _vp, _i32, _f64, _vp, _f64, _i32, _i32, _vp, _vp, _vp, _vp],
    "hs_step_static": [_vp, _vp, _vp, _vp, _i32, _f64, _vp, _f64, _i32, _i32, _vp, _vp, _vp],
    "hs_magnus4_workspace_bytes": [_vp, _vp, _i32, _i32, _pi64],
    "hs_apply_magnus4": [_vp, _vp, _vp, _vp, _vp, _i32, _f64, _vp, _vp, _vp, _vp],
    "hs_step_magnus4": [_vp, _vp, _vp, _vp, _vp, _i32, _f64, _vp, _f64, _i32, _i32, _vp, _vp, _vp, _vp],
    "hs_batch_create": [_i32, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp)],
    "hs_batch_destroy": [_vp],
    "hs_batch_offsets": [_vp, _pi64],
    "hs_batch_device_bytes": [_vp, _pi64],
    "hs_batch_upload": [_vp, _vp, _i64, _vp],
    "hs_batch_workspace_bytes": [_vp, _i32, _pi64],
    "hs_batch_apply_h": [_vp, _vp, _vp, _vp, _vp, _vp],
    "hs_batch_step": [_vp, _vp, _f64, _vp, _f64, _i32, _i32, _vp, _vp, _vp],
    "hs_batch_set_launch": [_vp, _i32, _i32],
    "hs_batch_get_launch": [_vp, _pi32, _pi32],
    "hs_batch_autotune_sync": [_vp, _vp, _vp, _vp, _vp, _vp],
    "hs_batch_tuning": [_vp, _pi32, _pi32],
    "hs_gh_ncoef": [_i32, _i32, _pi32],
    "hs_gh_rule": [_i32, _pf64, _pf64],
    "hs_gh_project": [_i32, _i32, _i32, _i32, _pf64, _i32, _vp, _vp, _vp],
    "hs_cheb_ncoef": [_i32, _i32, _i32, _pi32],
    "hs_cheb_interp": [_i32, _i32, _i32, _i32, _f64, _pf64, _i32, _vp, _vp, _vp],
    "hs_mlp_create": [_i32, _i32, _i32, C.POINTER(_vp)],
    "hs_mlp_destroy": [_vp],
    "hs_mlp_device_bytes": [_vp, _i32, _pi64],
    "hs_mlp_upload_params": [_vp, _vp, _pf32, _pf32, _vp],
    "hs_mlp_download_params": [_vp, _vp, _pf32, _vp],
    "hs_mlp_predict": [_vp, _vp, _i32, _vp, _vp, _vp],
    "hs_mlp_train_step": [_vp, _vp, _i32, _vp, _vp, _f32, _vp, _vp, _vp],
    "hs_sur_coeffs": [_vp, _vp, _i32, _i32, _i32, _i32, _pf64, _i32, _vp, _vp, _vp, _vp],
    "hs_debug_checks": [_pi32],
    "hs_index_debug_read": [_vp, _vp, C.POINTER(C.c_uint32), _i32, _vp],
    "hs_exact_workspace_bytes": [_vp, _vp, _vp, _i32, _pi64],
    "hs_apply_exact": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "hs_step_exact": [_vp, _vp, _vp, _vp, _vp, _vp, _f64, _vp, _f64, _i32, _i32, _vp, _vp, _vp, _vp],
    "hs_checkpoint_save": [C.c_char_p, C.c_char_p, _vp, _i64, _i32, _vp],
    "hs_checkpoint_info": [C.c_char_p, C.c_char_p, _i64, _pi64, _pi64],
    "hs_checkpoint_load": [C.c_char_p, _vp, _i64, _i32, _vp],
}

EXPORTED = sorted(list(_SIGS) + ["hs_version"])


class HSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def last_error() -> str:
    buf = C.create_string_buffer(1024)
    _lib.hs_last_error(buf, 1024)
    return buf.value.decode(errors="replace")


def _wrap(name, argtypes):
    f = getattr(_lib, name)
    f.argtypes = argtypes
    f.restype = C.c_int32

    def call(*args):
        st = f(*args)
        if st < 0:
            raise HSError(st, f"{name}: {last_error()}")
        return st

    call.__name__ = name
    return call


_lib.hs_version.restype = C.c_char_p
_lib.hs_version.argtypes = []
for _n, _a in _SIGS.items():
    globals()[_n] = _wrap(_n, _a)
_lib_raw = _lib


def hs_version() -> str:
    return _lib.hs_version().decode()


def debug_checks() -> bool:
    """Whether the loaded library is the debug build with neighbour-index checks."""
    b = C.c_int32()
    hs_debug_checks(C.byref(b))
    return bool(b.value)


# ---------------------------------------------------------------------------------------
# marshalling helpers (PyTorch only supplies device memory and the stream)
# ---------------------------------------------------------------------------------------


def _torch():
    import torch
    return torch


def stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def dev_buffer(nbytes: int, device="cuda"):
    """A 256-byte aligned uint8 device tensor of at least nbytes (>= 1)."""
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


# ---- argument checks before a launch: the C ABI carries no buffer lengths ------------

_DT_NAMES = {HS_C128: "complex128", HS_C64: "complex64"}


def _fail(msg):
    raise HSError(-1, msg)


def _check_vec(name, t, n, dtype=None, tdtype=None, device=None):
    """t must be a contiguous tensor of at least n elements of the complex type selected by
    dtype (or of torch dtype tdtype), on device (when given)."""
    torch = _torch()
    if t is None:
        _fail(f"{name}: a tensor is required")
    if not isinstance(t, torch.Tensor):
        _fail(f"{name}: expected a torch tensor, got {type(t).__name__}")
    want = tdtype
    if dtype is not None:
        if dtype not in _DT_NAMES:
            _fail(f"{name}: unknown dtype code {dtype}")
        want = torch.complex128 if dtype == HS_C128 else torch.complex64
    if want is not None and t.dtype != want:
        _fail(f"{name}: dtype {t.dtype} does not match {want}")
    if not t.is_contiguous():
        _fail(f"{name}: tensor must be contiguous")
    if t.numel() < n:
        _fail(f"{name}: {t.numel()} elements, {n} required")
    if device is not None and t.device != device:
        _fail(f"{name}: on {t.device}, expected {device}")


def _check_ws(name, ws, nbytes, device):
    torch = _torch()
    if not isinstance(ws, torch.Tensor) or not ws.is_contiguous():
        _fail(f"{name}: workspace must be a contiguous tensor")
    have = ws.numel() * ws.element_size()
    if have < nbytes:
        _fail(f"{name}: workspace of {have} bytes, {nbytes} required")
    if ws.device != device:
        _fail(f"{name}: workspace on {ws.device}, expected {device}")


def _dev_of(block, what):
    if block is None:
        _fail(f"{what} has no device block (created with upload=False)")
    return block.device


def _ws_bytes(idx, pot, dtype, m, magnus4=False):
    nb = C.c_int64()
    (hs_magnus4_workspace_bytes if magnus4 else hs_workspace_bytes)(idx.h, pot.h, dtype, m, C.byref(nb))
    return nb.value


def _check_step_args(name, idx, pot, dtype, m, c, ws, magnus4=False, pot_blocks=None):
    """A step's state c is complex128 in both forms (the FP32 form keeps complex64 Krylov
    vectors in the workspace); the workspace is sized for (dtype, m)."""
    _check_dtype_code(name, dtype)
    _check_h_args(name, idx, pot, HS_C128, m, [("c", c)], None, pot_blocks=pot_blocks)
    if ws is not None:
        _check_ws(name, ws, _ws_bytes(idx, pot, dtype, m, magnus4), c.device)


def _check_dtype_code(name, dtype):
    if dtype not in _DT_NAMES:
        _fail(f"{name}: unknown dtype code {dtype}")


def _check_distinct(name, *ts):
    live = [t for t in ts if t is not None]
    for i in range(len(live)):
        for j in range(i + 1, len(live)):
            a, b = live[i], live[j]
            a0, a1 = a.data_ptr(), a.data_ptr() + a.numel() * a.element_size()
            b0, b1 = b.data_ptr(), b.data_ptr() + b.numel() * b.element_size()
            if a0 < b1 and b0 < a1:
                _fail(f"{name}: input and output buffers overlap")


def _check_h_args(name, idx, pot, dtype, m, vecs, ws, magnus4=False, pot_blocks=None):
    """Shared checks of the single-instance calls: vectors (name, tensor) of idx.size
    elements of dtype, the workspace for (dtype, m), all on the index's device."""
    for vn, v in vecs:
        _check_vec(f"{name}: {vn}", v, idx.size, dtype=dtype)
    if ws is not None:
        _check_ws(name, ws, _ws_bytes(idx, pot, dtype, m, magnus4), ws.device)
    dev = _dev_of(idx.dev, "index")
    blocks = pot_blocks if pot_blocks is not None else [pot.dev]
    for b in blocks:
        if _dev_of(b, "potential") != dev:
            _fail(f"{name}: potential block on {b.device}, index on {dev}")
    for vn, v in vecs:
        if v.device != dev:
            _fail(f"{name}: {vn} on {v.device}, index on {dev}")
    if ws is not None and ws.device != dev:
        _fail(f"{name}: workspace on {ws.device}, index on {dev}")


class Index:
    """Host handle + uploaded device block of K_N(B)."""

    def __init__(self, N: int, B: int = 0, tile_dim: int = 0, device="cuda", upload=True, box: bool = False,
                 total_degree: bool = False, rows=None, pad: int = None, fibres: bool = False):
        """The hyperbolic cross prod(1 + k_l) <= B; with box=True the box {0..B}^N; with
        total_degree=True the set |k|_1 <= B; with rows (n x N integers) that explicit
        downward-closed set; with pad=w the padded cross prod(1 + max(k_l - w, 0)) <= B.
        fibres=True adds the per-axis fibres on which generic potentials run their chains
        of recurrence passes as single launches (hs_index_build_fibres)."""
        h = _vp()
        self.pad, self.rows_sha256 = pad, None
        if pad is not None:
            hs_index_create_padded(N, B, int(pad), tile_dim, C.byref(h))
            self.kind = "padded"
        elif rows is not None:
            k = np.ascontiguousarray(np.asarray(rows, dtype=np.uint16).reshape(-1, N))
            hs_index_create_from_list(N, k.shape[0], k.ctypes.data_as(_pu16), C.byref(h))
            self.kind = "list"
            import hashlib
            self.rows_sha256 = hashlib.sha256(np.ascontiguousarray(np.sort(k.view(
                np.dtype((np.void, 2 * N))).ravel())).tobytes()).hexdigest()
        else:
            make = hs_index_create_box if box else (hs_index_create_total_degree if total_degree else hs_index_create)
            make(N, B, tile_dim, C.byref(h))
            self.kind = "box" if box else ("total_degree" if total_degree else "hyperbolic")
        self.h, self.N, self.B, self.box = h, N, B, box
        n = C.c_int64()
        hs_index_size(h, C.byref(n))
        self.size = n.value
        d, nt, ng = C.c_int32(), C.c_int64(), C.c_int64()
        hs_index_info(h, C.byref(d), C.byref(nt), C.byref(ng))
        self.tile_dim, self.ntiles, self.nsuffix = d.value, nt.value, ng.value
        self.fibres = bool(fibres)
        if fibres:
            hs_index_build_fibres(h)
        self.dev = None
        if upload:
            nb = C.c_int64()
            hs_index_device_bytes(h, C.byref(nb))
            self.dev = dev_buffer(nb.value, device)
            hs_index_upload(h, ptr(self.dev), nb.value, stream_ptr())

    def describe(self) -> dict:
        """What identifies the set and its row order (the checkpoint header's "set")."""
        d = {"kind": self.kind, "N": self.N, "B": self.B, "tile_dim": self.tile_dim, "rows": self.size,
             "tiles": self.ntiles, "suffixes": self.nsuffix}
        if self.pad is not None:
            d["pad"] = int(self.pad)
        if self.rows_sha256 is not None:
            d["rows_sha256"] = self.rows_sha256
        return d

    def debug_counts(self, clear: bool = True):
        """(failed neighbour-index checks, code of the first) recorded on this index by the
        debug build's kernels (always (0, 0) with the release build)."""
        out = (C.c_uint32 * 2)()
        hs_index_debug_read(self.h, ptr(self.dev), out, 1 if clear else 0, stream_ptr())
        return int(out[0]), int(out[1])

    def multi_indices(self) -> np.ndarray:
        out = np.empty((self.size, self.N), dtype=np.uint16)
        hs_index_multi_indices(self.h, out.ctypes.data_as(_pu16))
        return out

    def embed_map(self, box: "Index") -> np.ndarray:
        """Row of box holding each of this set's multi-indices (-1 outside)."""
        out = np.empty(self.size, dtype=np.int32)
        hs_index_embed(self.h, box.h, out.ctypes.data_as(_pi32))
        return out

    def __del__(self):
        try:
            if getattr(self, "h", None):
                _lib.hs_index_destroy(self.h)
                self.h = None
        except Exception:
            pass


def index_count(N: int, B: int) -> int:
    """|K_N(B)| without building the set."""
    n = C.c_int64()
    hs_index_count(int(N), int(B), C.byref(n))
    return n.value


class Pot:
    """Potential handle + device parameter block.

    terms: list of (base, degrees) or (base, amp, freq, phase, degrees) tuples."""

    def __init__(self, N, terms, basis="mono", scale=1.0, subtract_harmonic=False,
                 device="cuda", upload=True):
        deg, base, amp, freq, phase = [], [], [], [], []
        for t in terms:
            if len(t) == 2:
                b, a = t
                am = fr = ph = 0.0
            else:
                b, am, fr, ph, a = t
            deg.append(list(a))
            base.append(b)
            amp.append(am)
            freq.append(fr)
            phase.append(ph)
        nt = len(terms)
        deg = np.ascontiguousarray(np.array(deg, dtype=np.uint16).reshape(nt, N))
        arrs = [np.ascontiguousarray(np.array(x, dtype=np.float64)) for x in (base, amp, freq, phase)]
        h = _vp()
        hs_pot_create(N, BASIS[basis] if isinstance(basis, str) else int(basis), float(scale), nt,
                      deg.ctypes.data_as(_pu16), *[x.ctypes.data_as(_pf64) for x in arrs],
                      1 if subtract_harmonic else 0, C.byref(h))
        self.h, self.N, self.nterms = h, N, nt + (N if subtract_harmonic else 0)  # terms as compiled
        f = C.c_int32()
        hs_pot_is_fused(h, C.byref(f))
        self.fused = bool(f.value)
        self.dev = None
        self.dev2 = None      # second parameter block of the fourth-order step
        self.device = device
        if upload:
            self.dev = self._new_block()

    def _new_block(self):
        nb = C.c_int64()
        hs_pot_device_bytes(self.h, C.byref(nb))
        dev = dev_buffer(nb.value, self.device)
        hs_pot_upload(self.h, ptr(dev), nb.value, stream_ptr())
        return dev

    def blocks2(self):
        """The two parameter blocks of the two-stage Magnus scheme (the second one is
        made on first use, a copy of the first)."""
        if self.dev2 is None:
            self.dev2 = self.dev.clone()
        return self.dev, self.dev2

    def set_time(self, t: float):
        hs_pot_set_time(self.h, ptr(self.dev), float(t), None, stream_ptr())

    def set_form(self, form: int):
        """HS_FORM_PAPER (the fast operator) or HS_FORM_SYM (its symmetric part)."""
        hs_pot_set_form(self.h, int(form))

    def set_coeffs_device(self, coef):
        """Base coefficients from a device float64 tensor (nterms values, term order);
        applied to both parameter blocks when the second one exists."""
        hs_pot_set_coeffs_device(self.h, ptr(self.dev), ptr(coef), stream_ptr())
        if self.dev2 is not None:
            hs_pot_set_coeffs_device(self.h, ptr(self.dev2), ptr(coef), stream_ptr())

    def __del__(self):
        try:
            if getattr(self, "h", None):
                _lib.hs_pot_destroy(self.h)
                self.h = None
        except Exception:
            pass


def workspace(idx: Index, pot: Pot, dtype: int, m: int, device="cuda"):
    nb = C.c_int64()
    hs_workspace_bytes(idx.h, pot.h, dtype, m, C.byref(nb))
    return dev_buffer(nb.value, device)


def apply_h(idx: Index, pot: Pot, c, y, dtype: int = HS_C128, ws=None):
    """y = H c; c, y complex device tensors in library row order."""
    _check_h_args("apply_h", idx, pot, dtype, 0, [("c", c), ("y", y)], ws)
    _check_distinct("apply_h", c, y)
    if ws is None:
        ws = workspace(idx, pot, dtype, 0, c.device)
    hs_apply_h(idx.h, ptr(idx.dev), pot.h, ptr(pot.dev), dtype, ptr(c), ptr(y), ptr(ws), stream_ptr())
    return y


def apply_x(idx: Index, axis: int, c, y, dtype: int = HS_C128):
    """y = X^(axis) c, the direct operation along one axis (0-based); c != y."""
    for vn, v in (("c", c), ("y", y)):
        _check_vec(f"apply_x: {vn}", v, idx.size, dtype=dtype, device=_dev_of(idx.dev, "index"))
    _check_distinct("apply_x", c, y)
    hs_apply_x(idx.h, ptr(idx.dev), int(axis), dtype, ptr(c), ptr(y), stream_ptr())
    return y


def step(idx: Index, pot: Pot, c, t: float, h: float, m: int, dtype: int = HS_C128,
         reorth: bool = True, ws=None, t_dev=None, diag=None):
    """One exponential-midpoint Lanczos step in place on c (complex128 device tensor)."""
    _check_step_args("step", idx, pot, dtype, m, c, ws)
    if ws is None:
        ws = workspace(idx, pot, dtype, m, c.device)
    hs_step(idx.h, ptr(idx.dev), pot.h, ptr(pot.dev), dtype, float(t), ptr(t_dev), float(h), int(m),
            1 if reorth else 0, ptr(c), ptr(ws), ptr(diag), stream_ptr())
    return c


def step_static(idx: Index, pot: Pot, c, t: float, h: float, m: int, dtype: int = HS_C128,
                reorth: bool = True, t_dev=None, diag=None):
    """hs_step with the library's fixed per-GPU workspace (no allocation anywhere)."""
    _check_step_args("step_static", idx, pot, dtype, m, c, None)
    hs_step_static(idx.h, ptr(idx.dev), pot.h, ptr(pot.dev), dtype, float(t), ptr(t_dev), float(h), int(m),
                   1 if reorth else 0, ptr(c), ptr(diag), stream_ptr())
    return c


def set_small_step_rows(rows: int) -> int:
    """Set the row limit of the one-workgroup step; returns the previous limit."""
    old = C.c_int64()
    hs_get_small_step_rows(C.byref(old))
    hs_set_small_step_rows(int(rows))
    return old.value


def propagate(idx: Index, pot: Pot, c, t0: float, h: float, m: int, nsteps: int, dtype: int = HS_C128,
              reorth: bool = True, ws=None, t_dev=None):
    """nsteps exponential-midpoint Lanczos steps in place on c (complex128 device tensor)."""
    _check_step_args("propagate", idx, pot, dtype, m, c, ws)
    if ws is None:
        ws = workspace(idx, pot, dtype, m, c.device)
    hs_propagate(idx.h, ptr(idx.dev), pot.h, ptr(pot.dev), dtype, float(t0), ptr(t_dev), float(h), int(m),
                 1 if reorth else 0, int(nsteps), ptr(c), ptr(ws), stream_ptr())
    return c


# ---- checkpoint and resume of (c^n, t_n, n) -------------------------------------------

CHECKPOINT_FORMAT = "hs-checkpoint"


def checkpoint_save(path: str, idx: Index, c, t: float, n: int, config=None, seeds=None):
    """Write the state (c, t, n) of a propagation on idx to path (hs_checkpoint_save).

    c is a contiguous complex128 or complex64 tensor on the GPU or the CPU with one entry
    per row of idx, in library row order.  t is stored exactly (as a hexadecimal float);
    config and seeds are JSON-serialisable descriptions kept in the header."""
    import json
    torch = _torch()
    if c.dtype not in (torch.complex128, torch.complex64) or c.numel() != idx.size or not c.is_contiguous():
        _fail(f"checkpoint_save: c must be a contiguous complex tensor of {idx.size} entries")
    header = {"format": CHECKPOINT_FORMAT, "version": 1, "set": idx.describe(),
              "dtype": "complex128" if c.dtype == torch.complex128 else "complex64",
              "t": float(t), "t_hex": float(t).hex(), "n": int(n),
              "config": config if config is not None else {}, "seeds": seeds if seeds is not None else {}}
    on_dev = bool(c.is_cuda)
    hs_checkpoint_save(os.fsencode(path), json.dumps(header, sort_keys=True).encode(), ptr(c),
                       c.numel() * c.element_size(), 1 if on_dev else 0, stream_ptr() if on_dev else None)


def checkpoint_info(path: str) -> dict:
    """The header of a checkpoint file, after checking its framing (hs_checkpoint_info)."""
    import json
    hl, dl = C.c_int64(), C.c_int64()
    hs_checkpoint_info(os.fsencode(path), None, 0, C.byref(hl), C.byref(dl))
    buf = C.create_string_buffer(hl.value + 1)
    hs_checkpoint_info(os.fsencode(path), buf, hl.value + 1, C.byref(hl), C.byref(dl))
    header = json.loads(buf.raw[:hl.value].decode())
    if header.get("format") != CHECKPOINT_FORMAT:
        _fail(f"checkpoint_info: {path} is not an {CHECKPOINT_FORMAT} file")
    header["data_bytes"] = dl.value
    return header


def checkpoint_load(path: str, idx: Index, device="cuda", out=None):
    """Read a checkpoint written for idx: returns (c, t, n, header).  The header's index
    set must be idx's (kind, sizes, bound, tile dimension), else HSError."""
    torch = _torch()
    header = checkpoint_info(path)
    want = idx.describe()
    if header.get("set") != want:
        _fail(f"checkpoint_load: {path} was written for the set {header.get('set')}, not {want}")
    tdtype = torch.complex128 if header["dtype"] == "complex128" else torch.complex64
    if out is None:
        out = torch.empty(idx.size, dtype=tdtype, device=device)
    elif out.dtype != tdtype or out.numel() != idx.size or not out.is_contiguous():
        _fail(f"checkpoint_load: out must be a contiguous {header['dtype']} tensor of {idx.size} entries")
    on_dev = bool(out.is_cuda)
    hs_checkpoint_load(os.fsencode(path), ptr(out), out.numel() * out.element_size(), 1 if on_dev else 0,
                       stream_ptr() if on_dev else None)
    return out, float.fromhex(header["t_hex"]), int(header["n"]), header


def workspace_magnus4(idx: Index, pot: Pot, dtype: int, m: int, device="cuda"):
    """Workspace of apply_magnus4 (m = 0) or step_magnus4 (m >= 1)."""
    nb = C.c_int64()
    hs_magnus4_workspace_bytes(idx.h, pot.h, dtype, m, C.byref(nb))
    return dev_buffer(nb.value, device)


def apply_magnus4(idx: Index, pot: Pot, h: float, c, y, dtype: int = HS_C128, ws=None):
    """y = M c, the operator of the two-stage Gauss-Legendre Magnus scheme, with the
    coefficients currently held in the potential's two parameter blocks."""
    d1, d2 = pot.blocks2()
    _check_h_args("apply_magnus4", idx, pot, dtype, 0, [("c", c), ("y", y)], ws, magnus4=True,
                  pot_blocks=[d1, d2])
    _check_distinct("apply_magnus4", c, y)
    if ws is None:
        ws = workspace_magnus4(idx, pot, dtype, 0, c.device)
    hs_apply_magnus4(idx.h, ptr(idx.dev), pot.h, ptr(d1), ptr(d2), dtype, float(h), ptr(c), ptr(y),
                     ptr(ws), stream_ptr())
    return y


def step_magnus4(idx: Index, pot: Pot, c, t: float, h: float, m: int, dtype: int = HS_C128,
                 reorth: bool = True, ws=None, t_dev=None, diag=None):
    """One fourth-order two-stage Gauss-Legendre Magnus step in place on c."""
    d1, d2 = pot.blocks2()
    _check_step_args("step_magnus4", idx, pot, dtype, m, c, ws, magnus4=True, pot_blocks=[d1, d2])
    if ws is None:
        ws = workspace_magnus4(idx, pot, dtype, m, c.device)
    hs_step_magnus4(idx.h, ptr(idx.dev), pot.h, ptr(d1), ptr(d2), dtype, float(t), ptr(t_dev),
                    float(h), int(m), 1 if reorth else 0, ptr(c), ptr(ws), ptr(diag), stream_ptr())
    return c


def error_split(sub: Index, box: Index, pad, pot: Pot, v, e_quad=None, e_red=None, maps=None, ws=None):
    """(e_quad, e_red) of the fast algorithm for v on sub (complex128 device tensor): the
    quadrature error against the padded box pad (None: e_quad is None) and the index-set
    reduction error against the box."""
    torch = _torch()
    _check_vec("error_split: v", v, sub.size, dtype=HS_C128, device=_dev_of(sub.dev, "index"))
    for vn, e in (("e_quad", e_quad), ("e_red", e_red)):
        if e is not None:
            _check_vec(f"error_split: {vn}", e, sub.size, dtype=HS_C128, device=v.device)
    if maps is None:
        maps = (torch.from_numpy(sub.embed_map(box)).to(v.device),
                torch.from_numpy(sub.embed_map(pad)).to(v.device) if pad is not None else None)
    if e_red is None:
        e_red = torch.empty_like(v)
    if pad is not None and e_quad is None:
        e_quad = torch.empty_like(v)
    if ws is None:
        nb = C.c_int64()
        hs_error_split_workspace_bytes(sub.h, box.h, pad.h if pad is not None else None, pot.h, C.byref(nb))
        ws = dev_buffer(nb.value, v.device)
    hs_error_split(sub.h, ptr(sub.dev), box.h, ptr(box.dev), ptr(maps[0]),
                   pad.h if pad is not None else None, ptr(pad.dev) if pad is not None else None,
                   ptr(maps[1]) if pad is not None else None, pot.h, ptr(pot.dev), ptr(v),
                   ptr(e_quad) if pad is not None else None, ptr(e_red), ptr(ws), stream_ptr())
    return e_quad, e_red


class ExactOperator:
    """The exact Galerkin operator D + W_{K,pol} on the rows of sub, carried by the padded
    set pad (a box, or the padded cross of a hyperbolic sub): hs_apply_exact and
    hs_step_exact, the unperturbed Lanczos process of the paper's perturbation analysis."""

    def __init__(self, sub: Index, pad: Index):
        torch = _torch()
        dev = _dev_of(sub.dev, "index")
        if _dev_of(pad.dev, "padded index") != dev:
            _fail("ExactOperator: sub and pad are uploaded to different devices")
        m = sub.embed_map(pad)
        if m.size and m.min() < 0:
            _fail("ExactOperator: pad does not contain sub")
        self.sub, self.pad, self.device = sub, pad, dev
        self.map = torch.from_numpy(m).to(dev)

    def workspace(self, pot: Pot, m: int = 0):
        nb = C.c_int64()
        hs_exact_workspace_bytes(self.sub.h, self.pad.h, pot.h, int(m), C.byref(nb))
        return dev_buffer(nb.value, self.device)

    def _ws(self, name, pot, m, ws):
        nb = C.c_int64()
        hs_exact_workspace_bytes(self.sub.h, self.pad.h, pot.h, int(m), C.byref(nb))
        if ws is None:
            return dev_buffer(nb.value, self.device)
        _check_ws(name, ws, nb.value, self.device)
        return ws

    def apply(self, pot: Pot, x, y, ws=None):
        """y = (D + W_{K,pol}) x on sub (complex128 device tensors, x != y)."""
        _check_vec("ExactOperator.apply: x", x, self.sub.size, dtype=HS_C128, device=self.device)
        _check_vec("ExactOperator.apply: y", y, self.sub.size, dtype=HS_C128, device=self.device)
        _check_distinct("ExactOperator.apply", x, y)
        ws = self._ws("ExactOperator.apply", pot, 0, ws)
        hs_apply_exact(self.sub.h, self.pad.h, ptr(self.pad.dev), ptr(self.map), pot.h, ptr(pot.dev), ptr(x),
                       ptr(y), ptr(ws), stream_ptr())
        return y

    def step(self, pot: Pot, c, t: float, h: float, m: int, reorth: bool = True, ws=None, t_dev=None,
             diag=None):
        """One exponential-midpoint step with m Lanczos steps on the exact operator, in
        place on c (complex128 device tensor)."""
        _check_vec("ExactOperator.step: c", c, self.sub.size, dtype=HS_C128, device=self.device)
        ws = self._ws("ExactOperator.step", pot, m, ws)
        hs_step_exact(self.sub.h, self.pad.h, ptr(self.pad.dev), ptr(self.map), pot.h, ptr(pot.dev), float(t),
                      ptr(t_dev), float(h), int(m), 1 if reorth else 0, ptr(c), ptr(ws), ptr(diag), stream_ptr())
        return c


class Batch:
    """Many (Index, Pot) instances advanced by one persistent launch per H application.
    Vectors are packed: instance i occupies elements offsets[i] .. offsets[i] + size_i."""

    def __init__(self, indices, pots, device="cuda"):
        n = len(indices)
        VP = _vp * n
        h = _vp()
        hs_batch_create(n, VP(*[i.h for i in indices]), VP(*[i.dev.data_ptr() for i in indices]),
                        VP(*[p.h for p in pots]), VP(*[p.dev.data_ptr() for p in pots]), C.byref(h))
        self.h, self.n = h, n
        self._keep = (list(indices), list(pots))  # device blocks must outlive the batch
        off = np.zeros(n + 1, dtype=np.int64)
        hs_batch_offsets(h, off.ctypes.data_as(_pi64))
        self.offsets = off
        self.total = int(off[-1])
        nb = C.c_int64()
        hs_batch_device_bytes(h, C.byref(nb))
        self.dev = dev_buffer(nb.value, device)
        hs_batch_upload(h, ptr(self.dev), nb.value, stream_ptr())

    def workspace(self, m: int, device="cuda"):
        nb = C.c_int64()
        hs_batch_workspace_bytes(self.h, m, C.byref(nb))
        return dev_buffer(nb.value, device)

    def _check(self, name, vecs, ws=None, m=0):
        dev = self.dev.device
        for vn, v in vecs:
            _check_vec(f"Batch.{name}: {vn}", v, self.total, tdtype=_torch().complex128, device=dev)
        if ws is not None:
            nb = C.c_int64()
            hs_batch_workspace_bytes(self.h, m, C.byref(nb))
            _check_ws(f"Batch.{name}", ws, nb.value, dev)

    def apply_h(self, c, y):
        self._check("apply_h", [("c", c), ("y", y)])
        _check_distinct("Batch.apply_h", c, y)
        hs_batch_apply_h(self.h, ptr(self.dev), ptr(c), ptr(y), None, stream_ptr())
        return y

    def step(self, c, t: float, h: float, m: int, reorth: bool = True, ws=None, t_dev=None):
        self._check("step", [("c", c)], ws, m)
        if ws is None:
            ws = self.workspace(m, c.device)
        hs_batch_step(self.h, ptr(self.dev), float(t), ptr(t_dev), float(h), int(m),
                      1 if reorth else 0, ptr(c), ptr(ws), stream_ptr())
        return c

    def set_launch(self, wg: int = 0, per_cu: int = 0):
        hs_batch_set_launch(self.h, wg, per_cu)

    def get_launch(self):
        a, b = C.c_int32(), C.c_int32()
        hs_batch_get_launch(self.h, C.byref(a), C.byref(b))
        return a.value, b.value

    def tuning(self):
        """(item order, [(N, prefix axes, kind, items, wg, per_cu, grab) for each class and
        kernel kind with work items]); kind 0 = row kernel, 1 = multi-tile kernel."""
        order = C.c_int32()
        t = np.zeros(70, dtype=np.int32)
        hs_batch_tuning(self.h, C.byref(order), t.ctypes.data_as(_pi32))
        rows = []
        for i in range(7):
            r = [int(v) for v in t[10 * i:10 * i + 10]]
            for kind in range(2):
                items, wg, pc, gr = r[2 + 4 * kind:6 + 4 * kind]
                if items > 0:
                    rows.append((r[0], r[1], kind, items, wg, pc, gr))
        return order.value, rows

    def autotune(self, c, y):
        self._check("autotune", [("c", c), ("y", y)])
        _check_distinct("Batch.autotune", c, y)
        hs_batch_autotune_sync(self.h, ptr(self.dev), ptr(c), ptr(y), None, stream_ptr())
        return self.get_launch()

    def __del__(self):
        try:
            if getattr(self, "h", None):
                _lib.hs_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass


# ---- learned coefficients -----------------------------------------------------------


def total_degree_multi_indices(N: int, D: int):
    """The multi-indices a with |a| <= D in lexicographic order: the coefficient order of
    hs_gh_project, hs_mlp_predict and hs_sur_coeffs (terms of the learned potential)."""
    import itertools
    return [a for a in itertools.product(range(D + 1), repeat=N) if sum(a) <= D]


def gh_ncoef(N: int, D: int) -> int:
    n = C.c_int32()
    hs_gh_ncoef(N, D, C.byref(n))
    return n.value


def geometry_array(geom) -> np.ndarray:
    """Host geometry block: base, u, w (G x N each), then phase (G)."""
    return np.ascontiguousarray(np.concatenate([np.asarray(geom[k], dtype=np.float64).ravel()
                                                for k in ("base", "u", "w", "phase")]))


def gh_project(geom, params, D: int, Q: int, out=None):
    """Gauss-Hermite coefficients for every row of params (device float64, nsamp x (4+G))."""
    torch = _torch()
    base = np.asarray(geom["base"])
    G, N = base.shape
    nc = gh_ncoef(N, D)
    ns = params.shape[0]
    _check_vec("gh_project: params", params, ns * (4 + G), tdtype=torch.float64)
    if out is None:
        out = torch.empty((ns, nc), dtype=torch.float64, device=params.device)
    _check_vec("gh_project: out", out, ns * nc, tdtype=torch.float64, device=params.device)
    g = geometry_array(geom)
    hs_gh_project(N, G, D, Q, g.ctypes.data_as(_pf64), ns, ptr(params), ptr(out), stream_ptr())
    return out


def cheb_ncoef(N: int, D: int, R: int) -> int:
    n = C.c_int32()
    hs_cheb_ncoef(N, D, R, C.byref(n))
    return n.value


def cheb_interp(geom, params, D: int, R: int, L: float, out=None):
    """Chebyshev coefficients (basis T_r(x/L), |r| <= D, r_l <= R) of the Gaussian-well
    potential for each parameter row (device float64 tensor, rows of 4 + G)."""
    torch = _torch()
    N = geom["base"].shape[1]
    G = geom["base"].shape[0]
    n = params.shape[0]
    _check_vec("cheb_interp: params", params, n * (4 + G), tdtype=torch.float64)
    if out is None:
        out = torch.empty((n, cheb_ncoef(N, D, R)), dtype=torch.float64, device=params.device)
    _check_vec("cheb_interp: out", out, n * cheb_ncoef(N, D, R), tdtype=torch.float64, device=params.device)
    g = geometry_array(geom)
    hs_cheb_interp(N, G, D, R, float(L), g.ctypes.data_as(_pf64), n, ptr(params), ptr(out), stream_ptr())
    return out


def cheb_degrees(N: int, D: int, R: int):
    """The multi-indices of cheb_interp's output, in its order."""
    out = []
    for m in itertools.product(range(R + 1), repeat=N):
        if sum(m) <= D:
            out.append(tuple(m))
    return out


class MLP:
    """in -> hidden -> hidden -> out SiLU network; weights and Adam state on the device."""

    def __init__(self, n_in: int, hidden: int, n_out: int, max_batch: int, device="cuda"):
        h = _vp()
        hs_mlp_create(n_in, hidden, n_out, C.byref(h))
        self.h, self.n_in, self.hidden, self.n_out = h, n_in, hidden, n_out
        self.max_batch = max_batch
        nb = C.c_int64()
        hs_mlp_device_bytes(h, max_batch, C.byref(nb))
        self.dev = dev_buffer(nb.value, device)
        self.nparam = hidden * n_in + hidden + hidden * hidden + hidden + n_out * hidden + n_out

    def upload(self, params: dict, in_lo, in_hi, out_mean, out_std):
        """params: W1, b1, W2, b2, W3, b3 (float arrays); also resets Adam."""
        w = np.ascontiguousarray(np.concatenate([np.asarray(params[k], dtype=np.float32).ravel()
                                                 for k in ("W1", "b1", "W2", "b2", "W3", "b3")]))
        assert w.size == self.nparam
        nrm = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float32).ravel()
                                                   for x in (in_lo, in_hi, out_mean, out_std)]))
        assert nrm.size == 2 * self.n_in + 2 * self.n_out
        hs_mlp_upload_params(self.h, ptr(self.dev), w.ctypes.data_as(_pf32), nrm.ctypes.data_as(_pf32),
                             stream_ptr())

    def unflatten(self, w: np.ndarray) -> dict:
        i, H, o = self.n_in, self.hidden, self.n_out
        shapes = [("W1", (H, i)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (o, H)), ("b3", (o,))]
        out, k = {}, 0
        for name, shp in shapes:
            n = int(np.prod(shp))
            out[name] = w[k:k + n].reshape(shp)
            k += n
        return out

    def download(self) -> dict:
        w = np.empty(self.nparam, dtype=np.float32)
        hs_mlp_download_params(self.h, ptr(self.dev), w.ctypes.data_as(_pf32), stream_ptr())
        return self.unflatten(w)

    def predict(self, x, out=None):
        torch = _torch()
        self._check_batch("predict", x)
        if out is None:
            out = torch.empty((x.shape[0], self.n_out), dtype=torch.float64, device=x.device)
        _check_vec("MLP.predict: out", out, x.shape[0] * self.n_out, tdtype=torch.float64, device=x.device)
        hs_mlp_predict(self.h, ptr(self.dev), x.shape[0], ptr(x), ptr(out), stream_ptr())
        return out

    def coeffs(self, geom, params, D: int, Q: int, out=None, used=None):
        """Network coefficients, quadrature for rows outside the training box."""
        torch = _torch()
        base = np.asarray(geom["base"])
        G, N = base.shape
        self._check_batch("coeffs", params)
        if out is None:
            out = torch.empty((params.shape[0], self.n_out), dtype=torch.float64, device=params.device)
        _check_vec("MLP.coeffs: out", out, params.shape[0] * self.n_out, tdtype=torch.float64,
                   device=params.device)
        if used is not None:
            _check_vec("MLP.coeffs: used", used, params.shape[0], tdtype=torch.int32, device=params.device)
        g = geometry_array(geom)
        hs_sur_coeffs(self.h, ptr(self.dev), N, G, D, Q, g.ctypes.data_as(_pf64), params.shape[0],
                      ptr(params), ptr(out), ptr(used), stream_ptr())
        return out

    def _check_batch(self, name, x):
        torch = _torch()
        if x.dim() != 2 or x.shape[1] != self.n_in:
            _fail(f"MLP.{name}: inputs must be (batch, {self.n_in})")
        if x.shape[0] > self.max_batch:
            _fail(f"MLP.{name}: batch {x.shape[0]} above max_batch {self.max_batch}")
        _check_vec(f"MLP.{name}: x", x, x.shape[0] * self.n_in, tdtype=torch.float64, device=self.dev.device)

    def train_step(self, x, target, lr: float, loss=None, grads=None):
        torch = _torch()
        self._check_batch("train_step", x)
        _check_vec("MLP.train_step: target", target, x.shape[0] * self.n_out, tdtype=torch.float64,
                   device=x.device)
        if loss is not None:
            _check_vec("MLP.train_step: loss", loss, 1, tdtype=torch.float32, device=x.device)
        if grads is not None:
            _check_vec("MLP.train_step: grads", grads, self.nparam, tdtype=torch.float32, device=x.device)
        hs_mlp_train_step(self.h, ptr(self.dev), x.shape[0], ptr(x), ptr(target), float(lr),
                          ptr(loss), ptr(grads), stream_ptr())

    def __del__(self):
        try:
            if getattr(self, "h", None):
                _lib.hs_mlp_destroy(self.h)
                self.h = None
        except Exception:
            pass
