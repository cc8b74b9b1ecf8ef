"""Thin ctypes binding of libexx.so (argument marshalling only).

Every function takes torch tensors that already live on the GPU, checks
their dtype, shape and contiguity, and passes raw device pointers plus the
current HIP stream to the C ABI declared in ``include/exx.h``. All arithmetic
runs in the library's HIP kernels; if the library is missing this module
raises at import time instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes
import pathlib

import torch

_LIB_PATH = pathlib.Path(__file__).resolve().parent / "libexx.so"

EXX_F64, EXX_F32, EXX_BF16, EXX_MIXED = 0, 1, 2, 3
PREC = {"f64": EXX_F64, "f32": EXX_F32, "bf16": EXX_BF16, "mixed": EXX_MIXED}
_STATUS = {
    0: "EXX_OK",
    -1: "EXX_ERR_ARG",
    -2: "EXX_ERR_SHAPE",
    -3: "EXX_ERR_NOMEM",
    -4: "EXX_ERR_NOT_PD",
    -5: "EXX_ERR_NONFINITE",
    -6: "EXX_ERR_DEVICE",
    -7: "EXX_ERR_UNSUPPORTED",
}

EXPORTED = (
    "exx_create",
    "exx_destroy",
    "exx_last_error",
    "exx_scratch_bytes",
    "exx_isdf_fit",
    "exx_coulomb_V",
    "exx_build_K",
    "exx_build",
    "exx_select_points",
    "exx_set_timing",
    "exx_set_refinement",
    "exx_phase_times",
    "exx_build_batched",
    "exx_mlp_features",
    "exx_mlp_forward",
    "exx_mlp_backward",
    "exx_mlp_adam",
    "exx_mlp_targets",
    "exx_mlp_nms",
    "exx_mlp_probe",
    "exx_select_points_mlp",
    "exx_workspace_size",
    "exx_set_workspace",
    "exx_set_checks",
    "exx_get_status",
    "exx_build_K_noalloc",
    "exx_save_tuning",
    "exx_load_tuning",
    "exx_set_contraction",
    "exx_set_fit",
    "exx_mlp_moments",
    "exx_exchange_gradient",
    "exx_build_robust",
)

EXX_BATCH_GRAPH, EXX_BATCH_TUNE, EXX_BATCH_CONCURRENT = 1, 2, 4
EXX_CALL_BUILD, EXX_CALL_SELECT, EXX_CALL_SELECT_MLP, EXX_CALL_GRADIENT = 0, 1, 2, 3
EXX_CHECK_FINITE, EXX_STRICT_PD, EXX_CHECK_SYNC = 1, 2, 4
EXX_ERR_NOT_PD, EXX_ERR_NONFINITE = -4, -5
EXX_CONTRACT_AUTO, EXX_CONTRACT_F64, EXX_CONTRACT_BF16, EXX_CONTRACT_BF16X3 = 0, 1, 2, 3
EXX_FIT_PER_Q, EXX_FIT_SHARED = 0, 1
EXX_MLP_NPARAM = 4481

PHASES = ("G", "S", "cholesky", "pinv", "gamma", "kcorr", "solve", "fft", "coulomb",
          "kconv", "K", "energy")


class ExxCell(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_double * 3),
        ("grid", ctypes.c_int32 * 3),
        ("kmesh", ctypes.c_int32 * 3),
        ("n_occ", ctypes.c_int32),
        ("n_ao", ctypes.c_int32),
        ("n_isdf", ctypes.c_int32),
    ]


class ExxBatchItem(ctypes.Structure):
    _fields_ = [
        ("cell", ExxCell),
        ("psi_grid", ctypes.c_void_p),
        ("occ_pts", ctypes.c_void_p),
        ("ao_pts", ctypes.c_void_p),
        ("pts", ctypes.c_void_p),
        ("K", ctypes.c_void_p),
        ("Ex", ctypes.c_void_p),
        ("rank", ctypes.c_void_p),
    ]


class ExxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not _LIB_PATH.exists():
        raise ImportError(
            f"{_LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
        )
    lib = ctypes.CDLL(str(_LIB_PATH))
    vp, i32p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)
    cellp = ctypes.POINTER(ExxCell)
    sig = {
        "exx_create": ([ctypes.POINTER(vp), ctypes.c_int], ctypes.c_int),
        "exx_destroy": ([vp], ctypes.c_int),
        "exx_last_error": ([vp], ctypes.c_char_p),
        "exx_scratch_bytes": ([vp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "exx_isdf_fit": ([vp, cellp, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "exx_coulomb_V": ([vp, cellp, ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
        "exx_build_K": ([vp, cellp, ctypes.c_int, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "exx_build": ([vp, cellp, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "exx_exchange_gradient": ([vp, cellp, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
                                  ctypes.c_int),
        "exx_build_robust": ([vp, cellp, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp],
                             ctypes.c_int),
        "exx_select_points": ([vp, cellp, vp, vp, vp, vp], ctypes.c_int),
        "exx_set_timing": ([vp, ctypes.c_int], ctypes.c_int),
        "exx_set_refinement": ([vp, ctypes.c_int32], ctypes.c_int),
        "exx_build_batched": ([vp, ctypes.c_int32, ctypes.POINTER(ExxBatchItem), ctypes.c_int,
                               ctypes.c_int32, vp], ctypes.c_int),
        "exx_phase_times": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                             ctypes.c_int32], ctypes.c_int),
        "exx_mlp_features": ([vp, cellp, vp, ctypes.POINTER(ctypes.c_double), vp, vp], ctypes.c_int),
        "exx_mlp_forward": ([vp, ctypes.c_int64, vp, vp, vp, vp], ctypes.c_int),
        "exx_mlp_backward": ([vp, ctypes.c_int64, vp, ctypes.c_int64, vp, vp, ctypes.c_float, vp,
                              vp, vp, vp], ctypes.c_int),
        "exx_mlp_adam": ([vp, ctypes.c_int32, vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float,
                          ctypes.c_float, ctypes.c_float, ctypes.c_float, vp], ctypes.c_int),
        "exx_mlp_targets": ([vp, cellp, vp, ctypes.c_int32, ctypes.c_double, vp, vp],
                            ctypes.c_int),
        "exx_mlp_nms": ([vp, cellp, vp, ctypes.c_int32, vp, vp], ctypes.c_int),
        "exx_mlp_probe": ([vp, cellp, vp, vp, ctypes.c_int32, ctypes.c_uint64, vp, vp],
                          ctypes.c_int),
        "exx_select_points_mlp": ([vp, cellp, vp, ctypes.POINTER(ctypes.c_double), vp,
                                   ctypes.c_double, ctypes.c_int32, vp, i32p,
                                   ctypes.POINTER(ctypes.c_double), vp], ctypes.c_int),
        "exx_workspace_size": ([vp, cellp, ctypes.c_int, ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "exx_set_workspace": ([vp, vp, ctypes.c_size_t], ctypes.c_int),
        "exx_set_checks": ([vp, ctypes.c_int32], ctypes.c_int),
        "exx_set_contraction": ([vp, ctypes.c_int32], ctypes.c_int),
        "exx_set_fit": ([vp, ctypes.c_int32], ctypes.c_int),
        "exx_mlp_moments": ([vp, ctypes.c_int64, vp, vp, vp], ctypes.c_int),
        "exx_get_status": ([vp, vp, i32p], ctypes.c_int),
        "exx_build_K_noalloc": ([vp, cellp, ctypes.c_int, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "exx_save_tuning": ([vp, ctypes.c_char_p], ctypes.c_int),
        "exx_load_tuning": ([vp, ctypes.c_char_p], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def library_path() -> str:
    return str(_LIB_PATH)


def make_cell(L, grid, kmesh, n_occ, n_ao, n_isdf) -> ExxCell:
    c = ExxCell()
    for i in range(3):
        c.L[i] = float(L[i])
        c.grid[i] = int(grid[i])
        c.kmesh[i] = int(kmesh[i])
    c.n_occ, c.n_ao, c.n_isdf = int(n_occ), int(n_ao), int(n_isdf)
    return c


def _nk(c: ExxCell) -> int:
    return c.kmesh[0] * c.kmesh[1] * c.kmesh[2]


def _ng(c: ExxCell) -> int:
    return c.grid[0] * c.grid[1] * c.grid[2]


def _ptr(t: torch.Tensor, name: str, dtype, shape, device) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _psi_dtype(prec: int):
    return torch.complex128 if prec in (EXX_F64, EXX_MIXED) else torch.complex64


def _xi_dtype(prec: int):
    return torch.complex128 if prec == EXX_F64 else torch.complex64


class Handle:
    """Owns an exx_handle_t bound to one GPU."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        st = _lib.exx_create(ctypes.byref(h), int(device))
        if st != 0:
            raise ExxError(st, f"exx_create(device={device}) failed")
        self._h = h
        self.device = torch.device("cuda", int(device))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.exx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != 0:
            raise ExxError(st, _lib.exx_last_error(self._h).decode())

    @property
    def raw(self):
        return self._h

    def set_refinement(self, steps: int):
        """Steps (0 or 1) of iterative refinement after every fit solve of this handle."""
        self._check(_lib.exx_set_refinement(self._h, int(steps)))

    def set_contraction(self, form: int):
        """Arithmetic of the Coulomb contraction on FP32-stored transforms
        (EXX_CONTRACT_AUTO, _F64, _BF16, _BF16X3)."""
        self._check(_lib.exx_set_contraction(self._h, int(form)))

    def set_fit(self, mode: int):
        """ISDF fit of the fused builds: EXX_FIT_PER_Q (default) or EXX_FIT_SHARED."""
        self._check(_lib.exx_set_fit(self._h, int(mode)))

    def set_timing(self, enable: bool, serial: bool = False):
        """Per-phase HIP events; serial also runs the normally overlapping phases one
        after another (exx_set_timing(h, 2))."""
        self._check(_lib.exx_set_timing(self._h, (2 if serial else 1) if enable else 0))

    def phase_times(self) -> dict:
        """{phase: (total_ms, calls)} since timing was enabled or last read."""
        n = len(PHASES)
        ms = (ctypes.c_double * n)()
        calls = (ctypes.c_int32 * n)()
        self._check(_lib.exx_phase_times(self._h, ms, calls, n))
        return {PHASES[i]: (ms[i], calls[i]) for i in range(n)}

    def scratch_bytes(self) -> int:
        b = ctypes.c_size_t()
        self._check(_lib.exx_scratch_bytes(self._h, ctypes.byref(b)))
        return b.value

    def workspace_size(self, cell: ExxCell, prec: int, call: int = EXX_CALL_BUILD) -> int:
        """Scratch bytes one kind of call needs for this cell (exx_workspace_size)."""
        b = ctypes.c_size_t()
        self._check(_lib.exx_workspace_size(self._h, ctypes.byref(cell), int(prec), int(call),
                                            ctypes.byref(b)))
        return b.value

    def set_workspace(self, buf):
        """Use a caller-owned device buffer (a uint8 torch tensor on this device) as the
        handle's scratch; None returns to library-owned scratch. The handle keeps a
        reference to the tensor while it is in use."""
        if buf is None:
            self._check(_lib.exx_set_workspace(self._h, None, 0))
            self._ws = None
            return
        if not isinstance(buf, torch.Tensor) or buf.device != self.device or not buf.is_contiguous():
            raise ValueError("workspace must be a contiguous tensor on the handle's device")
        self._check(_lib.exx_set_workspace(self._h, buf.data_ptr(),
                                           buf.numel() * buf.element_size()))
        self._ws = buf

    def save_tuning(self, path: str):
        """Write the autotuned tile table (exx_save_tuning)."""
        self._check(_lib.exx_save_tuning(self._h, str(path).encode()))

    def load_tuning(self, path: str):
        """Read a tile table written by save_tuning (exx_load_tuning)."""
        self._check(_lib.exx_load_tuning(self._h, str(path).encode()))

    def set_checks(self, flags: int):
        self._check(_lib.exx_set_checks(self._h, int(flags)))

    def status(self, stream=None):
        """exx_get_status on `stream` (current stream by default): returns
        (status code, first transfer that lost a pivot or -1, non-finite site or 0)
        without raising."""
        info = (ctypes.c_int32 * 2)()
        st = (stream.cuda_stream if stream is not None else _stream(self.device))
        code = _lib.exx_get_status(self._h, st, info)
        return code, info[0], info[1]


def exx_isdf_fit(h: Handle, cell: ExxCell, prec: int, psi_grid, occ_pts, pts, xi, S, rank):
    nk, ng, ni, no = _nk(cell), _ng(cell), cell.n_isdf, cell.n_occ
    d = h.device
    args = (
        _ptr(psi_grid, "psi_grid", _psi_dtype(prec), (nk, no, ng), d),
        _ptr(occ_pts, "occ_pts", torch.complex128, (nk, ni, no), d),
        _ptr(pts, "pts", torch.int32, (ni,), d),
        _ptr(xi, "xi", _xi_dtype(prec), (nk, ni, ng), d),
        _ptr(S, "S", torch.complex128, (nk, ni, ni), d),
        _ptr(rank, "rank", torch.int32, (nk,), d),
    )
    h._check(_lib.exx_isdf_fit(h.raw, ctypes.byref(cell), prec, *args, _stream(d)))


def exx_coulomb_V(h: Handle, cell: ExxCell, prec: int, xi, pts, V):
    nk, ng, ni = _nk(cell), _ng(cell), cell.n_isdf
    d = h.device
    args = (
        _ptr(xi, "xi", _xi_dtype(prec), (nk, ni, ng), d),
        _ptr(pts, "pts", torch.int32, (ni,), d),
        _ptr(V, "V", torch.complex128, (nk, ni, ni), d),
    )
    h._check(_lib.exx_coulomb_V(h.raw, ctypes.byref(cell), prec, *args, _stream(d)))


def exx_build_K(h: Handle, cell: ExxCell, prec: int, ao_pts, occ_pts, V, K, Ex):
    nk, ni, no, na = _nk(cell), cell.n_isdf, cell.n_occ, cell.n_ao
    d = h.device
    args = (
        _ptr(ao_pts, "ao_pts", torch.complex128, (nk, ni, na), d),
        _ptr(occ_pts, "occ_pts", torch.complex128, (nk, ni, no), d),
        _ptr(V, "V", torch.complex128, (nk, ni, ni), d),
        _ptr(K, "K", torch.complex128, (nk, na, na), d),
        _ptr(Ex, "Ex", torch.float64, (1,), d),
    )
    h._check(_lib.exx_build_K(h.raw, ctypes.byref(cell), prec, *args, _stream(d)))


def exx_build_K_noalloc(h: Handle, cell: ExxCell, prec: int, ao_pts, occ_pts, V, K, Ex):
    """exx_build_K on the library's fixed per-GPU scratch (no device allocation)."""
    nk, ni, no, na = _nk(cell), cell.n_isdf, cell.n_occ, cell.n_ao
    d = h.device
    args = (
        _ptr(ao_pts, "ao_pts", torch.complex128, (nk, ni, na), d),
        _ptr(occ_pts, "occ_pts", torch.complex128, (nk, ni, no), d),
        _ptr(V, "V", torch.complex128, (nk, ni, ni), d),
        _ptr(K, "K", torch.complex128, (nk, na, na), d),
        _ptr(Ex, "Ex", torch.float64, (1,), d),
    )
    h._check(_lib.exx_build_K_noalloc(h.raw, ctypes.byref(cell), prec, *args, _stream(d)))


def exx_build(h: Handle, cell: ExxCell, prec: int, psi_grid, occ_pts, ao_pts, pts, K, Ex, rank):
    nk, ng, ni, no, na = _nk(cell), _ng(cell), cell.n_isdf, cell.n_occ, cell.n_ao
    d = h.device
    args = (
        _ptr(psi_grid, "psi_grid", _psi_dtype(prec), (nk, no, ng), d),
        _ptr(occ_pts, "occ_pts", torch.complex128, (nk, ni, no), d),
        _ptr(ao_pts, "ao_pts", torch.complex128, (nk, ni, na), d),
        _ptr(pts, "pts", torch.int32, (ni,), d),
        _ptr(K, "K", torch.complex128, (nk, na, na), d),
        _ptr(Ex, "Ex", torch.float64, (1,), d),
        _ptr(rank, "rank", torch.int32, (nk,), d),
    )
    h._check(_lib.exx_build(h.raw, ctypes.byref(cell), prec, *args, _stream(d)))


def exx_exchange_gradient(h: Handle, cell: ExxCell, psi_grid, occ_pts, ao_pts, ao_grid, pts, K,
                          Kgrad, Ex, rank, prec: int = EXX_F64):
    """K, E_x and the density derivative Kgrad of the fitted exchange energy
    (prec EXX_F64 or EXX_MIXED)."""
    nk, ng, ni, no, na = _nk(cell), _ng(cell), cell.n_isdf, cell.n_occ, cell.n_ao
    d = h.device
    args = (
        _ptr(psi_grid, "psi_grid", torch.complex128, (nk, no, ng), d),
        _ptr(occ_pts, "occ_pts", torch.complex128, (nk, ni, no), d),
        _ptr(ao_pts, "ao_pts", torch.complex128, (nk, ni, na), d),
        _ptr(ao_grid, "ao_grid", torch.complex128, (nk, na, ng), d),
        _ptr(pts, "pts", torch.int32, (ni,), d),
        _ptr(K, "K", torch.complex128, (nk, na, na), d),
        _ptr(Kgrad, "Kgrad", torch.complex128, (nk, na, na), d),
        _ptr(Ex, "Ex", torch.float64, (1,), d),
        _ptr(rank, "rank", torch.int32, (nk,), d),
    )
    h._check(_lib.exx_exchange_gradient(h.raw, ctypes.byref(cell), prec, *args, _stream(d)))


def exx_build_robust(h: Handle, cell: ExxCell, psi_grid, occ_pts, ao_pts, ao_grid, pts, K, Ex,
                     rank, prec: int = EXX_F64):
    """The robust-fit exchange matrix K_rob and E_x (prec EXX_F64 or EXX_MIXED)."""
    nk, ng, ni, no, na = _nk(cell), _ng(cell), cell.n_isdf, cell.n_occ, cell.n_ao
    d = h.device
    args = (
        _ptr(psi_grid, "psi_grid", torch.complex128, (nk, no, ng), d),
        _ptr(occ_pts, "occ_pts", torch.complex128, (nk, ni, no), d),
        _ptr(ao_pts, "ao_pts", torch.complex128, (nk, ni, na), d),
        _ptr(ao_grid, "ao_grid", torch.complex128, (nk, na, ng), d),
        _ptr(pts, "pts", torch.int32, (ni,), d),
        _ptr(K, "K", torch.complex128, (nk, na, na), d),
        _ptr(Ex, "Ex", torch.float64, (1,), d),
        _ptr(rank, "rank", torch.int32, (nk,), d),
    )
    h._check(_lib.exx_build_robust(h.raw, ctypes.byref(cell), prec, *args, _stream(d)))


def exx_select_points(h: Handle, cell: ExxCell, psi_grid, pts, n_pivot):
    nk, ng, ni, no = _nk(cell), _ng(cell), cell.n_isdf, cell.n_occ
    d = h.device
    args = (
        _ptr(psi_grid, "psi_grid", torch.complex128, (nk, no, ng), d),
        _ptr(pts, "pts", torch.int32, (ni,), d),
        _ptr(n_pivot, "n_pivot", torch.int32, (1,), d),
    )
    h._check(_lib.exx_select_points(h.raw, ctypes.byref(cell), *args, _stream(d)))


def exx_build_batched(h: Handle, items, prec: int, flags: int = 0, stream=None):
    """Run many K-builds. ``items``: list of dicts with keys cell, psi_grid, occ_pts,
    ao_pts, pts, K, Ex, rank (device tensors as for exx_build). ``stream``: a
    torch.cuda.Stream (required with EXX_BATCH_GRAPH; the current stream otherwise)."""
    d = h.device
    arr = (ExxBatchItem * len(items))()
    for i, it in enumerate(items):
        c = it["cell"]
        nk, ng, ni, no, na = _nk(c), _ng(c), c.n_isdf, c.n_occ, c.n_ao
        arr[i].cell = c
        arr[i].psi_grid = _ptr(it["psi_grid"], "psi_grid", _psi_dtype(prec), (nk, no, ng), d)
        arr[i].occ_pts = _ptr(it["occ_pts"], "occ_pts", torch.complex128, (nk, ni, no), d)
        arr[i].ao_pts = _ptr(it["ao_pts"], "ao_pts", torch.complex128, (nk, ni, na), d)
        arr[i].pts = _ptr(it["pts"], "pts", torch.int32, (ni,), d)
        arr[i].K = _ptr(it["K"], "K", torch.complex128, (nk, na, na), d)
        arr[i].Ex = _ptr(it["Ex"], "Ex", torch.float64, (1,), d)
        arr[i].rank = _ptr(it["rank"], "rank", torch.int32, (nk,), d)
    if stream is None:
        if flags & EXX_BATCH_GRAPH:
            raise ValueError("EXX_BATCH_GRAPH needs an explicit non-default torch.cuda.Stream")
        st = _stream(d)
    else:
        st = stream.cuda_stream
    h._check(_lib.exx_build_batched(h.raw, len(items), arr, prec, flags, st))


# ---------------------------------------------------------------------------
# learned selector
# ---------------------------------------------------------------------------
def _norm6(norm):
    vals = [float(x) for x in norm]
    if len(vals) != 6:
        raise ValueError("norm must hold 6 numbers (mean, scale) x 3")
    return (ctypes.c_double * 6)(*vals)


def exx_mlp_features(h: Handle, cell: ExxCell, psi_grid, norm, feat):
    nk, ng, no = _nk(cell), _ng(cell), cell.n_occ
    d = h.device
    args = (_ptr(psi_grid, "psi_grid", torch.complex128, (nk, no, ng), d), _norm6(norm),
            _ptr(feat, "feat", torch.float32, (ng, 3), d))
    h._check(_lib.exx_mlp_features(h.raw, ctypes.byref(cell), *args, _stream(d)))


def exx_mlp_forward(h: Handle, feat, theta, score):
    d = h.device
    n = feat.shape[0]
    args = (_ptr(feat, "feat", torch.float32, (n, 3), d),
            _ptr(theta, "theta", torch.float32, (EXX_MLP_NPARAM,), d),
            _ptr(score, "score", torch.float32, (n,), d))
    h._check(_lib.exx_mlp_forward(h.raw, n, *args, _stream(d)))


def exx_mlp_moments(h: Handle, feat, sums):
    """sums[:3] += column sums, sums[3:] += column sums of squares of feat (n, 3)."""
    d = h.device
    n = feat.shape[0]
    args = (_ptr(feat, "feat", torch.float32, (n, 3), d),
            _ptr(sums, "sums", torch.float64, (6,), d))
    h._check(_lib.exx_mlp_moments(h.raw, n, *args, _stream(d)))


def exx_mlp_backward(h: Handle, feat, target, wpos: float, theta, grad, loss, idx=None):
    """Gradient over rows idx of (feat, target), or all rows when idx is None."""
    d = h.device
    rows = feat.shape[0]
    n = rows if idx is None else idx.shape[0]
    if idx is not None:
        _ptr(idx, "idx", torch.int32, (n,), d)
    args = (None if idx is None else idx.data_ptr(), rows,
            _ptr(feat, "feat", torch.float32, (rows, 3), d),
            _ptr(target, "target", torch.float32, (rows,), d), float(wpos),
            _ptr(theta, "theta", torch.float32, (EXX_MLP_NPARAM,), d),
            _ptr(grad, "grad", torch.float32, (EXX_MLP_NPARAM,), d),
            _ptr(loss, "loss", torch.float64, (1,), d))
    h._check(_lib.exx_mlp_backward(h.raw, n, *args, _stream(d)))


def exx_mlp_adam(h: Handle, theta, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999,
                 eps=1e-8):
    d = h.device
    n = theta.shape[0]
    args = [_ptr(t, name, torch.float32, (n,), d)
            for t, name in ((theta, "theta"), (grad, "grad"), (m, "m"), (v, "v"))]
    h._check(_lib.exx_mlp_adam(h.raw, n, *args, int(step), float(lr), float(beta1), float(beta2),
                               float(eps), _stream(d)))


def exx_mlp_targets(h: Handle, cell: ExxCell, pts, sigma: float, target):
    d = h.device
    npts = pts.shape[0]
    args = (_ptr(pts, "pts", torch.int32, (npts,), d), npts, float(sigma),
            _ptr(target, "target", torch.float32, (_ng(cell),), d))
    h._check(_lib.exx_mlp_targets(h.raw, ctypes.byref(cell), *args, _stream(d)))


def exx_mlp_nms(h: Handle, cell: ExxCell, score, pts):
    d = h.device
    k = pts.shape[0]
    args = (_ptr(score, "score", torch.float32, (_ng(cell),), d), k,
            _ptr(pts, "pts", torch.int32, (k,), d))
    h._check(_lib.exx_mlp_nms(h.raw, ctypes.byref(cell), *args, _stream(d)))


def exx_mlp_probe(h: Handle, cell: ExxCell, psi_grid, pts, n_probe: int, seed: int, resid):
    nk, ng, no, ni = _nk(cell), _ng(cell), cell.n_occ, cell.n_isdf
    d = h.device
    args = (_ptr(psi_grid, "psi_grid", torch.complex128, (nk, no, ng), d),
            _ptr(pts, "pts", torch.int32, (ni,), d), int(n_probe), int(seed) & (2**64 - 1),
            _ptr(resid, "resid", torch.float64, (1,), d))
    h._check(_lib.exx_mlp_probe(h.raw, ctypes.byref(cell), *args, _stream(d)))


def exx_select_points_mlp(h: Handle, cell: ExxCell, psi_grid, norm, theta, tau: float,
                          n_probe: int, pts):
    """Returns (used_fallback: bool, residual: float); pts is filled in place."""
    nk, ng, no, ni = _nk(cell), _ng(cell), cell.n_occ, cell.n_isdf
    d = h.device
    used = ctypes.c_int32(0)
    resid = ctypes.c_double(0.0)
    args = (_ptr(psi_grid, "psi_grid", torch.complex128, (nk, no, ng), d), _norm6(norm),
            _ptr(theta, "theta", torch.float32, (EXX_MLP_NPARAM,), d), float(tau), int(n_probe),
            _ptr(pts, "pts", torch.int32, (ni,), d), ctypes.byref(used), ctypes.byref(resid))
    h._check(_lib.exx_select_points_mlp(h.raw, ctypes.byref(cell), *args, _stream(d)))
    return bool(used.value), float(resid.value)
