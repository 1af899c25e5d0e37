"""Python binding of libspw (ctypes).  Argument marshalling only: every product
runs in the library's HIP kernels.  torch is used for device memory and
streams; it is imported first so that libspw binds to the same HIP runtime.

The functions mirror the C ABI in include/spw.h; ``SpwMatrix`` is a small
convenience wrapper over them.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspw.so")

SPW_OK = 0
STATUS_NAMES = ["SPW_OK", "SPW_ERR_INVALID_ARG", "SPW_ERR_BAD_MATRIX", "SPW_ERR_OUT_OF_MEMORY",
                "SPW_ERR_BUDGET", "SPW_ERR_DEVICE", "SPW_ERR_UNSUPPORTED", "SPW_ERR_BUSY",
                "SPW_ERR_TIMEOUT", "SPW_ERR_SHUTDOWN"]
SPW_CSC, SPW_CSR = 0, 1
SPW_F64, SPW_F32, SPW_BF16 = 0, 1, 2
SPW_PART_NONZERO, SPW_PART_COLUMN, SPW_PART_MERGE = 0, 1, 2
DTYPES = {SPW_F64: torch.float64, SPW_F32: torch.float32}


class SpwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        self.status_name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__("%s: %s" % (self.status_name, msg))


class CreateOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("value_storage", ctypes.c_int),
                ("chunk_nnz", ctypes.c_int32), ("relabel", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("panel_rows", ctypes.c_int32),
                ("device", ctypes.c_int32), ("transpose", ctypes.c_int32), ("partition", ctypes.c_int),
                ("canonicalize", ctypes.c_int32), ("wg_size", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class MatrixInfo(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("format", ctypes.c_int), ("value_storage", ctypes.c_int),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("inner_rows", ctypes.c_int64), ("inner_cols", ctypes.c_int64),
                ("chunk_nnz", ctypes.c_int64), ("n_chunks", ctypes.c_int64), ("n_zones", ctypes.c_int64),
                ("n_panels", ctypes.c_int64), ("panel_rows", ctypes.c_int64),
                ("mv_workgroups", ctypes.c_int64), ("index_bytes", ctypes.c_int64),
                ("relabeled", ctypes.c_int32), ("device", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("has_transpose", ctypes.c_int32), ("partition", ctypes.c_int), ("workers", ctypes.c_int64),
                ("worker_max_nnz", ctypes.c_int64), ("worker_min_nnz", ctypes.c_int64),
                ("wg_size_f64", ctypes.c_int32), ("wg_size_f32", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("fingerprint", ctypes.c_uint64)]


SPW_OP_MV, SPW_OP_VTM = 0, 1
SPW_PLAN_AUTO, SPW_PLAN_SINGLE, SPW_PLAN_PASSES, SPW_PLAN_TILE = 0, 1, 2, 3
PLAN_NAMES = {SPW_PLAN_SINGLE: "single", SPW_PLAN_PASSES: "passes", SPW_PLAN_TILE: "tile"}


class ServeOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_inflight", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64), ("streams", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("max_batch_cols", ctypes.c_int32), ("device", ctypes.c_int32), ("start_paused", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 7)]


class Request(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("matrix", ctypes.c_int32), ("op", ctypes.c_int),
                ("vdt", ctypes.c_int), ("k", ctypes.c_int32), ("in_", ctypes.c_void_p), ("ldi", ctypes.c_int64),
                ("out", ctypes.c_void_p), ("ldo", ctypes.c_int64), ("tag", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32)] + \
        [(n, ctypes.c_int64) for n in ("submitted", "completed", "rejected_busy", "groups", "merged_requests",
                                       "passes", "inflight", "registered", "hbm_budget_bytes", "hbm_used_bytes")] + \
        [(n, ctypes.c_double) for n in ("latency_p50_us", "latency_p99_us", "latency_mean_us", "model_bytes",
                                        "busy_seconds", "gbps")]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


# Every symbol include/spw.h declares, with (restype, argtypes).
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
SIGNATURES = {
    "spw_create_opts_default": (ctypes.c_int, [ctypes.POINTER(CreateOpts)]),
    "spw_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int, _I64, _I64, _I64, _VP, _VP, _VP,
                                  ctypes.POINTER(CreateOpts)]),
    "spw_create_coo": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int, _I64, _I64, _I64, _VP, _VP, _VP,
                                      ctypes.POINTER(CreateOpts)]),
    "spw_destroy": (ctypes.c_int, [_VP]),
    "spw_info": (ctypes.c_int, [_VP, ctypes.POINTER(MatrixInfo)]),
    "spw_mv": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "spw_vtm": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, _VP]),
    "spw_mv_batch": (ctypes.c_int, [_VP, ctypes.c_int, _I32, _VP, _I64, _VP, _I64, _VP]),
    "spw_vtm_batch": (ctypes.c_int, [_VP, ctypes.c_int, _I32, _VP, _I64, _VP, _I64, _VP]),
    "spw_round_values": (ctypes.c_int, [ctypes.c_int, _I64, _VP, _VP]),
    "spw_batch_plan": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _I32, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(_I32)]),
    "spw_set_batch_plan": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _I32, ctypes.c_int]),
    "spw_probe_bandwidth": (ctypes.c_int, [_VP, _VP, _I64, _I32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), _VP]),
    "spw_tune_cache_path": (ctypes.c_int, [ctypes.c_char_p]),
    "spw_tune_cache_clear": (ctypes.c_int, []),
    "spw_tune_cache_put": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_char_p, _I32]),
    "spw_tune_cache_get": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_char_p, ctypes.POINTER(_I32),
                                          ctypes.POINTER(_I32)]),
    "spw_matrix_fingerprint": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _I64, _I64, _I64, _VP, _VP,
                                              ctypes.POINTER(ctypes.c_uint64)]),
    "spw_cgls": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP, ctypes.c_int32, _VP, _VP]),
    "spw_serve_opts_default": (ctypes.c_int, [ctypes.POINTER(ServeOpts)]),
    "spw_serve_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(ServeOpts)]),
    "spw_serve_register": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(_I32)]),
    "spw_serve_submit": (ctypes.c_int, [_VP, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "spw_serve_resume": (ctypes.c_int, [_VP]),
    "spw_serve_poll": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(_I32)]),
    "spw_serve_wait": (ctypes.c_int, [_VP, ctypes.c_uint64, _I64]),
    "spw_serve_stats": (ctypes.c_int, [_VP, ctypes.POINTER(ServerStats)]),
    "spw_serve_destroy": (ctypes.c_int, [_VP]),
    "spw_plan_zones": (ctypes.c_int, [_I64, _VP, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                      _VP, _VP, _VP, _VP]),
    "spw_profile_enable": (ctypes.c_int, [_I32]),
    "spw_profile_select": (ctypes.c_int, [ctypes.c_char_p]),
    "spw_profile_reset": (ctypes.c_int, []),
    "spw_profile_read": (ctypes.c_int, [ctypes.POINTER(ProfileEntry), _I32, ctypes.POINTER(_I32)]),
    "spw_last_error": (ctypes.c_char_p, []),
    "spw_status_string": (ctypes.c_char_p, [ctypes.c_int]),
}

_lib = None


def load(path: str | None = None):
    """Load libspw.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError("libspw.so is not built (%s); run __graft_entry__.build()" % p)
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(status: int):
    if status != SPW_OK:
        raise SpwError(status, load().spw_last_error().decode(errors="replace"))


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def create_opts(**kw) -> CreateOpts:
    o = CreateOpts()
    _check(load().spw_create_opts_default(ctypes.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def spw_create(fmt: int, m: int, n: int, ptr, idx, val, opts: CreateOpts | None = None) -> int:
    """Create a matrix from host arrays (numpy); returns the opaque handle."""
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    nnz = int(idx.size)
    h = _VP()
    _check(load().spw_create(ctypes.byref(h), fmt, m, n, nnz, ptr.ctypes.data, idx.ctypes.data,
                             val.ctypes.data, ctypes.byref(opts) if opts is not None else None))
    return h.value


def spw_create_coo(fmt: int, m: int, n: int, rows, cols, val, opts: CreateOpts | None = None) -> int:
    """Create a matrix from coordinate triples (numpy, any order); returns the handle."""
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    if not (rows.size == cols.size == val.size):
        raise ValueError("rows, cols and val must have the same length")
    h = _VP()
    _check(load().spw_create_coo(ctypes.byref(h), fmt, m, n, int(val.size), rows.ctypes.data, cols.ctypes.data,
                                 val.ctypes.data, ctypes.byref(opts) if opts is not None else None))
    return h.value


def spw_destroy(h: int):
    _shapes.pop(h, None)
    _check(load().spw_destroy(h))


def spw_info(h: int) -> dict:
    info = MatrixInfo()
    info.struct_size = ctypes.sizeof(MatrixInfo)
    _check(load().spw_info(h, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in MatrixInfo._fields_ if name not in ("struct_size", "reserved")}


def _vec_dtype(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return SPW_F64
    if t.dtype == torch.float32:
        return SPW_F32
    raise TypeError("vectors must be float64 or float32 tensors")


def _dev(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)


# (m, n, device ordinal) of every live handle, so that the product calls can
# check their tensors against the matrix without a library call.
_shapes: dict = {}


def _shape(h: int):
    sh = _shapes.get(h)
    if sh is None:
        info = spw_info(h)
        sh = (info["m"], info["n"], info["device"])
        _shapes[h] = sh
    return sh


def check_operands(inp: torch.Tensor, out: torch.Tensor, in_len: int, out_len: int, device,
                   batch: bool, names=("in", "out")) -> int:
    """Checks a product's input and output tensors before any pointer reaches
    the library: float64 or float32, the same type on both sides, the lengths
    the matrix fixes, on `device` (a device ordinal; None skips the check).
    Single-vector operands are 1-D and contiguous; multi-RHS operands are 2-D
    (rows x k) with unit column stride and a row stride >= k (a 1-D tensor
    counts as k = 1).  Raises ValueError (TypeError for a wrong element type)
    and returns k."""
    ni, no = names
    _vec_dtype(inp)
    if out.dtype != inp.dtype:
        raise ValueError("%s is %s but %s is %s: the two must have the same type"
                         % (no, out.dtype, ni, inp.dtype))
    for t, nm in ((inp, ni), (out, no)):
        if device is not None and (not t.is_cuda or t.device.index != device):
            raise ValueError("%s must be on cuda:%d (the matrix's device), not %s" % (nm, device, t.device))
    if not batch or (inp.dim() == 1 and out.dim() == 1):
        for t, nm, ln in ((inp, ni, in_len), (out, no, out_len)):
            if t.dim() != 1:
                raise ValueError("%s must be 1-D, got shape %s" % (nm, tuple(t.shape)))
            if t.numel() != ln:
                raise ValueError("%s must have %d entries, got %d" % (nm, ln, t.numel()))
            if ln > 1 and t.stride(0) != 1:
                raise ValueError("%s must be contiguous (stride %d)" % (nm, t.stride(0)))
        return 1
    if inp.dim() != 2 or out.dim() != 2:
        raise ValueError("%s and %s must both be 2-D (rows x k), got shapes %s and %s"
                         % (ni, no, tuple(inp.shape), tuple(out.shape)))
    k = inp.shape[1]
    for t, nm, ln in ((inp, ni, in_len), (out, no, out_len)):
        if tuple(t.shape) != (ln, k):
            raise ValueError("%s must have shape (%d, %d), got %s" % (nm, ln, k, tuple(t.shape)))
        if k > 1 and t.stride(1) != 1:
            raise ValueError("%s must be row-major with unit column stride (strides %s)" % (nm, t.stride()))
        if ln > 1 and t.stride(0) < k:
            raise ValueError("%s row stride %d is below k = %d" % (nm, t.stride(0), k))
    return k


def _ld(t: torch.Tensor) -> int:
    return 1 if t.dim() == 1 else max(t.stride(0), t.shape[1])


def spw_mv(h: int, x: torch.Tensor, y: torch.Tensor, stream=None):
    m, n, dev = _shape(h)
    check_operands(x, y, n, m, dev, False, ("x", "y"))
    _check(load().spw_mv(h, _vec_dtype(x), x.data_ptr(), y.data_ptr(), _stream_ptr(stream)))


def spw_vtm(h: int, v: torch.Tensor, u: torch.Tensor, stream=None):
    m, n, dev = _shape(h)
    check_operands(v, u, m, n, dev, False, ("v", "u"))
    _check(load().spw_vtm(h, _vec_dtype(v), v.data_ptr(), u.data_ptr(), _stream_ptr(stream)))


def spw_mv_batch(h: int, X: torch.Tensor, Y: torch.Tensor, stream=None):
    m, n, dev = _shape(h)
    k = check_operands(X, Y, n, m, dev, True, ("X", "Y"))
    _check(load().spw_mv_batch(h, _vec_dtype(X), k, X.data_ptr(), _ld(X), Y.data_ptr(), _ld(Y),
                               _stream_ptr(stream)))


def spw_vtm_batch(h: int, V: torch.Tensor, U: torch.Tensor, stream=None):
    m, n, dev = _shape(h)
    k = check_operands(V, U, m, n, dev, True, ("V", "U"))
    _check(load().spw_vtm_batch(h, _vec_dtype(V), k, V.data_ptr(), _ld(V), U.data_ptr(), _ld(U),
                                _stream_ptr(stream)))


def spw_cgls(h: int, b: torch.Tensor, x: torch.Tensor, iters: int, hist: bool = True, stream=None):
    """CGLS on min ||b - A x||_2 in place on x (float64 device tensors).  With
    hist, returns (gamma, rho): ||A^T r_k||^2 and ||r_k||^2 for k = 0 .. iters."""
    m, n, dev = _shape(h)
    if b.dtype != torch.float64 or x.dtype != torch.float64:
        raise ValueError("spw_cgls takes float64 vectors")
    check_operands(b, x, m, n, dev, False, ("b", "x"))
    out = np.empty(2 * (iters + 1), dtype=np.float64) if hist else None
    _check(load().spw_cgls(h, SPW_F64, b.data_ptr(), x.data_ptr(), int(iters),
                           out.ctypes.data if hist else None, _stream_ptr(stream)))
    if not hist:
        return None
    return out[:iters + 1].copy(), out[iters + 1:].copy()


def spw_batch_plan(h: int, op: int, vdt: int, k: int):
    """(plan, tuned) that a k-column call of op with vector type vdt takes now."""
    plan, tuned = ctypes.c_int(), _I32()
    _check(load().spw_batch_plan(h, op, vdt, k, ctypes.byref(plan), ctypes.byref(tuned)))
    return plan.value, bool(tuned.value)


def spw_set_batch_plan(h: int, op: int, vdt: int, k: int, plan: int):
    _check(load().spw_set_batch_plan(h, op, vdt, k, plan))


def spw_probe_bandwidth(src: torch.Tensor, dst: torch.Tensor | None = None, reps: int = 5, stream=None):
    """Median ms of the library's read-only stream over src (and of a copy into
    dst when given): (read_ms, copy_ms or None)."""
    nbytes = src.numel() * src.element_size()
    if dst is not None and dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    r, c = ctypes.c_double(), ctypes.c_double()
    _check(load().spw_probe_bandwidth(src.data_ptr(), dst.data_ptr() if dst is not None else None, nbytes, reps,
                                      ctypes.byref(r), ctypes.byref(c), _stream_ptr(stream)))
    return r.value, (c.value if dst is not None else None)


def spw_tune_cache_path(path: str | None):
    """Use `path` as the tuning cache file (None: memory only) and load its records."""
    _check(load().spw_tune_cache_path(path.encode() if path else None))


def spw_round_values(storage: int, val) -> np.ndarray:
    """Host-only: the values spw_create stores for `storage`, promoted to float64."""
    val = np.ascontiguousarray(val, dtype=np.float64)
    out = np.empty_like(val)
    _check(load().spw_round_values(storage, val.size, val.ctypes.data, out.ctypes.data))
    return out


def spw_plan_zones(n: int, ptr, chunk_nnz: int):
    """Host-only chunk/zone plan: (owned[n_chunks+1], zone_col, zone_first, zone_last)."""
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    nc, nz = _I64(), _I64()
    lib = load()
    _check(lib.spw_plan_zones(n, ptr.ctypes.data, chunk_nnz, ctypes.byref(nc), ctypes.byref(nz),
                              None, None, None, None))
    owned = np.empty(nc.value + 1, dtype=np.int64)
    zc = np.empty(max(nz.value, 1), dtype=np.int64)
    zf = np.empty_like(zc)
    zl = np.empty_like(zc)
    _check(lib.spw_plan_zones(n, ptr.ctypes.data, chunk_nnz, ctypes.byref(nc), ctypes.byref(nz),
                              owned.ctypes.data, zc.ctypes.data, zf.ctypes.data, zl.ctypes.data))
    k = nz.value
    return owned, zc[:k].copy(), zf[:k].copy(), zl[:k].copy()


def spw_profile_enable(on: bool):
    _check(load().spw_profile_enable(1 if on else 0))


def spw_profile_select(prefix: str | None):
    """Time only kernels whose name begins with prefix (None: every kernel)."""
    _check(load().spw_profile_select(prefix.encode() if prefix else None))


def spw_profile_reset():
    _check(load().spw_profile_reset())


def spw_profile_read() -> dict:
    lib = load()
    cnt = _I32()
    _check(lib.spw_profile_read(None, 0, ctypes.byref(cnt)))
    arr = (ProfileEntry * max(cnt.value, 1))()
    _check(lib.spw_profile_read(arr, cnt.value, ctypes.byref(cnt)))
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(cnt.value)}


class SpwMatrix:
    """A created matrix.  `fmt` is SPW_CSC (wide, m x n, ptr over columns) or
    SPW_CSR (tall, m x n, ptr over rows)."""

    def __init__(self, fmt: int, m: int, n: int, ptr, idx, val, **opts):
        self.fmt, self.m, self.n = fmt, m, n
        self.handle = None
        self.handle = spw_create(fmt, m, n, ptr, idx, val, create_opts(**opts) if opts else None)

    @classmethod
    def from_coo(cls, fmt: int, m: int, n: int, rows, cols, val, **opts) -> "SpwMatrix":
        """A matrix from (row, column, value) triples in any order; see spw_create_coo."""
        self = cls.__new__(cls)
        self.fmt, self.m, self.n = fmt, m, n
        self.handle = None
        self.handle = spw_create_coo(fmt, m, n, rows, cols, val, create_opts(**opts) if opts else None)
        return self

    def info(self) -> dict:
        return spw_info(self.handle)

    def mv(self, x: torch.Tensor, y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if y is None:
            y = torch.empty(self.m, dtype=x.dtype, device=x.device)
        spw_mv(self.handle, x, y, stream)
        return y

    def vtm(self, v: torch.Tensor, u: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if u is None:
            u = torch.empty(self.n, dtype=v.dtype, device=v.device)
        spw_vtm(self.handle, v, u, stream)
        return u

    def mv_batch(self, X: torch.Tensor, Y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if Y is None:
            Y = torch.empty((self.m, X.shape[1]), dtype=X.dtype, device=X.device)
        spw_mv_batch(self.handle, X, Y, stream)
        return Y

    def vtm_batch(self, V: torch.Tensor, U: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if U is None:
            U = torch.empty((self.n, V.shape[1]), dtype=V.dtype, device=V.device)
        spw_vtm_batch(self.handle, V, U, stream)
        return U

    def batch_plan(self, op: int, vdt: int, k: int):
        """(plan, tuned) of a k-column call; see spw_batch_plan."""
        return spw_batch_plan(self.handle, op, vdt, k)

    def set_batch_plan(self, op: int, vdt: int, k: int, plan: int):
        spw_set_batch_plan(self.handle, op, vdt, k, plan)

    def cgls(self, b: torch.Tensor, x: torch.Tensor, iters: int, hist: bool = True, stream=None):
        """CGLS iterations on min ||b - A x||_2, in place on x; see spw_cgls."""
        return spw_cgls(self.handle, b, x, iters, hist, stream)

    def close(self):
        if self.handle:
            spw_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A serving instance over resident matrices (see the serving part of
    include/spw.h).  Requests keep references to their tensors until they
    are waited for."""

    def __init__(self, **opts):
        o = ServeOpts()
        _check(load().spw_serve_opts_default(ctypes.byref(o)))
        for k, v in opts.items():
            setattr(o, k, v)
        h = _VP()
        _check(load().spw_serve_create(ctypes.byref(h), ctypes.byref(o)))
        self.handle = h.value
        self._keep = {}
        self._shapes = {}

    def register(self, M: SpwMatrix) -> int:
        out = _I32()
        _check(load().spw_serve_register(self.handle, M.handle, ctypes.byref(out)))
        self._shapes[out.value] = _shape(M.handle)
        return out.value

    def submit(self, matrix: int, op: int, X: torch.Tensor, Y: torch.Tensor, tag: int = 0) -> int:
        """X, Y: device tensors, 1-D (k = 1) or 2-D row-major (rows x k)."""
        if matrix not in self._shapes:
            raise ValueError("matrix handle %r is not registered with this server" % (matrix,))
        if op not in (SPW_OP_MV, SPW_OP_VTM):
            raise ValueError("op must be SPW_OP_MV or SPW_OP_VTM")
        m, n, dev = self._shapes[matrix]
        in_len, out_len = (n, m) if op == SPW_OP_MV else (m, n)
        k = check_operands(X, Y, in_len, out_len, dev, True)
        r = Request()
        r.struct_size = ctypes.sizeof(Request)
        r.matrix, r.op, r.vdt, r.k = matrix, op, _vec_dtype(X), k
        r.in_, r.ldi = X.data_ptr(), _ld(X)
        r.out, r.ldo = Y.data_ptr(), _ld(Y)
        r.tag = tag
        t = ctypes.c_uint64()
        _check(load().spw_serve_submit(self.handle, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = (X, Y)
        return t.value

    def resume(self):
        _check(load().spw_serve_resume(self.handle))

    def poll(self, ticket: int) -> bool:
        d = _I32()
        _check(load().spw_serve_poll(self.handle, ticket, ctypes.byref(d)))
        if d.value:
            self._keep.pop(ticket, None)
        return bool(d.value)

    def wait(self, ticket: int, timeout_us: int = -1):
        _check(load().spw_serve_wait(self.handle, ticket, timeout_us))
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        st = ServerStats()
        st.struct_size = ctypes.sizeof(ServerStats)
        _check(load().spw_serve_stats(self.handle, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in ServerStats._fields_ if n != "struct_size"}

    def close(self):
        if self.handle:
            _check(load().spw_serve_destroy(self.handle))
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
