"""CPU oracle for the wide/tall sparse product path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, single-threaded fp64 reference written from Eckstein &
Matyasfalvi, arXiv:1812.00904.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package; the GPU
library never does, and the two share no code (they meet only on the seeded
inputs of the ``synth`` package).

The arithmetic lives in ``oracle.c`` (compiled with ``gcc -O2
-ffp-contract=off``); this module only marshals numpy arrays.  See the header
of ``oracle.c`` for which section of the paper each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_F64P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (plain gcc, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    override = os.environ.get("SPW_ORACLE_LIB")  # a mutated build, used by the mutation tests
    if override:
        lib = ctypes.CDLL(override)
    else:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
    op = [_i64, _i64, _I64P, _I32P, _F64P, _F64P, _F64P, ctypes.c_void_p]
    for name in ("orc_mv_csc", "orc_vtm_csc", "orc_mv_csr", "orc_vtm_csr"):
        f = getattr(lib, name)
        f.argtypes = op
        f.restype = None
    bop = [_i64, _i64, _I64P, _I32P, _F64P, _i64, _F64P, _i64, _F64P, _i64, ctypes.c_void_p, _i64]
    for name in ("orc_mv_csc_batch", "orc_vtm_csc_batch", "orc_mv_csr_batch", "orc_vtm_csr_batch"):
        f = getattr(lib, name)
        f.argtypes = bop
        f.restype = ctypes.c_int
    lib.orc_round_bits.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.orc_round_bits.restype = ctypes.c_double
    lib.orc_round_array.argtypes = [_F64P, _F64P, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.orc_round_array.restype = None
    lib.orc_offsets_paper.argtypes = [_i64, _i64, _I64P]
    lib.orc_offsets_paper.restype = None
    lib.orc_offsets_fixed.argtypes = [_i64, _i64, _I64P]
    lib.orc_offsets_fixed.restype = _i64
    lib.orc_cover.argtypes = [_i64, _I64P, _i64, _I64P, _I64P, _I64P]
    lib.orc_cover.restype = ctypes.c_int
    lib.orc_zones.argtypes = [_i64, _I64P, _i64, _I64P, _I64P, _I64P, _I64P]
    lib.orc_zones.restype = _i64
    lib.orc_setup_vars.argtypes = [_i64, _I64P, _I64P] + [_I64P] * 7
    lib.orc_setup_vars.restype = None
    nzp = [_i64, _i64, _I64P, _I32P, _F64P, _i64, _I64P, _F64P, _F64P]
    lib.orc_nzp_mv.argtypes = nzp
    lib.orc_nzp_mv.restype = ctypes.c_int
    lib.orc_nzp_vtm.argtypes = nzp
    lib.orc_nzp_vtm.restype = ctypes.c_int
    lib.orc_colp_imbalance.argtypes = [_i64, _I64P, _i64]
    lib.orc_colp_imbalance.restype = ctypes.c_double
    lib.orc_cgls.argtypes = [ctypes.c_int, _i64, _i64, _I64P, _I32P, _F64P, _F64P, _F64P, _i64, _F64P, _F64P]
    lib.orc_cgls.restype = ctypes.c_int
    _lib = lib
    return lib


def _arrs(ptr, idx, val):
    return (np.ascontiguousarray(ptr, dtype=np.int64), np.ascontiguousarray(idx, dtype=np.int32),
            np.ascontiguousarray(val, dtype=np.float64))


def _dptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Products (Section I; tall storage by swapping roles, Section II)
# --------------------------------------------------------------------------
def _single(name, out_len, m, n, ptr, idx, val, vec, with_d):
    lib = _load()
    ptr, idx, val = _arrs(ptr, idx, val)
    vec = np.ascontiguousarray(vec, dtype=np.float64)
    out = np.empty(out_len, dtype=np.float64)
    d = np.empty(out_len, dtype=np.float64) if with_d else None
    getattr(lib, name)(m, n, ptr, idx, val, vec, out, _dptr(d) if with_d else None)
    return (out, d) if with_d else out


def mv_csc(m, n, ptr, idx, val, x, with_d=False):
    """y = A x for wide CSC A (Section I).  Optionally also d_i = sum_j |a_ij||x_j|."""
    return _single("orc_mv_csc", m, m, n, ptr, idx, val, x, with_d)


def vtm_csc(m, n, ptr, idx, val, v, with_d=False):
    """u^T = v^T A for wide CSC A (Section I).  Optionally also d_j = sum_i |v_i||a_ij|."""
    return _single("orc_vtm_csc", n, m, n, ptr, idx, val, v, with_d)


def mv_csr(m, n, ptr, idx, val, x, with_d=False):
    """y = A x for tall CSR A."""
    return _single("orc_mv_csr", m, m, n, ptr, idx, val, x, with_d)


def vtm_csr(m, n, ptr, idx, val, v, with_d=False):
    """u^T = v^T A for tall CSR A."""
    return _single("orc_vtm_csr", n, m, n, ptr, idx, val, v, with_d)


def _batch(name, in_len, out_len, m, n, ptr, idx, val, X, with_d):
    lib = _load()
    ptr, idx, val = _arrs(ptr, idx, val)
    X = np.ascontiguousarray(X, dtype=np.float64)
    assert X.ndim == 2 and X.shape[0] == in_len
    k = X.shape[1]
    Y = np.empty((out_len, k), dtype=np.float64)
    D = np.empty((out_len, k), dtype=np.float64) if with_d else None
    rc = getattr(lib, name)(m, n, ptr, idx, val, k, X, max(k, 1), Y, max(k, 1),
                            _dptr(D) if with_d else None, max(k, 1))
    if rc != 0:
        raise MemoryError(name)
    return (Y, D) if with_d else Y


def mv_csc_batch(m, n, ptr, idx, val, X, with_d=False):
    """Y = A X for wide CSC A, X of shape (n, k) row-major."""
    return _batch("orc_mv_csc_batch", n, m, m, n, ptr, idx, val, X, with_d)


def vtm_csc_batch(m, n, ptr, idx, val, V, with_d=False):
    """U = A^T V for wide CSC A, V of shape (m, k) row-major."""
    return _batch("orc_vtm_csc_batch", m, n, m, n, ptr, idx, val, V, with_d)


def mv_csr_batch(m, n, ptr, idx, val, X, with_d=False):
    return _batch("orc_mv_csr_batch", n, m, m, n, ptr, idx, val, X, with_d)


def vtm_csr_batch(m, n, ptr, idx, val, V, with_d=False):
    return _batch("orc_vtm_csr_batch", m, n, m, n, ptr, idx, val, V, with_d)


# --------------------------------------------------------------------------
# Value-storage rounding (binary32 / bfloat16, one RNE step from binary64)
# --------------------------------------------------------------------------
FORMATS = {"f32": (24, -126, 127), "bf16": (8, -126, 127)}


def round_value(x: float, fmt: str) -> float:
    p, emin, emax = FORMATS[fmt]
    return _load().orc_round_bits(float(x), p, emin, emax)


def round_array(a, fmt: str) -> np.ndarray:
    p, emin, emax = FORMATS[fmt]
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.empty_like(a)
    _load().orc_round_array(a.reshape(-1), out.reshape(-1), a.size, p, emin, emax)
    return out


# --------------------------------------------------------------------------
# Partition, cover, zones and setup variables (Sections II and IV)
# --------------------------------------------------------------------------
def offsets_paper(Z: int, P: int) -> np.ndarray:
    off = np.empty(P + 1, dtype=np.int64)
    _load().orc_offsets_paper(Z, P, off)
    return off


def offsets_fixed(Z: int, C: int) -> np.ndarray:
    G = (Z + C - 1) // C
    off = np.empty(G + 1, dtype=np.int64)
    _load().orc_offsets_fixed(Z, C, off)
    return off


def cover(n, ptr, off):
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    off = np.ascontiguousarray(off, dtype=np.int64)
    P = off.size - 1
    jf = np.empty(P, dtype=np.int64)
    jl = np.empty(P, dtype=np.int64)
    rc = _load().orc_cover(n, ptr, P, off, jf, jl)
    if rc != 0:
        raise ValueError("orc_cover failed (%d): every group must hold a nonzero" % rc)
    return jf, jl


def zones(n, ptr, off):
    """Overlap zones from their definition: (zone columns, first group, last group)."""
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    off = np.ascontiguousarray(off, dtype=np.int64)
    P = off.size - 1
    zc = np.empty(max(P, 1), dtype=np.int64)
    sf = np.empty(max(P, 1), dtype=np.int64)
    sl = np.empty(max(P, 1), dtype=np.int64)
    z = _load().orc_zones(n, ptr, P, off, zc, sf, sl)
    if z < 0:
        raise MemoryError("orc_zones")
    return zc[:z].copy(), sf[:z].copy(), sl[:z].copy()


SETUP_NAMES = ("needLeft", "needRight", "leftGroupEnd", "rightGroup", "leftGroup",
               "procsOnLeft", "procsOnRight")


def setup_vars(jf, jl) -> dict:
    jf = np.ascontiguousarray(jf, dtype=np.int64)
    jl = np.ascontiguousarray(jl, dtype=np.int64)
    P = jf.size
    outs = [np.empty(P, dtype=np.int64) for _ in SETUP_NAMES]
    _load().orc_setup_vars(P, jf, jl, *outs)
    return dict(zip(SETUP_NAMES, outs))


def nzp_mv(m, n, ptr, idx, val, off, x):
    lib = _load()
    ptr, idx, val = _arrs(ptr, idx, val)
    off = np.ascontiguousarray(off, dtype=np.int64)
    y = np.empty(m, dtype=np.float64)
    if lib.orc_nzp_mv(m, n, ptr, idx, val, off.size - 1, off,
                      np.ascontiguousarray(x, dtype=np.float64), y) != 0:
        raise MemoryError("orc_nzp_mv")
    return y


def nzp_vtm(m, n, ptr, idx, val, off, v):
    lib = _load()
    ptr, idx, val = _arrs(ptr, idx, val)
    off = np.ascontiguousarray(off, dtype=np.int64)
    u = np.empty(n, dtype=np.float64)
    if lib.orc_nzp_vtm(m, n, ptr, idx, val, off.size - 1, off,
                       np.ascontiguousarray(v, dtype=np.float64), u) != 0:
        raise MemoryError("orc_nzp_vtm")
    return u


def colp_imbalance(n, ptr, P) -> float:
    return _load().orc_colp_imbalance(n, np.ascontiguousarray(ptr, dtype=np.int64), P)


def cgls(fmt, m, n, ptr, idx, val, b, x0, iters):
    """CGLS on min ||b - A x||_2 from x0 (Section VII's first-order use of the
    products; the variant is Hestenes-Stiefel / Bjorck, see oracle.c).  A is m x n,
    fmt "csc" (wide) or "csr" (tall).  Returns (x, gamma, rho) with gamma[k] =
    ||A^T r_k||^2 and rho[k] = ||r_k||^2 for k = 0 .. iters."""
    lib = _load()
    ptr, idx, val = _arrs(ptr, idx, val)
    x = np.array(x0, dtype=np.float64, copy=True)
    gamma = np.empty(iters + 1, dtype=np.float64)
    rho = np.empty(iters + 1, dtype=np.float64)
    if lib.orc_cgls(1 if fmt == "csr" else 0, m, n, ptr, idx, val,
                    np.ascontiguousarray(b, dtype=np.float64), x, iters, gamma, rho) != 0:
        raise MemoryError("orc_cgls")
    return x, gamma, rho
