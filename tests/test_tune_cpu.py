"""The autotuner's host side (no GPU): matrix fingerprints and the on-disk
tuning cache round trip through the C ABI."""
import ctypes
import os

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def spw():
    from paper_1812_00904_amd import spw as mod
    mod.load()
    return mod


def _fp(spw, fmt, storage, A):
    out = ctypes.c_uint64()
    ptr = np.ascontiguousarray(A.ptr, dtype=np.int64)
    idx = np.ascontiguousarray(A.idx, dtype=np.int32)
    m, n = (A.m, A.n) if fmt == spw.SPW_CSC else (A.n, A.m)
    spw._check(spw.load().spw_matrix_fingerprint(fmt, storage, m, n, int(idx.size), ptr.ctypes.data,
                                                 idx.ctypes.data, ctypes.byref(out)))
    return out.value


def test_fingerprint_is_deterministic_and_structure_sensitive(spw):
    A = synth.random_csc(300, 5000, 4.0, 1)
    same = synth.random_csc(300, 5000, 4.0, 1)
    other = synth.random_csc(300, 5000, 4.0, 2)       # same shape, other structure
    f = _fp(spw, spw.SPW_CSC, spw.SPW_F64, A)
    assert f == _fp(spw, spw.SPW_CSC, spw.SPW_F64, same)
    assert f != _fp(spw, spw.SPW_CSC, spw.SPW_F64, other)
    assert f != _fp(spw, spw.SPW_CSR, spw.SPW_F64, A)             # the transpose
    assert f != _fp(spw, spw.SPW_CSC, spw.SPW_F32, A)             # another value storage
    # values do not enter the fingerprint: the tuned choices depend on structure only
    B = synth.random_csc(300, 5000, 4.0, 1, values="lognormal")
    assert f == _fp(spw, spw.SPW_CSC, spw.SPW_F64, B)


def test_tuning_cache_round_trip(spw, tmp_path):
    lib = spw.load()
    path = str(tmp_path / "tune.txt")
    spw._check(lib.spw_tune_cache_path(path.encode()))
    spw._check(lib.spw_tune_cache_clear())
    recs = {(0x0123456789ABCDEF, b"vtm.f64.k16"): 3, (0x0123456789ABCDEF, b"chunk"): 512,
            (0xFFFFFFFFFFFFFFFF, b"mv.f32.k4"): 2, (1, b"wg.f64"): -7}
    for (fp, key), v in recs.items():
        spw._check(lib.spw_tune_cache_put(fp, key, v))
    spw._check(lib.spw_tune_cache_put(1, b"wg.f64", 256))           # a later record replaces
    recs[(1, b"wg.f64")] = 256
    # forget everything in memory, then read the file back
    spw._check(lib.spw_tune_cache_clear())
    val, found = ctypes.c_int32(), ctypes.c_int32()
    spw._check(lib.spw_tune_cache_get(1, b"wg.f64", ctypes.byref(val), ctypes.byref(found)))
    assert found.value == 0
    spw._check(lib.spw_tune_cache_path(path.encode()))
    for (fp, key), v in recs.items():
        spw._check(lib.spw_tune_cache_get(fp, key, ctypes.byref(val), ctypes.byref(found)))
        assert found.value == 1 and val.value == v, (fp, key)
    spw._check(lib.spw_tune_cache_get(2, b"wg.f64", ctypes.byref(val), ctypes.byref(found)))
    assert found.value == 0
    text = open(path).read().splitlines()
    assert text[0].startswith("# spw tuning cache") and len(text) == 1 + len(recs)
    # a damaged line is ignored, the rest still loads
    with open(path, "a") as f:
        f.write("not a record\n")
    spw._check(lib.spw_tune_cache_clear())
    spw._check(lib.spw_tune_cache_path(path.encode()))
    spw._check(lib.spw_tune_cache_get(0x0123456789ABCDEF, b"chunk", ctypes.byref(val), ctypes.byref(found)))
    assert found.value == 1 and val.value == 512
    # keys with blanks are refused; memory-only mode writes no file
    with pytest.raises(spw.SpwError):
        spw._check(lib.spw_tune_cache_put(1, b"bad key", 1))
    spw._check(lib.spw_tune_cache_path(None))
    os.remove(path)
    spw._check(lib.spw_tune_cache_put(5, b"k", 1))
    assert not os.path.exists(path)
    spw._check(lib.spw_tune_cache_clear())
