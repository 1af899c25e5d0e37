"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every declared symbol, argument and matrix validation reports errors before
touching a device, and the host chunk/zone plan matches the oracle's zones."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spw.h")


@pytest.fixture(scope="module")
def spw():
    from paper_1812_00904_amd import spw as mod
    mod.load()
    return mod


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spw_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(spw):
    lib = ctypes.CDLL(spw.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    # and the binding knows the signature of each one
    assert set(names) <= set(spw.SIGNATURES), set(names) - set(spw.SIGNATURES)


def test_only_declared_c_symbols_are_exported(spw):
    """Internal helpers keep internal linkage: every exported function with
    an unmangled (C) name is one that include/spw.h declares."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm is not installed")
    out = subprocess.run([nm, "-D", "--defined-only", spw.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set()
    for line in out.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[1] in ("T", "W"):
            name = parts[2]
            if not name.startswith(("_Z", "__hip", "_init", "_fini")):
                exported.add(name)
    assert exported, "no exported C functions found"
    assert exported <= set(declared_symbols()), sorted(exported - set(declared_symbols()))


def test_status_strings(spw):
    lib = spw.load()
    for i, name in enumerate(spw.STATUS_NAMES):
        assert lib.spw_status_string(i).decode() == name
    assert lib.spw_status_string(99).decode() == "SPW_UNKNOWN_STATUS"


def _expect(spw, status_name, fn, *args):
    with pytest.raises(spw.SpwError) as ei:
        fn(*args)
    assert ei.value.status_name == status_name, str(ei.value)
    return str(ei.value)


def test_create_rejects_bad_matrices_before_device_use(spw):
    ptr = np.array([0, 2, 3], dtype=np.int64)
    idx = np.array([0, 1, 1], dtype=np.int32)
    val = np.ones(3)
    # ptr must start at 0
    _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create, spw.SPW_CSC, 2, 2, np.array([1, 2, 3]), idx, val)
    # decreasing pointer
    _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create, spw.SPW_CSC, 2, 3,
            np.array([0, 2, 1, 3]), idx, val)
    # index out of range, named by position
    msg = _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create, spw.SPW_CSC, 2, 2, ptr,
                  np.array([0, 1, 2], dtype=np.int32), val)
    assert "position 2" in msg
    # not strictly increasing inside a column (duplicate)
    msg = _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create, spw.SPW_CSC, 2, 2, ptr,
                  np.array([1, 1, 0], dtype=np.int32), val)
    assert "position 1" in msg
    # CSR: ptr over rows, indices are columns
    _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create, spw.SPW_CSR, 2, 1, ptr, idx, val)


def test_create_rejects_bad_arguments(spw):
    lib = spw.load()
    h = ctypes.c_void_p()
    ptr = np.zeros(3, dtype=np.int64)
    assert lib.spw_create(None, 0, 2, 2, 0, ptr.ctypes.data, None, None, None) == 1
    assert lib.spw_create(ctypes.byref(h), 7, 2, 2, 0, ptr.ctypes.data, None, None, None) == 1
    assert lib.spw_create(ctypes.byref(h), 0, -1, 2, 0, ptr.ctypes.data, None, None, None) == 1
    assert lib.spw_create(ctypes.byref(h), 0, 2, 2, 0, None, None, None, None) == 1
    assert lib.spw_create(ctypes.byref(h), 0, 2, 2, 3, ptr.ctypes.data, None, None, None) == 1
    bad = spw.create_opts()
    bad.struct_size = 3
    assert lib.spw_create(ctypes.byref(h), 0, 2, 2, 0, ptr.ctypes.data, None, None, ctypes.byref(bad)) == 1
    assert "struct_size" in lib.spw_last_error().decode()
    assert lib.spw_mv(None, 0, None, None, None) == 1
    assert lib.spw_destroy(None) == 0


def _check_plan_against_oracle(spw, A, C):
    owned, zc, zf, zl = spw.spw_plan_zones(A.n, A.ptr, C)
    off = oracle.offsets_fixed(A.nnz, C)
    ozc, osf, osl = oracle.zones(A.n, A.ptr, off)
    assert np.array_equal(zc, ozc)
    assert np.array_equal(zf, osf)
    assert np.array_equal(zl, osl)
    # owned: first column whose start lies at or after the chunk start; last = n
    G = off.size - 1
    assert owned.size == G + 1 and owned[G] == A.n
    for c in range(G):
        first_at_or_after = int(np.searchsorted(A.ptr, off[c], side="left"))
        assert owned[c] == first_at_or_after
    # the zone chunk sets agree with the paper's setup scans over the same split
    if G >= 1 and A.nnz:
        jf, jl = oracle.cover(A.n, A.ptr, off)
        sv = oracle.setup_vars(jf, jl)
        assert zc.size == int(sv["leftGroupEnd"].sum())
        for g in range(G):
            if sv["needRight"][g]:
                k = int(sv["rightGroup"][g])
                assert zf[k] <= g and zl[k] == g + sv["procsOnRight"][g]
            if sv["needLeft"][g]:
                k = int(sv["leftGroup"][g])
                assert zf[k] == g - sv["procsOnLeft"][g]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("C", [1, 3, 16, 512])
def test_plan_zones_match_oracle(spw, seed, C):
    A = synth.random_csc(50, 700, 4.0, seed, empty_frac=0.3)
    A = synth.from_lengths(50, np.r_[np.diff(A.ptr)[:300], [50, 0, 0, 50, 1], np.diff(A.ptr)[300:]], seed)
    _check_plan_against_oracle(spw, A, C)


def test_plan_zones_worked_example(spw):
    import json
    ex = json.load(open(os.path.join(ROOT, "tests", "golden", "worked_example.json")))
    lengths = [len(c) for c in ex["fig1_rows_per_column"]]
    ptr = np.r_[0, np.cumsum(lengths)].astype(np.int64)
    owned, zc, zf, zl = spw.spw_plan_zones(8, ptr, ex["group_size"])
    assert [int(c) + 1 for c in zc] == [z["column"] for z in ex["table1_zones"]]
    assert [list(range(a, b + 1)) for a, b in zip(zf, zl)] == [z["S"] for z in ex["table1_zones"]]


def test_plan_zones_edge_cases(spw):
    # empty matrix: no chunks, no zones
    owned, zc, _, _ = spw.spw_plan_zones(5, np.zeros(6, dtype=np.int64), 4)
    assert owned.tolist() == [5] and zc.size == 0
    # one long column across many chunks: one zone spanning all of them
    owned, zc, zf, zl = spw.spw_plan_zones(1, np.array([0, 100], dtype=np.int64), 7)
    assert zc.tolist() == [0] and zf.tolist() == [0] and zl.tolist() == [14]
    # boundaries that fall exactly on column starts cut nothing
    owned, zc, _, _ = spw.spw_plan_zones(4, np.array([0, 4, 8, 12, 16], dtype=np.int64), 4)
    assert zc.size == 0 and owned.tolist() == [0, 1, 2, 3, 4]


# ---------------------------------------------------------------------------
# Create-time value rounding (host code of the library) against the oracle's
# rounding, which is pinned to the hardware binary32 conversion and to the
# bfloat16 definition in test_oracle_pins.
# ---------------------------------------------------------------------------
def _rounding_inputs():
    rng = np.random.default_rng(11)
    x = rng.standard_normal(50000) * np.exp2(rng.integers(-150, 127, 50000))
    # ties and near-ties of both formats, subnormal range, signed zeros
    t = [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -24, 1.0 + 3 * 2.0 ** -24,
         1.0 + 2.0 ** -8 + 2.0 ** -40, 2.0 ** -134, 3 * 2.0 ** -134, 2.0 ** -149, 2.0 ** -150,
         3 * 2.0 ** -150, 2.0 ** -126 * (1 - 2.0 ** -9), 0.0, -0.0, 1e-300, -1e-310]
    return np.concatenate([x, t, [-v for v in t]])


@pytest.mark.parametrize("fmt,storage", [("f32", 1), ("bf16", 2)])
def test_library_rounding_matches_oracle(spw, fmt, storage):
    x = _rounding_inputs()
    ours = spw.spw_round_values(storage, x)
    ref = oracle.round_array(x, fmt)
    assert np.array_equal(ours.view(np.uint64), ref.view(np.uint64))


def test_library_rounding_f64_is_identity(spw):
    x = _rounding_inputs()
    assert np.array_equal(spw.spw_round_values(0, x).view(np.uint64), x.view(np.uint64))


def test_library_rounding_reports_overflow(spw):
    # largest finite bfloat16 is (2 - 2^-7) * 2^127; halfway to 2^128 rounds to even = overflow
    big = (2 - 2.0 ** -7) * 2.0 ** 127
    assert spw.spw_round_values(2, np.array([big]))[0] == big
    msg = _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_round_values, 2, np.array([1.0, (2 - 2.0 ** -8) * 2.0 ** 127]))
    assert "position 1" in msg
    _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_round_values, 1, np.array([0.0, 0.0, 1e39]))
    # a bad storage type is an argument error
    _expect(spw, "SPW_ERR_INVALID_ARG", spw.spw_round_values, 7, np.array([1.0]))


def test_create_rejects_value_overflow_before_device_use(spw):
    ptr = np.array([0, 1, 3], dtype=np.int64)
    idx = np.array([0, 0, 1], dtype=np.int32)
    val = np.array([1.0, 3.4e38, 1e39])   # 3.4e38 fits binary32, not bfloat16
    msg = _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create, spw.SPW_CSC, 2, 2, ptr, idx, val,
                  spw.create_opts(value_storage=spw.SPW_F32))
    assert "position 2" in msg
    msg = _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create, spw.SPW_CSC, 2, 2, ptr, idx, val,
                  spw.create_opts(value_storage=spw.SPW_BF16))
    assert "position 1" in msg
    _expect(spw, "SPW_ERR_INVALID_ARG", spw.spw_create, spw.SPW_CSC, 2, 2, ptr, idx, val,
            spw.create_opts(value_storage=5))


def test_create_coo_rejects_bad_triples_before_device_use(spw):
    rows = np.array([0, 1, 1], dtype=np.int32)
    cols = np.array([1, 0, 2], dtype=np.int32)
    val = np.ones(3)
    # a column index outside the matrix, named by its triple
    msg = _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create_coo, spw.SPW_CSC, 2, 2, rows, cols, val)
    assert "triple 2" in msg
    _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create_coo, spw.SPW_CSR, 1, 3, rows, cols, val)
    # a (row, column) pair given twice, in either layout
    dup_r = np.array([1, 0, 1], dtype=np.int32)
    dup_c = np.array([2, 1, 2], dtype=np.int32)
    for fmt in (spw.SPW_CSC, spw.SPW_CSR):
        msg = _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create_coo, fmt, 2, 3, dup_r, dup_c, val)
        assert "(1, 2)" in msg
    _expect(spw, "SPW_ERR_INVALID_ARG", spw.spw_create_coo, 7, 2, 3, rows, cols, val)
    lib = spw.load()
    h = ctypes.c_void_p()
    assert lib.spw_create_coo(ctypes.byref(h), 0, 2, 3, 3, None, None, None, None) == 1   # NULL triples
    assert lib.spw_create_coo(None, 0, 2, 3, 0, None, None, None, None) == 1               # NULL out


def test_news20_shaped_statistics():
    # the published shape of the paper's data set (Section VI): 19,996 x
    # 1,355,191, 9,097,916 nonzeros, 25 columns with at least 9,998 nonzeros,
    # the 10 densest between 11,872 and 18,531
    A = synth.news20_shaped()
    assert (A.m, A.n, A.nnz) == (19996, 1355191, 9097916)
    L = np.diff(A.ptr)
    top = np.sort(L)[::-1]
    assert int((L >= 9998).sum()) == 25
    assert top[0] == 18531 and top[9] == 11872 and top[10] < 11872
    assert 6.5 < L.mean() < 7.0
    assert np.all(np.diff(A.idx[A.ptr[0]:A.ptr[1]]) > 0)
    B = synth.news20_shaped()
    assert np.array_equal(A.ptr, B.ptr) and np.array_equal(A.idx, B.idx) and np.array_equal(A.val, B.val)


def test_canonicalize_still_rejects_out_of_range_before_device_use(spw):
    ptr = np.array([0, 3, 4], dtype=np.int64)
    val = np.ones(4)
    opts = spw.create_opts(canonicalize=1)
    # unsorted and repeated rows are fine with canonicalize; a row past the end is not
    msg = _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create, spw.SPW_CSC, 3, 2, ptr,
                  np.array([2, 0, 3, 1], dtype=np.int32), val, opts)
    assert "position 2" in msg
    _expect(spw, "SPW_ERR_BAD_MATRIX", spw.spw_create, spw.SPW_CSC, 3, 2, np.array([0, 3, 5]),
            np.array([2, 0, 2, 1], dtype=np.int32), val, opts)
    assert ctypes.sizeof(spw.CreateOpts) == 60


_OOM_CHILD = r'''
import resource, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_1812_00904_amd import spw
spw.load()
n, m = 200_000, 1000
ptr = np.arange(0, 150 * (n + 1), 150, dtype=np.int64)
nnz = int(ptr[-1])
idx = (np.arange(nnz) % m).astype(np.int32)
val = np.ones(nnz)
with open("/proc/self/status") as f:
    vm = next(int(l.split()[1]) * 1024 for l in f if l.startswith("VmSize"))
lim = vm + 150 * 2**20          # far less than the canonical copy of 3e7 entries needs
resource.setrlimit(resource.RLIMIT_AS, (lim, lim))
try:
    spw.SpwMatrix(spw.SPW_CSC, m, n, ptr, idx, val, canonicalize=1)
    print("created")
except spw.SpwError as e:
    print(e.status_name)
'''


def test_host_allocation_failure_is_a_status_not_an_abort():
    # A C++ exception must not cross the C ABI: with the address space capped,
    # the host copy made by canonicalize fails and the call returns
    # SPW_ERR_OUT_OF_MEMORY (before any device use) instead of terminating.
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _OOM_CHILD, root], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "SPW_ERR_OUT_OF_MEMORY", r.stdout


# ---------------------------------------------------------------------------
# The binding's operand checks run before any pointer reaches the library, so
# they are exercised here with host tensors (device check off).
# ---------------------------------------------------------------------------
def test_binding_rejects_mismatched_operands(spw):
    import torch
    chk = spw.check_operands
    f64, f32 = torch.float64, torch.float32
    x, y = torch.zeros(7, dtype=f64), torch.zeros(5, dtype=f64)
    assert chk(x, y, 7, 5, None, False) == 1
    bad_single = [
        (torch.zeros(7, dtype=f64), torch.zeros(5, dtype=f32)),        # output narrower than input
        (torch.zeros(7, dtype=f32), torch.zeros(5, dtype=f64)),        # output wider than input
        (torch.zeros(6, dtype=f64), torch.zeros(5, dtype=f64)),        # short input
        (torch.zeros(7, dtype=f64), torch.zeros(4, dtype=f64)),        # short output
        (torch.zeros(14, dtype=f64)[::2], torch.zeros(5, dtype=f64)),  # strided view
        (torch.zeros(7, 1, dtype=f64), torch.zeros(5, dtype=f64)),     # 2-D in a single-vector call
    ]
    for a, b in bad_single:
        with pytest.raises(ValueError):
            chk(a, b, 7, 5, None, False)
    with pytest.raises(TypeError):
        chk(torch.zeros(7, dtype=torch.int64), torch.zeros(5, dtype=torch.int64), 7, 5, None, False)
    # multi-RHS blocks: (rows x k), unit column stride, row stride >= k
    X, Y = torch.zeros(7, 3, dtype=f64), torch.zeros(5, 3, dtype=f64)
    assert chk(X, Y, 7, 5, None, True) == 3
    wide = torch.zeros(7, 8, dtype=f64)
    assert chk(wide[:, :3], Y, 7, 5, None, True) == 3                 # padded leading dimension
    assert chk(x, y, 7, 5, None, True) == 1                           # 1-D pair: k = 1
    bad_batch = [
        (X, torch.zeros(5, 3, dtype=f32)),                             # types differ
        (X, torch.zeros(5, 2, dtype=f64)),                             # k differs
        (X, torch.zeros(4, 3, dtype=f64)),                             # short output
        (torch.zeros(6, 3, dtype=f64), Y),                             # short input
        (torch.zeros(3, 7, dtype=f64).t(), Y),                         # column-major view
        (wide[:, ::2][:, :3], Y),                                      # column stride 2
        (x, Y),                                                        # 1-D against 2-D
    ]
    for a, b in bad_batch:
        with pytest.raises(ValueError):
            chk(a, b, 7, 5, None, True)
