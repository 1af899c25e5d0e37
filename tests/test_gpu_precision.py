"""GPU parity of reduced-precision value storage (binary32 and bfloat16
values, rounded once at create) with binary32 or binary64 vectors.

Two references, both from the CPU oracle in binary64:
  (ii) the oracle on the stored values (oracle.round_array, pinned separately
       against the hardware conversion and the bfloat16 definition) with the
       same vector entries: |gpu - ref| <= tol * d, d = sum |a_stored| |x|,
       tol = 1e-5 for binary32 vectors and 1e-13 for binary64 vectors;
  (i)  the oracle on the original binary64 values: the difference is bounded
       by the storage rounding, u_s * sum |a| |x| (u_s = 2^-24 binary32,
       2^-8 bfloat16), plus (ii)'s tolerance.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

STORAGE = {"f32": (1, 2.0 ** -24), "bf16": (2, 2.0 ** -8)}


@pytest.fixture(scope="module")
def spw():
    from paper_1812_00904_amd import spw as mod
    mod.load()
    assert torch.cuda.is_available()
    return mod


def within(got, ref, d, tol, what):
    err = np.abs(got - ref)
    bad = err > tol * d
    if bad.any():
        i = np.argwhere(bad)[0]
        raise AssertionError("%s: %d entries off; first %s: got %r want %r d=%r"
                             % (what, int(bad.sum()), tuple(i), got[tuple(i)], ref[tuple(i)], d[tuple(i)]))


def oracle_products(A, fmt, val, X, V):
    """(Y, DY, U, DU) for block inputs X (long side) and V (short side)."""
    if fmt == 0:
        Y, DY = oracle.mv_csc_batch(A.m, A.n, A.ptr, A.idx, val, X, with_d=True)
        U, DU = oracle.vtm_csc_batch(A.m, A.n, A.ptr, A.idx, val, V, with_d=True)
    else:
        Y, DY = oracle.mv_csr_batch(A.n, A.m, A.ptr, A.idx, val, X, with_d=True)
        U, DU = oracle.vtm_csr_batch(A.n, A.m, A.ptr, A.idx, val, V, with_d=True)
    return Y, DY, U, DU


def run(spw, A, fmt, storage, vdt, k, seed, name):
    code, us = STORAGE[storage]
    m, n = (A.m, A.n) if fmt == 0 else (A.n, A.m)
    print("precision case %s fmt=%d storage=%s vdt=%s k=%d m=%d n=%d nnz=%d"
          % (name, fmt, storage, vdt, k, m, n, A.nnz), flush=True)
    M = spw.SpwMatrix(fmt, m, n, A.ptr, A.idx, A.val, value_storage=code)
    assert M.info()["value_storage"] == code
    X = synth.vector(n * k, seed, 1).reshape(n, k)
    V = synth.vector(m * k, seed, 2).reshape(m, k)
    if vdt == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
        V = V.astype(np.float32).astype(np.float64)
    Xd = torch.from_numpy(X).to(vdt).cuda()
    Vd = torch.from_numpy(V).to(vdt).cuda()
    outs = []
    for _ in range(2):
        if k == 1:
            y = M.mv(Xd[:, 0].contiguous())[:, None]
            u = M.vtm(Vd[:, 0].contiguous())[:, None]
        else:
            y = M.mv_batch(Xd)
            u = M.vtm_batch(Vd)
        torch.cuda.synchronize()
        outs.append((y.double().cpu().numpy(), u.double().cpu().numpy()))
    M.close()
    (Y, U), (Y2, U2) = outs
    assert np.array_equal(Y, Y2) and np.array_equal(U, U2), "not bit-identical from run to run"
    tol = 1e-5 if vdt == torch.float32 else 1e-13
    stored = oracle.round_array(A.val, storage)
    Yr, DY, Ur, DU = oracle_products(A, fmt, stored, X, V)
    within(Y, Yr, DY, tol, "%s mv vs stored values" % name)
    within(U, Ur, DU, tol, "%s vtm vs stored values" % name)
    Yo, DYo, Uo, DUo = oracle_products(A, fmt, A.val, X, V)
    within(Y, Yo, DYo, us + tol * (1 + us), "%s mv vs original values" % name)
    within(U, Uo, DUo, us + tol * (1 + us), "%s vtm vs original values" % name)


@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("vdt", [torch.float32, torch.float64])
@pytest.mark.parametrize("k", [1, 3, 16])
def test_storage_small_config(spw, fmt, storage, vdt, k):
    A = synth.config_matrix("c0", scale=0.2)
    run(spw, A, fmt, storage, vdt, k, seed=40 + k, name="c0x0.2")


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("case", ["wide_index", "many_empty", "lognormal"])
def test_storage_structures(spw, storage, case):
    if case == "wide_index":
        A = synth.random_csc(70000, 3000, 12.0, 10, values="lognormal", row_alpha=0.8)
    elif case == "many_empty":
        A = synth.random_csc(300, 20000, 3.0, 4, empty_frac=0.8)
    else:
        A = synth.random_csc(5000, 40000, 9.0, 12, values="lognormal", row_alpha=0.8)
    for fmt in (0, 1):
        run(spw, A, fmt, storage, torch.float32, 1, seed=5, name=case)
        run(spw, A, fmt, storage, torch.float32, 8, seed=6, name=case)


def test_storage_bytes_shrink(spw):
    A = synth.config_matrix("c0", scale=0.2)
    sizes = {}
    for code in (0, 1, 2):
        M = spw.SpwMatrix(0, A.m, A.n, A.ptr, A.idx, A.val, value_storage=code, transpose=0)
        sizes[code] = M.info()["device_bytes"]
        M.close()
    assert sizes[0] > sizes[1] > sizes[2]


def test_integer_values_exact_in_every_storage(spw):
    # small integers are exact in bfloat16 and every partial sum is an integer
    # below 2^24, so each storage / vector type gives the exact result
    rng = np.random.default_rng(3)
    A = synth.random_csc(400, 30000, 6.0, 21)
    A.val[:] = rng.integers(-8, 9, A.nnz)
    x = rng.integers(-8, 9, A.n).astype(np.float64)
    v = rng.integers(-8, 9, A.m).astype(np.float64)
    y_ref = oracle.mv_csc(A.m, A.n, A.ptr, A.idx, A.val, x)
    u_ref = oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, v)
    for code in (0, 1, 2):
        M = spw.SpwMatrix(0, A.m, A.n, A.ptr, A.idx, A.val, value_storage=code)
        for dt in (torch.float32, torch.float64):
            y = M.mv(torch.from_numpy(x).to(dt).cuda()).double().cpu().numpy()
            u = M.vtm(torch.from_numpy(v).to(dt).cuda()).double().cpu().numpy()
            assert np.array_equal(y, y_ref) and np.array_equal(u, u_ref), (code, dt)
        M.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_storage_full_size(spw, storage):
    # the 2e8-nonzero matrix with binary32 / bfloat16 values and binary32
    # vectors, single vectors, as the benchmark runs it
    A = synth.config_matrix("c1")
    run(spw, A, 0, storage, torch.float32, 1, seed=60, name="c1 full")
