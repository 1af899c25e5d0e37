"""GPU tests of the tunable shapes and the autotuner, through the C ABI.

Every column-dot chunk size (512, 1024) and workgroup size (256, 512, 1024)
meets the oracle's bar (binary64: 1e-13 * sum|a||x|, binary32 vectors: 1e-5 *
sum|a||x| on the stored values); the workgroup size does not change a single
bit (it only changes which wave reduces which chunk).  Every multi-RHS plan
(SINGLE, PASSES, TILE) meets the bar in both directions, and SINGLE / PASSES
columns equal single-vector calls bit for bit.  A matrix created with
autotune records its choices in the tuning cache, and a second creation of the
same matrix takes them from there.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spw():
    from paper_1812_00904_amd import spw as mod
    mod.load()
    assert torch.cuda.is_available()
    return mod


def dev(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()


def check(got, ref, d, tol, what):
    got = np.asarray(got, dtype=np.float64)
    assert got.shape == ref.shape, what
    assert not np.isnan(got).any(), "%s: unwritten components" % what
    bad = np.abs(got - ref) > tol * d
    assert not bad.any(), "%s: %d components off, first %d" % (what, int(bad.sum()), int(np.argmax(bad)))


def coldot_case(spw, fmt, A, vec, dt, **opts):
    """The column-dot direction: v^T A of a CSC matrix or A x of a CSR one."""
    if fmt == spw.SPW_CSC:
        M = spw.SpwMatrix(fmt, A.m, A.n, A.ptr, A.idx, A.val, **opts)
        out = torch.full((A.n,), float("nan"), dtype=dt, device="cuda")
        M.vtm(dev(vec, dt), out)
    else:
        M = spw.SpwMatrix(fmt, A.n, A.m, A.ptr, A.idx, A.val, **opts)
        out = torch.full((A.n,), float("nan"), dtype=dt, device="cuda")
        M.mv(dev(vec, dt), out)
    torch.cuda.synchronize()
    info = M.info()
    M.close()
    return out.double().cpu().numpy(), info


CASES = {
    "ragged": lambda: synth.random_csc(37, 5000, 5.0, 3, values="lognormal"),
    "many_empty": lambda: synth.random_csc(300, 40000, 3.0, 4, empty_frac=0.8),
    "dense_cols": lambda: synth.from_lengths(6000, np.r_[np.full(300, 2), [6000] * 3, np.full(500, 1), [6000],
                                                        np.full(77, 3)], 5, row_alpha=0.8, values="lognormal"),
    "small_wide": lambda: synth.config_matrix("c0", scale=0.2),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("fmt", [0, 1])
def test_chunk_and_workgroup_sizes(spw, case, fmt):
    A = CASES[case]()
    v = synth.vector(A.m, 9, 2)
    v32 = v.astype(np.float32).astype(np.float64)
    # the column dots of the CSC arrays with the short vector, in both formats
    ref, d = oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, v, with_d=True)
    ref32, d32 = oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, v32, with_d=True)
    for chunk in (512, 1024):
        outs64, outs32 = [], []
        for wg in (256, 512, 1024):
            print("tune case %s fmt=%d chunk=%d wg=%d" % (case, fmt, chunk, wg), flush=True)
            u, info = coldot_case(spw, fmt, A, v, torch.float64, chunk_nnz=chunk, wg_size=wg)
            assert info["chunk_nnz"] == chunk
            check(u, ref, d, 1e-13, "%s chunk %d wg %d f64" % (case, chunk, wg))
            outs64.append(u)
            u32, info = coldot_case(spw, fmt, A, v32, torch.float32, chunk_nnz=chunk, wg_size=wg)
            check(u32, ref32, d32, 1e-5, "%s chunk %d wg %d f32" % (case, chunk, wg))
            outs32.append(u32)
        for o in outs64[1:]:
            assert np.array_equal(o, outs64[0]), "workgroup size changed binary64 bits"
        for o in outs32[1:]:
            assert np.array_equal(o, outs32[0]), "workgroup size changed binary32 bits"


def _batch_ref(A, fmt, op, X):
    """Oracle for a k-column call on the matrix made from A's CSC arrays in format fmt."""
    if fmt == 0:
        f = oracle.mv_csc_batch if op == 0 else oracle.vtm_csc_batch
        return f(A.m, A.n, A.ptr, A.idx, A.val, X, with_d=True)
    f = oracle.mv_csr_batch if op == 0 else oracle.vtm_csr_batch
    return f(A.n, A.m, A.ptr, A.idx, A.val, X, with_d=True)


@pytest.mark.parametrize("chunk", [512, 1024])
@pytest.mark.parametrize("fmt", [0, 1])
def test_every_plan_in_both_directions(spw, fmt, chunk):
    A = synth.random_csc(700, 30000, 6.0, 12, values="lognormal", empty_frac=0.2)
    m, n = (A.m, A.n) if fmt == 0 else (A.n, A.m)
    M = spw.SpwMatrix(fmt, m, n, A.ptr, A.idx, A.val, chunk_nnz=chunk, transpose=1)
    for op in (spw.SPW_OP_MV, spw.SPW_OP_VTM):
        in_len, out_len = (n, m) if op == spw.SPW_OP_MV else (m, n)
        for dt, vdt, tol in ((torch.float64, spw.SPW_F64, 1e-13), (torch.float32, spw.SPW_F32, 1e-5)):
            for k in (2, 5, 16):
                X = synth.vector(in_len * k, 40 + k, 3).reshape(in_len, k)
                if dt == torch.float32:
                    X = X.astype(np.float32).astype(np.float64)
                ref, D = _batch_ref(A, fmt, op, X)
                Xd = dev(X, dt)
                singles = []
                for c in range(k):
                    y = M.mv(Xd[:, c].contiguous()) if op == spw.SPW_OP_MV else M.vtm(Xd[:, c].contiguous())
                    singles.append(y)
                for plan in (spw.SPW_PLAN_SINGLE, spw.SPW_PLAN_PASSES, spw.SPW_PLAN_TILE):
                    print("plan case fmt=%d chunk=%d op=%d %s k=%d plan=%d" % (fmt, chunk, op, dt, k, plan), flush=True)
                    M.set_batch_plan(op, vdt, k, plan)
                    assert M.batch_plan(op, vdt, k) == (plan, True)
                    Y = torch.full((out_len, k), float("nan"), dtype=dt, device="cuda")
                    if op == spw.SPW_OP_MV:
                        M.mv_batch(Xd, Y)
                    else:
                        M.vtm_batch(Xd, Y)
                    torch.cuda.synchronize()
                    check(Y.double().cpu().numpy(), ref, D, tol, "fmt %d op %d k %d plan %d" % (fmt, op, k, plan))
                    if plan != spw.SPW_PLAN_TILE:
                        for c in range(k):
                            assert torch.equal(Y[:, c].contiguous(), singles[c]), (plan, c)
                M.set_batch_plan(op, vdt, k, spw.SPW_PLAN_AUTO)
                assert M.batch_plan(op, vdt, k)[1] is False
    M.close()


def test_autotune_records_and_reuses_choices(spw, tmp_path):
    path = str(tmp_path / "tune.txt")
    spw.spw_tune_cache_path(path)
    try:
        A = synth.config_matrix("c0", scale=0.3)
        x, v = synth.config_vectors("c0", A.m, A.n)
        y_ref, dy = oracle.mv_csc(A.m, A.n, A.ptr, A.idx, A.val, x, with_d=True)
        u_ref, du = oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, v, with_d=True)
        M = spw.SpwMatrix(spw.SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val, autotune=1)
        info = M.info()
        assert info["tuned"] == 1 and info["chunk_nnz"] in (512, 1024)
        assert info["wg_size_f64"] in (256, 512) and info["wg_size_f32"] in (256, 512)
        check(M.mv(dev(x)).cpu().numpy(), y_ref, dy, 1e-13, "tuned mv")
        check(M.vtm(dev(v)).cpu().numpy(), u_ref, du, 1e-13, "tuned vtm")
        # first multi-RHS calls time the plans on these buffers, then keep the winner
        for op, in_len in ((spw.SPW_OP_MV, A.n), (spw.SPW_OP_VTM, A.m)):
            for k in (4, 16):
                X = synth.vector(in_len * k, 60 + k, 3).reshape(in_len, k)
                ref, D = _batch_ref(A, 0, op, X)
                Y = M.mv_batch(dev(X)) if op == spw.SPW_OP_MV else M.vtm_batch(dev(X))
                torch.cuda.synchronize()
                check(Y.cpu().numpy(), ref, D, 1e-13, "tuned op %d k %d" % (op, k))
                plan, tuned = M.batch_plan(op, spw.SPW_F64, k)
                assert tuned and plan in (1, 2, 3)
        choices = {(op, k): M.batch_plan(op, spw.SPW_F64, k) for op in (0, 1) for k in (4, 16)}
        M.close()
        lines = open(path).read().splitlines()
        assert any(" coldot.chunk " in l for l in lines) and any(" plan.sc.f64.k16 " in l for l in lines)
        # a new process state: forget memory, reload the file, create again
        spw.load().spw_tune_cache_clear()
        spw.spw_tune_cache_path(path)
        M2 = spw.SpwMatrix(spw.SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val, autotune=1)
        i2 = M2.info()
        assert i2["tuned"] == 1 and i2["fingerprint"] == info["fingerprint"]
        assert (i2["chunk_nnz"], i2["wg_size_f64"], i2["wg_size_f32"]) == \
            (info["chunk_nnz"], info["wg_size_f64"], info["wg_size_f32"])
        for (op, k), c in choices.items():
            assert M2.batch_plan(op, spw.SPW_F64, k) == c
        check(M2.vtm(dev(v)).cpu().numpy(), u_ref, du, 1e-13, "cached vtm")
        M2.close()
    finally:
        spw.spw_tune_cache_path(None)
        spw.load().spw_tune_cache_clear()


def test_bad_tuning_options_are_refused(spw):
    A = synth.random_csc(10, 50, 2.0, 1)
    for opts in ({"chunk_nnz": 768}, {"chunk_nnz": 2048}, {"wg_size": 384}, {"autotune": 2}):
        with pytest.raises(spw.SpwError):
            spw.SpwMatrix(spw.SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val, **opts)
    M = spw.SpwMatrix(spw.SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val, transpose=0)
    with pytest.raises(spw.SpwError) as ei:
        M.set_batch_plan(spw.SPW_OP_MV, spw.SPW_F64, 4, spw.SPW_PLAN_TILE)   # scatter side, no transpose
    assert ei.value.status_name == "SPW_ERR_UNSUPPORTED"
    M.close()
