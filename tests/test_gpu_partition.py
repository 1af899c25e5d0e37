"""Column partitioning (the comparison of Section VI) through the C ABI: the
column dots give bit-identical results whichever way the work is divided,
the scatter product agrees with the oracle, and the reported worker
imbalance equals the oracle's Delta = P * (max - min) / nnz."""
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


CASES = {
    "small_wide": lambda: synth.config_matrix("c0", scale=0.3),
    "sorted": lambda: synth.sort_columns_by_length(synth.config_matrix("c0", scale=0.3)),
    "uniform": lambda: synth.uniform_lengths(600, 20000, 0.05, 10, 10, 7),
    "many_empty": lambda: synth.random_csc(300, 40000, 3.0, 4, empty_frac=0.8),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("fmt", [0, 1])
def test_column_partition(spw, case, fmt):
    A = CASES[case]()
    m, n = (A.m, A.n) if fmt == 0 else (A.n, A.m)
    print("partition case %s fmt=%d nnz=%d" % (case, fmt, A.nnz), flush=True)
    Mn = spw.SpwMatrix(fmt, m, n, A.ptr, A.idx, A.val, transpose=0)
    Mc = spw.SpwMatrix(fmt, m, n, A.ptr, A.idx, A.val, transpose=0, partition=spw.SPW_PART_COLUMN)
    x = torch.from_numpy(synth.vector(n, 3, 1)).cuda()
    v = torch.from_numpy(synth.vector(m, 3, 2)).cuda()
    yn, un = Mn.mv(x), Mn.vtm(v)
    yc, uc = Mc.mv(x), Mc.vtm(v)
    # the column-dot direction runs the same chunks: bit-identical
    if fmt == 0:
        assert torch.equal(un, uc)
    else:
        assert torch.equal(yn, yc)
    if fmt == 0:
        yr, dy = oracle.mv_csc(A.m, A.n, A.ptr, A.idx, A.val, x.cpu().numpy(), with_d=True)
        ur, du = oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, v.cpu().numpy(), with_d=True)
    else:
        yr, dy = oracle.mv_csr(A.n, A.m, A.ptr, A.idx, A.val, x.cpu().numpy(), with_d=True)
        ur, du = oracle.vtm_csr(A.n, A.m, A.ptr, A.idx, A.val, v.cpu().numpy(), with_d=True)
    for got, ref, d in ((yc, yr, dy), (uc, ur, du)):
        assert np.all(np.abs(got.cpu().numpy() - ref) <= 1e-13 * d)
    # imbalance of the column-dot workers
    ic, inz = Mc.info(), Mn.info()
    assert ic["partition"] == 1 and inz["partition"] == 0
    P = ic["workers"]
    assert P == inz["workers"] and P >= 1
    delta = P * (ic["worker_max_nnz"] - ic["worker_min_nnz"]) / A.nnz
    assert delta == pytest.approx(oracle.colp_imbalance(A.n, A.ptr, P), rel=1e-12, abs=1e-15)
    # the nonzero split gives every worker the same number of chunks, give or take one
    assert inz["worker_max_nnz"] - inz["worker_min_nnz"] <= 1024
    Mn.close()
    Mc.close()


MERGE_CASES = dict(CASES, news20=lambda: synth.news20_shaped(scale=0.15),
                   news20_sorted=lambda: synth.sort_columns_by_length(synth.news20_shaped(scale=0.15)))


@pytest.mark.parametrize("case", sorted(MERGE_CASES))
@pytest.mark.parametrize("fmt", [0, 1])
def test_merge_path_partition(spw, case, fmt):
    # merge-path workers balance nonzeros plus columns: the column dots stay
    # bit-identical to the nonzero split, the scatter product meets the bar
    A = MERGE_CASES[case]()
    m, n = (A.m, A.n) if fmt == 0 else (A.n, A.m)
    print("merge partition case %s fmt=%d nnz=%d" % (case, fmt, A.nnz), flush=True)
    Mn = spw.SpwMatrix(fmt, m, n, A.ptr, A.idx, A.val, transpose=0)
    Mm = spw.SpwMatrix(fmt, m, n, A.ptr, A.idx, A.val, transpose=0, partition=spw.SPW_PART_MERGE)
    x = torch.from_numpy(synth.vector(n, 5, 1)).cuda()
    v = torch.from_numpy(synth.vector(m, 5, 2)).cuda()
    yn, un = Mn.mv(x), Mn.vtm(v)
    ym, um = Mm.mv(x), Mm.vtm(v)
    if fmt == 0:
        assert torch.equal(un, um)
    else:
        assert torch.equal(yn, ym)
    if fmt == 0:
        yr, dy = oracle.mv_csc(A.m, A.n, A.ptr, A.idx, A.val, x.cpu().numpy(), with_d=True)
        ur, du = oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, v.cpu().numpy(), with_d=True)
    else:
        yr, dy = oracle.mv_csr(A.n, A.m, A.ptr, A.idx, A.val, x.cpu().numpy(), with_d=True)
        ur, du = oracle.vtm_csr(A.n, A.m, A.ptr, A.idx, A.val, v.cpu().numpy(), with_d=True)
    for got, ref, d in ((ym, yr, dy), (um, ur, du)):
        g = got.cpu().numpy()
        assert not np.isnan(g).any()
        assert np.all(np.abs(g - ref) <= 1e-13 * d)
    im = Mm.info()
    assert im["partition"] == 2 and im["workers"] == Mn.info()["workers"]
    assert 0 <= im["worker_min_nnz"] <= im["worker_max_nnz"] <= A.nnz
    Mn.close()
    Mm.close()
