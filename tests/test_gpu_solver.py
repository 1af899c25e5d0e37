"""GPU parity of the CGLS loop (spw_cgls) against the oracle's CGLS.

Iterates of two correct CGLS runs drift apart by rounding: the products agree
to 1e-13 * sum|a||x| per component, the inner products are summed in different
orders, and each iteration can amplify a relative perturbation of its inputs
by about the condition number kappa(A^T A) = kappa(A)^2 (the step sizes are
ratios of squared norms).  So after k iterations the bar is
    |x_gpu - x_oracle|_inf <= 1e-12 * (4 kappa^2)^k * |x_oracle|_inf
(likewise for the histories, relative to their first entry), with kappa(A)
computed from the test matrix; the matrices here are well conditioned, so the
bar stays small.  Repeated runs must be bit-identical, and from x0 = 0 the
iterates must reach numpy's minimum-norm least-squares solution.
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def layout(spw, B, fmt):
    """(format code, m, n, dense A) for the arrays of B read as wide CSC or tall CSR."""
    D = synth.to_dense(B) if B.m * B.n <= 4e7 else None
    if fmt == "csc":
        return spw.SPW_CSC, B.m, B.n, D
    return spw.SPW_CSR, B.n, B.m, (None if D is None else D.T)


def bar(kappa, iters):
    return min(1e-12 * (4.0 * kappa * kappa) ** iters, 1e-6)


def run(spw, B, fmt, b, x0, iters, opts=None):
    code, m, n, _ = layout(spw, B, fmt)
    M = spw.SpwMatrix(code, m, n, B.ptr, B.idx, B.val, **(opts or {}))
    x = dev(x0)
    gamma, rho = M.cgls(dev(b), x, iters)
    out = x.cpu().numpy()
    M.close()
    return out, gamma, rho


@pytest.mark.parametrize("fmt", ["csc", "csr"])
@pytest.mark.parametrize("iters", [0, 1, 6])
def test_cgls_matches_oracle(spw, fmt, iters):
    # 300 x 20,000 (wide) or its transpose (tall): several chunks, panels and a
    # ragged tail; random start so every vector path is exercised
    B = synth.random_csc(300, 20000, 4.0, 11)
    code, m, n, D = layout(spw, B, fmt)
    rng = np.random.default_rng(3)
    b, x0 = rng.uniform(-1, 1, m), rng.uniform(-1, 1, n)
    kappa = np.linalg.cond(D)
    x, gamma, rho = run(spw, B, fmt, b, x0, iters)
    xo, go, ro = oracle.cgls(fmt, m, n, B.ptr, B.idx, B.val, b, x0, iters)
    tol = bar(kappa, iters)
    assert np.max(np.abs(x - xo)) <= tol * np.max(np.abs(xo)), (kappa, np.max(np.abs(x - xo)))
    assert np.all(np.abs(gamma - go) <= tol * go[0])
    assert np.all(np.abs(rho - ro) <= tol * ro[0])
    if iters == 0:
        assert np.array_equal(x, x0)


@pytest.mark.parametrize("fmt", ["csc", "csr"])
def test_cgls_reaches_min_norm_least_squares(spw, fmt):
    B = synth.random_csc(64, 3000, 3.0, 12)
    code, m, n, D = layout(spw, B, fmt)
    b = np.random.default_rng(4).uniform(-1, 1, m)
    x, gamma, rho = run(spw, B, fmt, b, np.zeros(n), 4 * min(m, n))
    x_ref = np.linalg.lstsq(D, b, rcond=None)[0]
    assert np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    assert np.all(np.diff(rho) <= 1e-14 * rho[0])


def test_cgls_bit_identical_runs_and_plan_options(spw):
    B = synth.random_csc(500, 40000, 5.0, 13, row_alpha=0.8)
    rng = np.random.default_rng(5)
    b, x0 = rng.uniform(-1, 1, 500), rng.uniform(-1, 1, 40000)
    x1, g1, r1 = run(spw, B, "csc", b, x0, 5)
    x2, g2, r2 = run(spw, B, "csc", b, x0, 5)
    assert np.array_equal(x1, x2) and np.array_equal(g1, g2) and np.array_equal(r1, r2)
    # another plan (no row renumbering, column partitioning) changes the
    # rounding order of the products only
    xo, go, _ = oracle.cgls("csc", 500, 40000, B.ptr, B.idx, B.val, b, x0, 5)
    kappa = np.linalg.cond(synth.to_dense(B))
    for opts in (dict(relabel=0), dict(partition=spw.SPW_PART_COLUMN), dict(panel_rows=97)):
        x3, g3, _ = run(spw, B, "csc", b, x0, 5, opts)
        assert np.max(np.abs(x3 - xo)) <= bar(kappa, 5) * np.max(np.abs(xo)), opts


def test_cgls_zero_right_hand_side_and_empty_columns(spw):
    B = synth.random_csc(200, 5000, 2.0, 14, empty_frac=0.3)
    x, gamma, rho = run(spw, B, "csc", np.zeros(200), np.zeros(5000), 4)
    assert not np.any(x) and not np.any(gamma) and not np.any(rho)
    # exact solution reached: later steps have zero size, nothing turns into NaN
    D = synth.to_dense(B)
    xs = np.random.default_rng(6).uniform(-1, 1, 5000)
    xs[np.diff(B.ptr) == 0] = 0.0
    b = D @ xs
    x, gamma, rho = run(spw, B, "csc", b, np.zeros(5000), 400)
    assert np.isfinite(x).all() and np.isfinite(gamma).all()
    assert np.linalg.norm(D @ x - b) <= 1e-9 * np.linalg.norm(b)


def test_cgls_full_size_matches_oracle(spw):
    # The 2e8-nonzero benchmark matrix, 3 iterations from x0 = 0 against the
    # oracle (about 10 s of CPU).  kappa(A) is not computable at this size; the
    # ratio of the largest to the smallest squared row norm (about 5e3 for
    # Zipf(0.8) rows) already puts the bar above its 1e-6 cap, which still
    # catches any wrong step (those are off by O(1)).
    A = synth.config_matrix("c1")
    _, b = synth.config_vectors("c1", A.m, A.n)
    M = spw.SpwMatrix(spw.SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val, transpose=0)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    gamma, rho = M.cgls(dev(b), x, 3)
    xg = x.cpu().numpy()
    M.close()
    xo, go, ro = oracle.cgls("csc", A.m, A.n, A.ptr, A.idx, A.val, b, np.zeros(A.n), 3)
    tol = bar(1e9, 3)
    print("full-size CGLS drift: x %.3g, gamma %.3g, rho %.3g" % (
        np.max(np.abs(xg - xo)) / np.max(np.abs(xo)), np.max(np.abs(gamma - go)) / go[0],
        np.max(np.abs(rho - ro)) / ro[0]))
    assert np.max(np.abs(xg - xo)) <= tol * np.max(np.abs(xo))
    assert np.all(np.abs(gamma - go) <= tol * go[0]) and np.all(np.abs(rho - ro) <= tol * ro[0])
    assert rho[3] < rho[0]


def test_cgls_argument_errors(spw):
    lib = spw.load()
    B = synth.random_csc(50, 400, 2.0, 15)
    M = spw.SpwMatrix(spw.SPW_CSC, 50, 400, B.ptr, B.idx, B.val)
    b, x = dev(np.ones(50)), dev(np.zeros(400))
    hist = np.empty(4)
    assert lib.spw_cgls(M.handle, spw.SPW_F32, b.data_ptr(), x.data_ptr(), 1, hist.ctypes.data, None) != 0
    assert lib.spw_cgls(M.handle, spw.SPW_F64, b.data_ptr(), x.data_ptr(), -1, None, None) != 0
    assert lib.spw_cgls(M.handle, spw.SPW_F64, None, x.data_ptr(), 1, None, None) != 0
    assert lib.spw_cgls(None, spw.SPW_F64, b.data_ptr(), x.data_ptr(), 1, None, None) != 0
    # the failed calls left x alone; a good call without a history only enqueues
    assert lib.spw_cgls(M.handle, spw.SPW_F64, b.data_ptr(), x.data_ptr(), 2, None, None) == 0
    torch.cuda.synchronize()
    assert torch.isfinite(x).all()
    M.close()


def test_cgls_call_captured_in_a_graph(spw):
    # A call without a history only enqueues launches that are the same on
    # every call, so a caller can capture it in a graph: each replay must give
    # the bits of one more direct call, with other work and synchronizations
    # between the replays.
    B = synth.random_csc(400, 30000, 4.0, 16, row_alpha=0.8)
    rng = np.random.default_rng(9)
    b, x0 = rng.uniform(-1, 1, 400), rng.uniform(-1, 1, 30000)
    M = spw.SpwMatrix(spw.SPW_CSC, 400, 30000, B.ptr, B.idx, B.val)
    bd = dev(b)
    # direct: three calls of 2 iterations, each from the previous result
    xe = dev(x0)
    expected = []
    for _ in range(3):
        M.cgls(bd, xe, 2, hist=False)
        torch.cuda.synchronize()
        expected.append(xe.cpu().numpy().copy())
    # captured: the workspace exists already (grown by the calls above)
    xg = dev(x0)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        M.cgls(bd, xg, 2, hist=False)
    xg.copy_(dev(x0))           # capture does not run the work
    torch.cuda.synchronize()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(xg.cpu().numpy(), expected[rep]), rep
        M.mv(dev(x0), torch.empty(400, dtype=torch.float64, device="cuda"))   # other work between replays
        torch.cuda.synchronize()
    del graph
    M.close()


@pytest.mark.parametrize("fmt", ["csc", "csr"])
def test_cgls_long_run_reaches_least_squares(spw, fmt):
    # 250 iterations (five direct q = A p refreshes): the iterate must sit at
    # numpy's least-squares solution and at the oracle's, and the recurred
    # residual norm must match the residual of the returned iterate, so the
    # recurrences have not drifted
    B = synth.random_csc(40, 1500, 4.0, 21)
    code, m, n, D = layout(spw, B, fmt)
    rng = np.random.default_rng(8)
    b = rng.uniform(-1, 1, m)
    x, gamma, rho = run(spw, B, fmt, b, np.zeros(n), 250)
    xo, go, ro = oracle.cgls(fmt, m, n, B.ptr, B.idx, B.val, b, np.zeros(n), 250)
    xs = np.linalg.lstsq(D, b, rcond=None)[0]
    scale = np.max(np.abs(xs))
    assert np.max(np.abs(x - xs)) <= 1e-9 * scale
    assert np.max(np.abs(x - xo)) <= 1e-9 * scale
    r_true = b - D @ x
    assert abs(rho[-1] - r_true @ r_true) <= 1e-9 * (b @ b)
    assert np.all(np.isfinite(gamma)) and np.all(np.isfinite(rho))
