"""GPU tests of the server: results against the CPU oracle, the same output
alone and in a mix (bit for bit), merging, the HBM budget, a full queue, a
wait time-out, draining on destroy, bad requests and submits from several
threads."""
import ctypes
import threading

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


@pytest.fixture(scope="module")
def mats(spw):
    """Four small matrices: two wide CSC, two tall CSR (one binary32-stored)."""
    out = []
    specs = [(0, synth.random_csc(300, 20000, 6.0, 31, values="lognormal"), 0),
             (0, synth.random_csc(5000, 30000, 8.0, 32, row_alpha=0.8), 1),
             (1, synth.random_csc(700, 15000, 5.0, 33), 0),
             (1, synth.random_csc(80, 9000, 3.0, 34, empty_frac=0.3), 0)]
    for fmt, A, storage in specs:
        m, n = (A.m, A.n) if fmt == 0 else (A.n, A.m)
        M = spw.SpwMatrix(fmt, m, n, A.ptr, A.idx, A.val, value_storage=storage, transpose=0)
        out.append((fmt, A, storage, M))
    yield out
    for *_, M in out:
        M.close()


def make_requests(mats, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        mi = int(rng.integers(len(mats)))
        fmt, A, storage, M = mats[mi]
        op = int(rng.integers(2))
        k = int(rng.integers(1, 9))
        dt = torch.float32 if (storage or rng.random() < 0.5) else torch.float64
        in_len = M.n if op == 0 else M.m
        out_len = M.m if op == 0 else M.n
        X = synth.vector(in_len * k, 1000 + i, 3).reshape(in_len, k)
        if dt == torch.float32:
            X = X.astype(np.float32).astype(np.float64)
        reqs.append(dict(mat=mi, op=op, k=k, dt=dt, X=X, in_len=in_len, out_len=out_len))
    return reqs


def oracle_out(mats, r):
    fmt, A, storage, M = mats[r["mat"]]
    val = A.val if storage == 0 else oracle.round_array(A.val, "f32")
    if fmt == 0:
        f = oracle.mv_csc_batch if r["op"] == 0 else oracle.vtm_csc_batch
        return f(A.m, A.n, A.ptr, A.idx, val, r["X"], with_d=True)
    f = oracle.mv_csr_batch if r["op"] == 0 else oracle.vtm_csr_batch
    return f(A.n, A.m, A.ptr, A.idx, val, r["X"], with_d=True)


def run_server(spw, mats, reqs, together, **opts):
    S = spw.Server(start_paused=1 if together else 0, **opts)
    handles = [S.register(M) for *_, M in mats]
    outs, tickets = [], []
    for r in reqs:
        Xd = torch.from_numpy(r["X"]).to(r["dt"]).cuda()
        Yd = torch.full((r["out_len"], r["k"]), float("nan"), dtype=r["dt"], device="cuda")
        t = S.submit(handles[r["mat"]], r["op"], Xd, Yd)
        if not together:
            S.wait(t)
        outs.append(Yd)
        tickets.append(t)
    if together:
        S.resume()
    for t in tickets:
        S.wait(t)
    st = S.stats()
    S.close()
    return [o.double().cpu().numpy() for o in outs], st


def test_serve_matches_oracle(spw, mats):
    reqs = make_requests(mats, 60, 1)
    outs, st = run_server(spw, mats, reqs, together=True)
    assert st["completed"] == len(reqs) and st["inflight"] == 0
    assert st["merged_requests"] > 0 and st["groups"] < len(reqs)
    for i, (r, Y) in enumerate(zip(reqs, outs)):
        ref, d = oracle_out(mats, r)
        tol = 1e-13 if r["dt"] == torch.float64 else 1e-5
        bad = np.abs(Y - ref) > tol * d
        assert not bad.any(), ("request", i, r["mat"], r["op"], r["k"], r["dt"], int(bad.sum()))


def test_same_alone_and_in_a_mix(spw, mats):
    reqs = make_requests(mats, 40, 2)
    alone, st_a = run_server(spw, mats, reqs, together=False)
    mixed, st_m = run_server(spw, mats, reqs, together=True, streams=3)
    assert st_m["merged_requests"] > 0
    for i, (a, b) in enumerate(zip(alone, mixed)):
        assert np.array_equal(a, b), "request %d differs between alone and mixed" % i


def test_merged_scatter_group_reads_the_matrix_once(spw, mats):
    # four 2-column A x requests on a wide matrix (the scatter direction) queued
    # while paused: one group, one pass over the matrix for all 8 columns, and
    # every column equal bit for bit to a lone single-vector product
    for mi in (0, 1):
        fmt, A, storage, M = mats[mi]
        S = spw.Server(start_paused=1)
        h = S.register(M)
        dt = torch.float32 if storage else torch.float64
        xs = [torch.from_numpy(synth.vector(M.n * 2, 50 + i, 3).reshape(M.n, 2)).to(dt).cuda() for i in range(4)]
        ys = [torch.full((M.m, 2), float("nan"), dtype=dt, device="cuda") for _ in range(4)]
        tickets = [S.submit(h, spw.SPW_OP_MV, x, y) for x, y in zip(xs, ys)]
        S.resume()
        for t in tickets:
            S.wait(t)
        st = S.stats()
        S.close()
        assert st["groups"] == 1 and st["merged_requests"] == 4 and st["passes"] == 1, st
        for x, y in zip(xs, ys):
            for c in range(2):
                ref = M.mv(x[:, c].contiguous())
                torch.cuda.synchronize()
                assert torch.equal(y[:, c].contiguous(), ref), (mi, c)


def test_budget(spw, mats):
    # registration grows each matrix's scratch to 8 columns; measure after that
    S0 = spw.Server()
    for *_, M in mats:
        S0.register(M)
    S0.close()
    sizes = [M.info()["device_bytes"] for *_, M in mats]
    S = spw.Server(hbm_budget_bytes=sizes[0] + sizes[1] // 2)
    assert S.register(mats[0][3]) == 0
    with pytest.raises(spw.SpwError) as ei:
        S.register(mats[1][3])
    assert ei.value.status_name == "SPW_ERR_BUDGET"
    st = S.stats()
    assert st["registered"] == 1 and st["hbm_used_bytes"] <= st["hbm_budget_bytes"]
    S.close()


def test_busy_timeout_and_resume(spw, mats):
    S = spw.Server(start_paused=1, max_inflight=2)
    h = S.register(mats[0][3])
    M = mats[0][3]
    x = torch.ones(M.n, dtype=torch.float64, device="cuda")
    ys = [torch.empty(M.m, dtype=torch.float64, device="cuda") for _ in range(3)]
    t1 = S.submit(h, spw.SPW_OP_MV, x, ys[0])
    t2 = S.submit(h, spw.SPW_OP_MV, x, ys[1])
    with pytest.raises(spw.SpwError) as ei:
        S.submit(h, spw.SPW_OP_MV, x, ys[2])
    assert ei.value.status_name == "SPW_ERR_BUSY"
    assert not S.poll(t1)
    with pytest.raises(spw.SpwError) as ei:
        S.wait(t1, timeout_us=2000)
    assert ei.value.status_name == "SPW_ERR_TIMEOUT"
    S.resume()
    S.wait(t1)
    S.wait(t2)
    assert S.poll(t1) and S.poll(t2)
    ref = M.mv(x)
    assert torch.equal(ys[0], ref) and torch.equal(ys[1], ref)
    assert S.stats()["rejected_busy"] == 1
    S.close()


def test_destroy_drains_queue(spw, mats):
    S = spw.Server(start_paused=1)
    h = S.register(mats[2][3])
    M = mats[2][3]
    v = torch.linspace(-1, 1, M.m, dtype=torch.float64, device="cuda")
    us = [torch.full((M.n,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(5)]
    for u in us:
        S.submit(h, spw.SPW_OP_VTM, v, u)
    S.close()                      # never resumed: destroy still runs the queue
    torch.cuda.synchronize()
    ref = M.vtm(v)
    for u in us:
        assert torch.equal(u, ref)


def test_bad_requests(spw, mats):
    S = spw.Server()
    h = S.register(mats[0][3])
    M = mats[0][3]
    x = torch.ones((M.n, 2), dtype=torch.float64, device="cuda")
    y = torch.empty((M.m, 2), dtype=torch.float64, device="cuda")
    for bad in (lambda: S.submit(h + 5, spw.SPW_OP_MV, x, y),
                lambda: S.submit(h, 7, x, y),
                lambda: S.submit(h, spw.SPW_OP_MV, x[:, :0], y[:, :0]),
                lambda: S.submit(h, spw.SPW_OP_MV, x.to(torch.int64), y)):
        with pytest.raises((spw.SpwError, TypeError, ValueError)):
            bad()
    # an output leading dimension of 2^18 or more on the column-dot side is
    # refused before anything touches the (here too small) buffers
    lib = spw.load()
    r = spw.Request()
    r.struct_size = ctypes.sizeof(spw.Request)
    csc = M.info()["format"] == spw.SPW_CSC
    r.matrix, r.op, r.vdt, r.k = h, (spw.SPW_OP_VTM if csc else spw.SPW_OP_MV), spw.SPW_F64, 2
    r.in_, r.ldi, r.out, r.ldo = x.data_ptr(), 2, y.data_ptr(), 1 << 18
    t = ctypes.c_uint64()
    assert lib.spw_serve_submit(S.handle, ctypes.byref(r), ctypes.byref(t)) == 6     # SPW_ERR_UNSUPPORTED
    with pytest.raises(spw.SpwError) as ei:
        S.register(mats[0][3])                   # twice
    assert ei.value.status_name == "SPW_ERR_INVALID_ARG"
    with pytest.raises(spw.SpwError):
        S.wait(12345)
    S.close()


def test_submits_from_threads(spw, mats):
    reqs = make_requests(mats, 48, 3)
    S = spw.Server(streams=4)
    handles = [S.register(M) for *_, M in mats]
    outs = [None] * len(reqs)
    errors = []

    def worker(lo, hi):
        try:
            for i in range(lo, hi):
                r = reqs[i]
                Xd = torch.from_numpy(r["X"]).to(r["dt"]).cuda()
                Yd = torch.empty((r["out_len"], r["k"]), dtype=r["dt"], device="cuda")
                torch.cuda.synchronize()
                t = S.submit(handles[r["mat"]], r["op"], Xd, Yd)
                S.wait(t)
                outs[i] = Yd.double().cpu().numpy()
        except Exception as e:          # reported below
            errors.append(e)

    th = [threading.Thread(target=worker, args=(q * 12, q * 12 + 12)) for q in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    S.close()
    assert not errors, errors
    for r, Y in zip(reqs, outs):
        ref, d = oracle_out(mats, r)
        tol = 1e-13 if r["dt"] == torch.float64 else 1e-5
        assert np.all(np.abs(Y - ref) <= tol * d)
