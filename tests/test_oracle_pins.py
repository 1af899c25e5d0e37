"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

None of these re-types the oracle's own loops: each compares it with an
independent route (dense brute force in exact integer arithmetic, a library
routine, a closed form, an invariant, or the worked example printed in the
paper, stored under tests/golden/ with its citation).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def _ex():
    with open(GOLDEN) as f:
        return json.load(f)


def _csc_from_cols(cols_1based, m):
    lengths = [len(c) for c in cols_1based]
    ptr = np.zeros(len(cols_1based) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(lengths)
    idx = np.array([r - 1 for c in cols_1based for r in c], dtype=np.int32)
    return ptr, idx


def _int_matrix(m, n, mean_len, seed, empty_frac=0.0):
    return synth.random_csc(m, n, mean_len, seed, values="int", empty_frac=empty_frac)


def _dense_int(A):
    D = synth.to_dense(A)
    assert np.all(D == np.round(D))
    return D.astype(np.int64)


# ---------------------------------------------------------------------------
# Products: exact integer arithmetic (every partial sum is an exact binary64
# integer), so the oracle must agree bit for bit with int64 dense products.
# A dropped term, a wrong index, a transposed operand or a sign slip all fail.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(1, 1), (5, 8), (17, 64), (64, 3), (40, 200)])
@pytest.mark.parametrize("seed", [0, 1])
def test_products_exact_on_integers(shape, seed):
    m, n = shape
    A = _int_matrix(m, n, 3.0, seed, empty_frac=0.2)
    D = _dense_int(A)
    x = synth.vector(n, seed, 1, kind="int")
    v = synth.vector(m, seed, 2, kind="int")
    y, dy = oracle.mv_csc(m, n, A.ptr, A.idx, A.val, x, with_d=True)
    u, du = oracle.vtm_csc(m, n, A.ptr, A.idx, A.val, v, with_d=True)
    xi, vi = x.astype(np.int64), v.astype(np.int64)
    assert np.array_equal(y, (D @ xi).astype(np.float64))
    assert np.array_equal(u, (vi @ D).astype(np.float64))
    assert np.array_equal(dy, (np.abs(D) @ np.abs(xi)).astype(np.float64))
    assert np.array_equal(du, (np.abs(vi) @ np.abs(D)).astype(np.float64))
    # the tall (row-major) forms: the same arrays read as CSR of the n x m transpose
    yt, dyt = oracle.mv_csr(n, m, A.ptr, A.idx, A.val, v, with_d=True)
    ut, dut = oracle.vtm_csr(n, m, A.ptr, A.idx, A.val, x, with_d=True)
    assert np.array_equal(yt, (D.T @ vi).astype(np.float64))
    assert np.array_equal(ut, (xi @ D.T).astype(np.float64))
    assert np.array_equal(dyt, (np.abs(D.T) @ np.abs(vi)).astype(np.float64))
    # the tall v^T A denominator, d_j = sum_i |v_i||a_ij| over the n x m transpose
    assert np.array_equal(dut, (np.abs(xi) @ np.abs(D.T)).astype(np.float64))


@pytest.mark.parametrize("shape", [(1, 1), (9, 40), (33, 7)])
@pytest.mark.parametrize("k", [1, 3])
def test_batched_products_and_denominators_exact_on_integers(shape, k):
    # Every output and every error denominator of the four multi-RHS forms
    # against int64 dense products: |A| |X| for the y side, |V|^T |A| for u.
    m, n = shape
    A = _int_matrix(m, n, 3.0, 20 + k, empty_frac=0.2)
    D = _dense_int(A)
    X = synth.vector(n * k, 21, 1, kind="int").reshape(n, k)
    V = synth.vector(m * k, 21, 2, kind="int").reshape(m, k)
    Xi, Vi = X.astype(np.int64), V.astype(np.int64)
    f = lambda a: a.astype(np.float64)
    Y, DY = oracle.mv_csc_batch(m, n, A.ptr, A.idx, A.val, X, with_d=True)
    U, DU = oracle.vtm_csc_batch(m, n, A.ptr, A.idx, A.val, V, with_d=True)
    assert np.array_equal(Y, f(D @ Xi)) and np.array_equal(DY, f(np.abs(D) @ np.abs(Xi)))
    assert np.array_equal(U, f(D.T @ Vi)) and np.array_equal(DU, f(np.abs(D.T) @ np.abs(Vi)))
    # the same arrays read as CSR of the n x m transpose
    Yt, DYt = oracle.mv_csr_batch(n, m, A.ptr, A.idx, A.val, V, with_d=True)
    Ut, DUt = oracle.vtm_csr_batch(n, m, A.ptr, A.idx, A.val, X, with_d=True)
    assert np.array_equal(Yt, f(D.T @ Vi)) and np.array_equal(DYt, f(np.abs(D.T) @ np.abs(Vi)))
    assert np.array_equal(Ut, f(D @ Xi)) and np.array_equal(DUt, f(np.abs(D) @ np.abs(Xi)))


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_products_float_against_dense_within_bound(seed):
    m, n = 31, 57
    A = synth.random_csc(m, n, 6.0, seed, values="lognormal", empty_frac=0.1)
    D = synth.to_dense(A)
    x = synth.vector(n, seed, 1)
    v = synth.vector(m, seed, 2)
    y, dy = oracle.mv_csc(m, n, A.ptr, A.idx, A.val, x, with_d=True)
    u, du = oracle.vtm_csc(m, n, A.ptr, A.idx, A.val, v, with_d=True)
    # Higham's bound for a length-L dot product: |err| <= gamma_L sum|a||x| with
    # gamma_L = L u / (1 - L u); both routes obey it, so they differ by <= 2 gamma_L.
    uround = 2.0 ** -53
    L = max(m, n)
    g = 2 * L * uround / (1 - L * uround)
    assert np.all(np.abs(y - D @ x) <= g * dy)
    assert np.all(np.abs(u - v @ D) <= g * du)
    assert np.allclose(dy, np.abs(D) @ np.abs(x), rtol=4 * g, atol=0)


@pytest.mark.parametrize("seed", [0, 9])
def test_products_match_scipy_sparse(seed):
    A = synth.random_csc(300, 2000, 5.0, seed, values="lognormal", empty_frac=0.05)
    x = synth.vector(A.n, seed, 1)
    v = synth.vector(A.m, seed, 2)
    S = sp.csc_matrix((A.val, A.idx, A.ptr), shape=(A.m, A.n))
    y = oracle.mv_csc(A.m, A.n, A.ptr, A.idx, A.val, x)
    u = oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, v)
    # scipy's compressed-column kernels accumulate in the same storage order
    np.testing.assert_allclose(y, S @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(u, S.T @ v, rtol=1e-13, atol=1e-13)


def test_identity_and_permutation_exact():
    n = 50
    rng = np.random.default_rng(11)
    perm = rng.permutation(n)
    x = synth.vector(n, 11, 1)
    # identity: A = I
    ptr = np.arange(n + 1, dtype=np.int64)
    idx = np.arange(n, dtype=np.int32)
    val = np.ones(n)
    assert np.array_equal(oracle.mv_csc(n, n, ptr, idx, val, x), x)
    assert np.array_equal(oracle.vtm_csc(n, n, ptr, idx, val, x), x)
    # permutation: column j has its one entry in row perm[j], so (A x)[perm[j]] = x[j]
    idxp = perm.astype(np.int32)
    y = oracle.mv_csc(n, n, ptr, idxp, val, x)
    expect = np.empty(n)
    expect[perm] = x
    assert np.array_equal(y, expect)
    u = oracle.vtm_csc(n, n, ptr, idxp, val, x)
    assert np.array_equal(u, x[perm])


def test_unit_vectors_pick_columns_and_rows():
    A = synth.random_csc(23, 41, 4.0, 5, values="lognormal", empty_frac=0.2)
    D = synth.to_dense(A)
    for j in (0, 7, 40):
        e = np.zeros(A.n)
        e[j] = 1.0
        assert np.array_equal(oracle.mv_csc(A.m, A.n, A.ptr, A.idx, A.val, e), D[:, j])
    for i in (0, 11, 22):
        e = np.zeros(A.m)
        e[i] = 1.0
        assert np.array_equal(oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, e), D[i, :])


def test_all_ones_matrix_sums():
    m, n = 9, 13
    lengths = np.full(n, m, dtype=np.int64)
    A = synth.from_lengths(m, lengths, 3, values="ones")
    x = synth.vector(n, 3, 1, kind="int")
    v = synth.vector(m, 3, 2, kind="int")
    assert np.array_equal(oracle.mv_csc(m, n, A.ptr, A.idx, A.val, x), np.full(m, x.sum()))
    assert np.array_equal(oracle.vtm_csc(m, n, A.ptr, A.idx, A.val, v), np.full(n, v.sum()))


@pytest.mark.parametrize("seed", [1, 2])
def test_adjoint_identity(seed):
    A = synth.random_csc(200, 3000, 8.0, seed, values="lognormal", empty_frac=0.1)
    x = synth.vector(A.n, seed, 1)
    v = synth.vector(A.m, seed, 2)
    y = oracle.mv_csc(A.m, A.n, A.ptr, A.idx, A.val, x)
    u = oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, v)
    lhs = float(np.dot(v, y))
    rhs = float(np.dot(u, x))
    absA = A.val.copy()
    np.abs(absA, out=absA)
    scale = float(np.abs(v) @ oracle.mv_csc(A.m, A.n, A.ptr, A.idx, absA, np.abs(x)))
    uround = 2.0 ** -53
    col_len = int(np.diff(A.ptr).max())
    row_len = int(np.bincount(A.idx, minlength=A.m).max())
    L = max(A.n + row_len, A.m + col_len)
    g = L * uround / (1 - L * uround)
    assert abs(lhs - rhs) <= 2 * g * scale


def test_batched_columns_equal_single_calls():
    A = synth.random_csc(37, 90, 5.0, 8, values="lognormal", empty_frac=0.1)
    k = 5
    X = synth.vector(A.n * k, 8, 3).reshape(A.n, k)
    V = synth.vector(A.m * k, 8, 4).reshape(A.m, k)
    Y, DY = oracle.mv_csc_batch(A.m, A.n, A.ptr, A.idx, A.val, X, with_d=True)
    U = oracle.vtm_csc_batch(A.m, A.n, A.ptr, A.idx, A.val, V)
    D = synth.to_dense(A)
    for c in range(k):
        y, dy = oracle.mv_csc(A.m, A.n, A.ptr, A.idx, A.val, X[:, c], with_d=True)
        assert np.array_equal(Y[:, c], y)
        assert np.array_equal(DY[:, c], dy)
        assert np.array_equal(U[:, c], oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, V[:, c]))
    np.testing.assert_allclose(Y, D @ X, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(U, D.T @ V, rtol=1e-12, atol=1e-12)
    Yt = oracle.mv_csr_batch(A.n, A.m, A.ptr, A.idx, A.val, V)
    Ut = oracle.vtm_csr_batch(A.n, A.m, A.ptr, A.idx, A.val, X)
    np.testing.assert_allclose(Yt, D.T @ V, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Ut, D @ X, rtol=1e-12, atol=1e-12)


def test_empty_matrix_and_zero_sizes():
    ptr = np.zeros(6, dtype=np.int64)
    idx = np.zeros(0, dtype=np.int32)
    val = np.zeros(0)
    y = oracle.mv_csc(4, 5, ptr, idx, val, np.ones(5))
    u = oracle.vtm_csc(4, 5, ptr, idx, val, np.ones(4))
    assert np.array_equal(y, np.zeros(4)) and np.array_equal(u, np.zeros(5))


# ---------------------------------------------------------------------------
# Value-storage rounding: binary32 against the hardware conversion, bfloat16
# against its defining properties and against torch on binary32 inputs.
# ---------------------------------------------------------------------------
def test_round_f32_matches_hardware_cast():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(20000) * np.exp2(rng.integers(-140, 120, 20000))
    x = np.concatenate([x, [0.0, -0.0, 1.0, 3.4028234663852886e38, 1.1754943508222875e-38,
                            1.401298464324817e-45, 0.7e-45, 0.71e-45]])
    r = oracle.round_array(x, "f32")
    assert np.array_equal(r, x.astype(np.float32).astype(np.float64))


def test_round_bf16_properties_and_ties():
    rng = np.random.default_rng(6)
    x = rng.standard_normal(20000) * np.exp2(rng.integers(-60, 60, 20000))
    r = oracle.round_array(x, "bf16")
    # representable: as binary32, the low 16 bits are zero
    bits = r.astype(np.float32).view(np.uint32)
    assert np.all(r.astype(np.float32).astype(np.float64) == r)
    assert np.all(bits & 0xFFFF == 0)
    # nearest: within half a unit of the 8-bit significand
    e = np.floor(np.log2(np.abs(x)))
    half_ulp = np.exp2(e - 8)
    assert np.all(np.abs(r - x) <= half_ulp * (1 + 1e-12))
    # ties go to the even significand: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert oracle.round_value(1.0 + 2.0 ** -8, "bf16") == 1.0
    assert oracle.round_value(1.0 + 3 * 2.0 ** -8, "bf16") == 1.0 + 2 * 2.0 ** -7
    assert oracle.round_value(-(1.0 + 2.0 ** -8), "bf16") == -1.0
    # one rounding from binary64, not two: just above the tie rounds up
    assert oracle.round_value(1.0 + 2.0 ** -8 + 2.0 ** -40, "bf16") == 1.0 + 2.0 ** -7


def test_round_bf16_matches_torch_on_binary32_inputs():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(20000) * np.exp2(rng.integers(-60, 60, 20000))).astype(np.float32)
    xd = x.astype(np.float64)
    ours = oracle.round_array(xd, "bf16")
    theirs = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, theirs)


# ---------------------------------------------------------------------------
# Partition, cover, zones, setup variables: the worked example of Figures 1-3
# and Tables I-II, and invariants stated in Section IV.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("fig", ["fig1_rows_per_column", "fig2_rows_per_column"])
def test_worked_example_partition_and_zones(fig):
    ex = _ex()
    ptr, idx = _csc_from_cols(ex[fig], ex["m"])
    assert int(ptr[-1]) == ex["Z"]
    off = oracle.offsets_paper(ex["Z"], ex["P"])
    assert np.array_equal(np.diff(off), np.full(ex["P"], ex["group_size"]))
    jf, jl = oracle.cover(ex["n"], ptr, off)
    # cover sets: every column between jf and jl with a nonzero in the group
    J = []
    for g in range(ex["P"]):
        cols = sorted({int(np.searchsorted(ptr, p, side="right") - 1) + 1 for p in range(off[g], off[g + 1])})
        J.append(cols)
        assert cols[0] == jf[g] + 1 and cols[-1] == jl[g] + 1
    assert J[0] == ex["J0"] and J[1] == ex["J1"]
    assert J == ex["fig3_x_replication"]
    zc, sf, sl = oracle.zones(ex["n"], ptr, off)
    assert [int(c) + 1 for c in zc] == [z["column"] for z in ex["table1_zones"]]
    assert [list(range(a, b + 1)) for a, b in zip(sf, sl)] == [z["S"] for z in ex["table1_zones"]]
    sv = oracle.setup_vars(jf, jl)
    for name, row in ex["table2"].items():
        assert list(sv[name]) == row, name


def _check_setup_against_zones(n, ptr, off):
    P = off.size - 1
    jf, jl = oracle.cover(n, ptr, off)
    sv = oracle.setup_vars(jf, jl)
    zc, sf, sl = oracle.zones(n, ptr, off)
    z = zc.size
    assert z <= P - 1 or P == 1 and z == 0
    rank = {int(c): k for k, c in enumerate(zc)}
    groups_of = [[] for _ in range(P)]
    for k in range(z):
        for g in range(sf[k], sl[k] + 1):
            groups_of[g].append(k)
    for g in range(P):
        # a processor is in at most two groups (Section IV-B)
        assert len(groups_of[g]) <= 2
        if sv["needLeft"][g]:
            k = rank[int(jf[g])]
            assert sv["leftGroup"][g] == k
            assert sv["procsOnLeft"][g] == g - sf[k]
        if sv["needRight"][g]:
            k = rank[int(jl[g])]
            assert sv["rightGroup"][g] == k
            assert sv["procsOnRight"][g] == sl[k] - g
        assert bool(sv["needLeft"][g]) == (int(jf[g]) in rank and sf[rank[int(jf[g])]] < g)
        assert bool(sv["needRight"][g]) == (int(jl[g]) in rank and sl[rank[int(jl[g])]] > g)
    # only consecutive zones intersect, by at most one processor; even zones are
    # pairwise disjoint and so are odd zones (Section IV-A)
    for a in range(z):
        for b in range(a + 1, z):
            inter = max(0, min(sl[a], sl[b]) - max(sf[a], sf[b]) + 1)
            if b == a + 1:
                assert inter <= 1
            else:
                assert inter == 0
    return z


@pytest.mark.parametrize("P", [1, 2, 3, 7, 16, 64])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_setup_scans_agree_with_zone_definition(P, seed):
    A = synth.random_csc(30, 400, 4.0, seed, empty_frac=0.2, max_len=30)
    # make one long column spanning several groups
    A2 = synth.from_lengths(200, np.r_[np.diff(A.ptr), [200, 3, 200]], seed)
    for B in (A, A2):
        off = oracle.offsets_paper(B.nnz, P)
        _check_setup_against_zones(B.n, B.ptr, off)
        if B.nnz >= 40:
            offf = oracle.offsets_fixed(B.nnz, max(B.nnz // (P + 1), 1))
            _check_setup_against_zones(B.n, B.ptr, offf)


def test_offsets_rules():
    for Z, P in [(21, 7), (22, 7), (100, 3), (5, 5), (1000003, 64)]:
        off = oracle.offsets_paper(Z, P)
        sizes = np.diff(off)
        assert off[0] == 0 and off[-1] == Z
        assert sizes.max() - sizes.min() <= 1
        assert np.all(sizes[: Z % P] == -(-Z // P)) and np.all(sizes[Z % P:] == Z // P)
    off = oracle.offsets_fixed(10, 4)
    assert list(off) == [0, 4, 8, 10]


def test_random_generator_zone_count_matches_expectation():
    # A balanced matrix in the spirit of the paper's random generator: with
    # column lengths near the mean L, a group boundary falls inside a column
    # (and so creates a zone) unless it lands exactly on a column start:
    # E[z] ~ (P - 1)(1 - 1/L).  Statistical check only.
    m, n, L = 200, 20000, 20
    rng = np.random.default_rng(1)
    lengths = rng.integers(L - 5, L + 6, n)
    A = synth.from_lengths(m, lengths, 1)
    for P in (64, 512):
        off = oracle.offsets_paper(A.nnz, P)
        zc, _, _ = oracle.zones(A.n, A.ptr, off)
        expect = (P - 1) * (1 - 1 / L)
        assert abs(zc.size - expect) <= 4 * np.sqrt(P) + 2


# ---------------------------------------------------------------------------
# Serial simulation of the nonzero-partitioned algorithms (Sections III, IV-A):
# the split changes only the grouping of the sums, so on integer data it must
# equal the plain product exactly, and within rounding otherwise.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("P", [1, 2, 3, 7, 64])
def test_nzp_simulation_equals_plain_product(P):
    A = _int_matrix(40, 500, 6.0, 21, empty_frac=0.1)
    A = synth.from_lengths(40, np.r_[np.diff(A.ptr), [40, 40]], 21, values="int")
    x = synth.vector(A.n, 21, 1, kind="int")
    v = synth.vector(A.m, 21, 2, kind="int")
    off = oracle.offsets_paper(A.nnz, P)
    assert np.array_equal(oracle.nzp_mv(A.m, A.n, A.ptr, A.idx, A.val, off, x),
                          oracle.mv_csc(A.m, A.n, A.ptr, A.idx, A.val, x))
    assert np.array_equal(oracle.nzp_vtm(A.m, A.n, A.ptr, A.idx, A.val, off, v),
                          oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, v))
    B = synth.random_csc(40, 500, 6.0, 22, values="lognormal", empty_frac=0.1)
    xf = synth.vector(B.n, 22, 1)
    vf = synth.vector(B.m, 22, 2)
    offb = oracle.offsets_paper(B.nnz, P)
    y, dy = oracle.mv_csc(B.m, B.n, B.ptr, B.idx, B.val, xf, with_d=True)
    u, du = oracle.vtm_csc(B.m, B.n, B.ptr, B.idx, B.val, vf, with_d=True)
    g = 2 * 600 * 2.0 ** -53
    assert np.all(np.abs(oracle.nzp_mv(B.m, B.n, B.ptr, B.idx, B.val, offb, xf) - y) <= g * dy)
    assert np.all(np.abs(oracle.nzp_vtm(B.m, B.n, B.ptr, B.idx, B.val, offb, vf) - u) <= g * du)


def test_colp_imbalance_closed_form():
    # column counts 2,4,2,5,1,4,1,2 (Figure 1); two spans of 4 columns hold 13 and 8
    ex = _ex()
    ptr, _ = _csc_from_cols(ex["fig1_rows_per_column"], ex["m"])
    assert oracle.colp_imbalance(8, ptr, 2) == pytest.approx(2 * (13 - 8) / 21)
    assert oracle.colp_imbalance(8, ptr, 1) == 0.0
    # eight single-column spans: max 5, min 1
    assert oracle.colp_imbalance(8, ptr, 8) == pytest.approx(8 * (5 - 1) / 21)
    # three spans, the first 8 mod 3 = 2 one column longer: columns 0-2, 3-5,
    # 6-7 hold 8, 10 and 3 nonzeros
    assert oracle.colp_imbalance(8, ptr, 3) == pytest.approx(3 * (10 - 3) / 21)


# ---------------------------------------------------------------------------
# CGLS (Section VII: first-order methods alternating the two products)
# ---------------------------------------------------------------------------
def _cgls_case(fmt, seed, m_w=12, n_w=40):
    """A small random matrix in the requested layout with its dense copy: wide
    CSC (m_w x n_w), or the same arrays read as tall CSR (n_w x m_w)."""
    B = synth.random_csc(m_w, n_w, 3.0, seed)
    D = synth.to_dense(B)
    if fmt == "csr":
        return B, D.T.copy(), n_w, m_w
    return B, D, m_w, n_w


@pytest.mark.parametrize("fmt", ["csc", "csr"])
@pytest.mark.parametrize("seed", [1, 2])
def test_cgls_converges_to_min_norm_least_squares(fmt, seed):
    # From x0 = 0, CGLS iterates stay in range(A^T) and converge to the
    # minimum-norm least-squares solution, which numpy's SVD-based lstsq returns.
    B, D, m, n = _cgls_case(fmt, seed)
    rng = np.random.default_rng(seed)
    b = rng.uniform(-1, 1, m)
    x, gamma, rho = oracle.cgls(fmt, m, n, B.ptr, B.idx, B.val, b, np.zeros(n), 4 * min(m, n))
    x_ref = np.linalg.lstsq(D, b, rcond=None)[0]
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    assert gamma[-1] <= 1e-18 * gamma[0]


@pytest.mark.parametrize("fmt", ["csc", "csr"])
def test_cgls_residual_history_matches_direct_residual(fmt):
    # rho_k is carried by recursion (r <- r - alpha q); it must equal ||b - A x||^2
    # recomputed densely from the returned iterate, and ||r_k|| never grows.
    B, D, m, n = _cgls_case(fmt, 5)
    b = np.random.default_rng(5).uniform(-1, 1, m)
    x0 = np.random.default_rng(6).uniform(-1, 1, n)
    for iters in (0, 1, 3, 7):
        x, gamma, rho = oracle.cgls(fmt, m, n, B.ptr, B.idx, B.val, b, x0, iters)
        r = b - D @ x
        assert abs(rho[-1] - r @ r) <= 1e-12 * (1.0 + r @ r)
        g = D.T @ r
        assert abs(gamma[-1] - g @ g) <= 1e-10 * (1.0 + g @ g)
        assert np.all(np.diff(rho) <= 1e-14 * rho[0])
    assert np.array_equal(oracle.cgls(fmt, m, n, B.ptr, B.idx, B.val, b, x0, 0)[0], x0)


def test_cgls_finite_termination_two_singular_values():
    # A = [diag(1, 1, 2, 2) | 0] has two distinct singular values: exact CG
    # finishes in two steps, so x_2 is the minimum-norm solution up to rounding.
    cols = [[1], [2], [3], [4], [], []]
    ptr, idx = _csc_from_cols(cols, 4)
    val = np.array([1.0, 1.0, 2.0, 2.0])
    b = np.array([1.0, -2.0, 3.0, 0.5])
    x, gamma, _ = oracle.cgls("csc", 4, 6, ptr, idx, val, b, np.zeros(6), 2)
    assert np.allclose(x, [1.0, -2.0, 1.5, 0.25, 0.0, 0.0], rtol=0, atol=1e-15)
    assert gamma[2] <= 1e-28
    # one step is not enough: the first step is a steepest-descent step
    x1, _, _ = oracle.cgls("csc", 4, 6, ptr, idx, val, b, np.zeros(6), 1)
    s0 = np.array([1.0, -2.0, 6.0, 1.0, 0, 0])
    Ds = np.array([1.0, -2.0, 12.0, 2.0])
    assert np.allclose(x1, (s0 @ s0) / (Ds @ Ds) * s0, rtol=1e-15, atol=0)


def test_cgls_zero_right_hand_side_stays_zero():
    B, D, m, n = _cgls_case("csc", 3)
    x, gamma, rho = oracle.cgls("csc", m, n, B.ptr, B.idx, B.val, np.zeros(m), np.zeros(n), 5)
    assert not np.any(x) and not np.any(gamma) and not np.any(rho)
