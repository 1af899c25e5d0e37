"""Seeded synthetic inputs for the wide/tall sparse product path.

This package is shared by the tests, the CPU oracle checks and the benchmark.
It holds none of the product arithmetic: it only decides sparsity patterns,
values and dense vectors, deterministically from a seed.

Workloads (all column-major / CSC; a tall row-major matrix is the same arrays
read as CSR of the transpose):

* ``c0`` -- small wide matrix, m=1,000, n=100,000, ~1.0e6 nonzeros: column
  lengths from a truncated Zipf(1.1) law plus 5 fully dense columns, rows
  uniform without repeats, values / x / v uniform in [-1, 1).
* ``c1`` -- large document-term-shaped wide matrix, m=50,000, n=2e7, ~2.0e8
  nonzeros: Zipf(1.1) column lengths plus 100 columns at 50% fill, rows drawn
  with Zipf(0.8) popularity over a seeded permutation of the rows, values
  lognormal(0,1) with a random sign, x / v uniform in [-1, 1).
* ``c2`` -- batching matrix, m=20,000, n=5e6, ~5.0e7 nonzeros, c1's law.

The column-length law is read as i.i.d. Zipf(1.1) truncated to {1..K}, with K
the smallest integer whose mean reaches (nnz - dense nonzeros) / n; the long
columns are the explicit dense ones.  These stand in for the document-term
matrix (News20) the paper measures on, which is not available here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libsynth.so")

SEED_BASE = 18120904


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.syn_fill.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                 ctypes.c_void_p, ctypes.c_void_p]
        lib.syn_fill.restype = ctypes.c_int
        lib.syn_vector.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                   ctypes.c_void_p]
        lib.syn_vector.restype = None
        _lib = lib
    return _lib


VALUE_KINDS = {"uniform": 0, "lognormal": 1, "int": 2, "ones": 3}


@dataclass
class Sparse:
    """Column-major arrays of an m x n matrix (or, read as CSR, of its n x m transpose)."""
    m: int
    n: int
    ptr: np.ndarray   # int64, n+1
    idx: np.ndarray   # int32, nnz, strictly increasing within each column
    val: np.ndarray   # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.ptr[-1])


def zipf_lengths_K(alpha: float, target_mean: float, kmax: int) -> int:
    """Smallest K such that Zipf(alpha) truncated to {1..K} has mean >= target_mean."""
    ls = np.arange(1, kmax + 1, dtype=np.float64)
    w = ls ** (-alpha)
    means = np.cumsum(w * ls) / np.cumsum(w)
    hit = np.nonzero(means >= target_mean)[0]
    return int(hit[0] + 1) if hit.size else kmax


def _seed64(ss: np.random.SeedSequence) -> int:
    return int(ss.generate_state(1, dtype=np.uint64)[0])


def from_lengths(m: int, lengths: np.ndarray, seed: int, row_alpha: float | None = None,
                 values: str = "uniform", row_perm_seed: int | None = None) -> Sparse:
    """Fill a pattern whose column lengths are given (each <= m)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    n = lengths.size
    if lengths.size and (lengths.min() < 0 or lengths.max() > m):
        raise ValueError("column lengths must lie in [0, m]")
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=ptr[1:])
    nnz = int(ptr[-1])
    idx = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    ss = np.random.SeedSequence(seed)
    s_fill, s_perm = ss.spawn(2)
    cdf = perm = None
    if row_alpha is not None and m > 0:
        w = np.arange(1, m + 1, dtype=np.float64) ** (-row_alpha)
        cdf = np.cumsum(w) / w.sum()
        cdf[-1] = 1.0
        rng = np.random.Generator(np.random.PCG64(s_perm if row_perm_seed is None else row_perm_seed))
        perm = rng.permutation(m).astype(np.int32)
    rc = _load().syn_fill(m, n, _seed64(s_fill), ptr.ctypes.data,
                          cdf.ctypes.data if cdf is not None else None,
                          perm.ctypes.data if perm is not None else None,
                          VALUE_KINDS[values], idx.ctypes.data, val.ctypes.data)
    if rc != 0:
        raise MemoryError("syn_fill failed")
    return Sparse(m, n, ptr, idx, val)


def vector(length: int, seed: int, stream: int = 0, kind: str = "uniform") -> np.ndarray:
    """Dense vector, uniform in [-1, 1) or integers in [-8, 8]."""
    out = np.empty(length, dtype=np.float64)
    if length:
        _load().syn_vector(length, _seed64(np.random.SeedSequence([seed, stream])), stream,
                           2 if kind == "int" else 0, out.ctypes.data)
    return out


def wide(m: int, n: int, nnz: int, seed: int, len_alpha: float = 1.1, n_dense: int = 0,
         dense_fill: float = 1.0, row_alpha: float | None = None, values: str = "uniform") -> Sparse:
    """Wide matrix with truncated-Zipf column lengths plus `n_dense` dense columns."""
    ss = np.random.SeedSequence(seed)
    s_len, s_dense, s_fill = ss.spawn(3)
    dense_len = int(round(dense_fill * m))
    target = max(nnz - n_dense * dense_len, 0) / max(n, 1)
    K = min(zipf_lengths_K(len_alpha, target, max(m // 2, 1)), m)
    ls = np.arange(1, K + 1, dtype=np.float64)
    pmf = ls ** (-len_alpha)
    cdf = np.cumsum(pmf) / pmf.sum()
    cdf[-1] = 1.0
    rng = np.random.Generator(np.random.PCG64(s_len))
    if target < 1.0:
        # fewer nonzeros than columns: a column holds one nonzero with probability target
        lengths = (rng.random(n) < target).astype(np.int64)
    else:
        lengths = (np.searchsorted(cdf, rng.random(n), side="right") + 1).astype(np.int64)
        np.minimum(lengths, K, out=lengths)
    if n_dense:
        rd = np.random.Generator(np.random.PCG64(s_dense))
        cols = rd.choice(n, size=min(n_dense, n), replace=False)
        lengths[cols] = dense_len
    return from_lengths(m, lengths, _seed64(s_fill), row_alpha=row_alpha, values=values)


CONFIGS = {
    "c0": dict(m=1_000, n=100_000, nnz=1_000_000, len_alpha=1.1, n_dense=5, dense_fill=1.0,
               row_alpha=None, values="uniform"),
    "c1": dict(m=50_000, n=20_000_000, nnz=200_000_000, len_alpha=1.1, n_dense=100, dense_fill=0.5,
               row_alpha=0.8, values="lognormal"),
    "c2": dict(m=20_000, n=5_000_000, nnz=50_000_000, len_alpha=1.1, n_dense=100, dense_fill=0.5,
               row_alpha=0.8, values="lognormal"),
}
CONFIG_IDS = {"c0": 0, "c1": 1, "c2": 2, "c3": 3, "c4": 4}


def config_matrix(name: str, scale: float = 1.0) -> Sparse:
    """The named workload's matrix; `scale` < 1 shrinks n and nnz (same law) for quick runs."""
    c = dict(CONFIGS[name])
    if scale != 1.0:
        c["n"] = max(int(c["n"] * scale), 1)
        dense_nnz = c["n_dense"] * int(round(c["dense_fill"] * c["m"]))
        c["nnz"] = int((c["nnz"] - dense_nnz) * scale) + dense_nnz
    return wide(seed=SEED_BASE + CONFIG_IDS[name], **c)


def config_vectors(name: str, m: int, n: int, k: int = 1):
    """(x, v) for a workload: x has n entries (or n x k), v has m entries (or m x k)."""
    sid = SEED_BASE + CONFIG_IDS[name]
    if k == 1:
        return vector(n, sid, 1), vector(m, sid, 2)
    return vector(n * k, sid, 3).reshape(n, k), vector(m * k, sid, 4).reshape(m, k)


def random_csc(m: int, n: int, mean_len: float, seed: int, values: str = "uniform",
               empty_frac: float = 0.0, max_len: int | None = None,
               row_alpha: float | None = None) -> Sparse:
    """Small test matrices: geometric-ish lengths with a given mean, optional empty columns."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7])))
    cap = m if max_len is None else min(max_len, m)
    if n == 0:
        lengths = np.zeros(0, dtype=np.int64)
    else:
        lengths = np.minimum(rng.geometric(1.0 / max(mean_len, 1.0), size=n), cap).astype(np.int64)
        if empty_frac > 0:
            lengths[rng.random(n) < empty_frac] = 0
    return from_lengths(m, lengths, seed, row_alpha=row_alpha, values=values)


def to_dense(A: Sparse) -> np.ndarray:
    """Dense m x n copy (for brute-force checks on tiny matrices only)."""
    D = np.zeros((A.m, A.n), dtype=np.float64)
    for j in range(A.n):
        s, e = A.ptr[j], A.ptr[j + 1]
        D[A.idx[s:e], j] = A.val[s:e]
    return D


# --------------------------------------------------------------------------
# Serving workload: many resident matrices and a stream of requests
# --------------------------------------------------------------------------
def serving_specs(count: int = 64, seed: int | None = None) -> list:
    """Shapes of the resident matrices: m ~ logU[500, 5e4], n ~ logU[5e4, 5e6],
    nnz ~ logU[1e5, 5e7] clamped to m*n/2; the first half are used as wide CSC
    matrices, the second half as tall CSR matrices (the transposed arrays of a
    generated wide one)."""
    sid = SEED_BASE + CONFIG_IDS["c4"] if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([sid, 1])))
    out = []
    for i in range(count):
        m = int(round(np.exp(rng.uniform(np.log(500), np.log(5e4)))))
        n = int(round(np.exp(rng.uniform(np.log(5e4), np.log(5e6)))))
        nnz = int(round(np.exp(rng.uniform(np.log(1e5), np.log(5e7)))))
        nnz = min(nnz, m * n // 2)
        out.append({"id": i, "m": m, "n": n, "nnz": nnz, "tall": i >= count // 2, "seed": sid * 1000 + i})
    return out


def serving_matrix(spec: dict) -> Sparse:
    """The wide m x n matrix of a spec: the small-matrix generator (truncated
    Zipf(1.1) column lengths, 5 dense columns, uniform rows and values)."""
    return wide(spec["m"], spec["n"], spec["nnz"], spec["seed"], len_alpha=1.1,
                n_dense=min(5, spec["n"]), dense_fill=1.0, row_alpha=None, values="uniform")


def serving_requests(count: int, n_matrices: int, seed: int | None = None) -> dict:
    """Request stream: matrix uniform, operation A x / v^T A 50/50, k ~ U{1..8},
    vector type binary64 / binary32 50/50, exponential inter-arrival gaps of
    mean 1 (scale by 1/rate)."""
    sid = SEED_BASE + CONFIG_IDS["c4"] if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([sid, 2])))
    return {"matrix": rng.integers(0, n_matrices, count), "op": rng.integers(0, 2, count),
            "k": rng.integers(1, 9, count), "f32": rng.random(count) < 0.5,
            "gap": rng.exponential(1.0, count)}


# --------------------------------------------------------------------------
# Column-partitioning comparison (the paper's Section VI experiments)
# --------------------------------------------------------------------------
def sort_columns_by_length(A: Sparse) -> Sparse:
    """The same matrix with its columns in descending order of length (ties by
    index): the worst case for column partitioning."""
    lengths = np.diff(A.ptr)
    order = np.lexsort((np.arange(A.n), -lengths))
    ptr = np.zeros(A.n + 1, dtype=np.int64)
    np.cumsum(lengths[order], out=ptr[1:])
    idx = np.empty_like(A.idx)
    val = np.empty_like(A.val)
    for new, old in enumerate(order):
        s, e = A.ptr[old], A.ptr[old + 1]
        idx[ptr[new]:ptr[new + 1]] = A.idx[s:e]
        val[ptr[new]:ptr[new + 1]] = A.val[s:e]
    return Sparse(A.m, A.n, ptr, idx, val)


def uniform_lengths(m: int, n: int, rho: float, iota_minus: int, iota_plus: int, seed: int) -> Sparse:
    """Column lengths uniform on [floor(rho m) - iota_minus, ceil(rho m) + iota_plus], rows uniform
    without repeats, values uniform [-1, 1): the balanced random matrix of the comparison."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 3])))
    lo = max(int(np.floor(rho * m)) - iota_minus, 0)
    hi = min(int(np.ceil(rho * m)) + iota_plus, m)
    lengths = rng.integers(lo, hi + 1, n).astype(np.int64)
    return from_lengths(m, lengths, seed)


# --------------------------------------------------------------------------
# A stand-in for the paper's document-term matrix (its Section VI data set,
# which is not available here): the published shape and column statistics,
# the rest chosen.
# --------------------------------------------------------------------------
NEWS20_M, NEWS20_N, NEWS20_NNZ = 19996, 1355191, 9097916


def news20_shaped(seed: int | None = None, scale: float = 1.0) -> Sparse:
    """m = 19,996 documents, n = 1,355,191 terms, exactly 9,097,916 nonzeros;
    25 columns hold at least 9,998 nonzeros, the 10 densest 18,531 down to
    11,872 (geometric steps), the next 15 from 11,700 down to 9,998; every other
    column has a length drawn from a Zipf law on {1, ..., 9,997} whose exponent
    is fitted to the remaining nonzeros (term document-frequencies are heavy
    tailed), then a few lengths move by one to hit the total exactly.  Columns
    are in random order, rows follow Zipf(0.5) weights over permuted documents
    (document lengths differ), values are lognormal (tf-idf weights are
    positive).  `scale` < 1 shrinks n and nnz together (tests only)."""
    seed = SEED_BASE + 20 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    m = NEWS20_M
    n = max(int(round(NEWS20_N * scale)), 30)
    total = max(int(round(NEWS20_NNZ * scale)), n + 400000)
    heavy = np.r_[np.round(np.geomspace(18531, 11872, 10)), np.round(np.linspace(11700, 9998, 15))].astype(np.int64)
    rest_n, rest_nnz = n - heavy.size, total - int(heavy.sum())
    kmax = 9997
    ks = np.arange(1, kmax + 1, dtype=np.float64)

    def mean_for(a):
        w = ks ** -a
        return float((ks * w).sum() / w.sum())

    lo, hi = 1.01, 4.0            # mean_for decreases in a
    target = rest_nnz / rest_n
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if mean_for(mid) > target else (lo, mid)
    w = ks ** -(0.5 * (lo + hi))
    lengths = rng.choice(kmax, size=rest_n, p=w / w.sum()).astype(np.int64) + 1
    diff = rest_nnz - int(lengths.sum())
    while diff != 0:
        step = 1 if diff > 0 else -1
        ok = np.nonzero((lengths < kmax) if step > 0 else (lengths > 1))[0]
        pick = rng.choice(ok, size=min(abs(diff), ok.size), replace=False)
        lengths[pick] += step
        diff -= step * pick.size
    lengths = np.r_[heavy, lengths]
    lengths = lengths[rng.permutation(n)]
    return from_lengths(m, lengths, seed, row_alpha=0.5, values="lognormal")
