#!/usr/bin/env python3
"""Benchmark of the wide/tall sparse product path on one MI355X.

A step is one pass of the hot path over the 2e8-nonzero wide matrix
(m = 50,000, n = 2e7, FP64): y = A x followed by u^T = v^T A, the
multiply pair the paper's driver repeats.  `value` is the effective HBM
bandwidth of that pair under the algorithmic byte model

    bytes(A x)   = nnz*(8 + 4) + 4*(n+1) + 8*n (read x) + 8*m (write y)
    bytes(v^T A) = nnz*(8 + 4) + 4*(n+1) + 8*m (read v) + 8*n (write u)

(8-byte values, 4-byte indices and pointers), divided by the measured time.
Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  The timed steps take four different x and v in turn
(4 x 160 MB of x), so that no input stays in the 256 MB Infinity Cache from
one step to the next; the rate with one fixed x and v is reported beside it.
Also reports, outside the timed steps: the tall mirror
(the same arrays read as a 2e7 x 50,000 CSR matrix), per-kernel roofline
figures, plain-call latency percentiles, reduced-precision value storage on
the same matrix (binary32 / bfloat16 values, binary32 vectors, with their
error against binary64 products), multi-RHS blocks on the 5e7-nonzero
batching matrix, and the CPU oracle timed on the host.

`--counter-summary WORKLOAD DIR...` folds the rocprofv3 --pmc runs of
`--profile-run` (WORKLOAD wide) or `--profile-batched` (WORKLOAD batched), one
run per counter pass of PMC_PASSES, into the counter summary under profiles/:
HBM bytes per launch from the 32-, 64- and 128-byte request counts, cache hit
rates, LDS and wave-state figures.  `--stats-summary DIR` turns a
`rocprofv3 --kernel-trace --stats` run of the main benchmark into the kernel
statistics summary there (`--batched-stats-summary DIR` the same for
`--batched-only`).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Ax / vᵀA effective HBM GB/s (% of peak); batched vs plain; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
NROT = 4          # input vectors the timed pairs rotate through
# the sources of the single-vector kernels the headline roofline is taken on, and of the tiles
KERNEL_SRCS = [os.path.join(ROOT, "paper_1812_00904_amd", "csrc", f) for f in ("spw_device.h", "spw_kernels.hip")]
TILE_SRCS = [os.path.join(ROOT, "paper_1812_00904_amd", "csrc", "spw_tile.hip")]
COUNTER_FILES = {"wide": os.path.join(ROOT, "profiles", "pmc_counters_wide_2e8.txt"),
                 "batched": os.path.join(ROOT, "profiles", "pmc_counters_batched_5e7.txt")}
TRAFFIC_FILE = COUNTER_FILES["wide"]
STATS_FILE = os.path.join(ROOT, "profiles", "kernel_stats_wide_2e8.txt")
BATCHED_STATS_FILE = os.path.join(ROOT, "profiles", "kernel_stats_batched_5e7.txt")
BATCHED_STATS_COMMAND = "rocprofv3 --kernel-trace --stats -f csv -d <dir> -- python3 bench.py --batched-only"
# One rocprofv3 --pmc run per pass (each within the per-block counter limits).
PMC_PASSES = {
    "read": "TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum",
    "write": "TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum TCC_EA0_RDREQ_DRAM_sum TCC_EA0_WRREQ_DRAM_sum",
    "cache": ("TCC_HIT_sum TCC_MISS_sum TCP_TOTAL_CACHE_ACCESSES_sum TCP_TCC_READ_REQ_sum SQ_LDS_BANK_CONFLICT "
              "SQ_LDS_IDX_ACTIVE SQ_INSTS_LDS SQ_INSTS_LDS_ATOMIC SQ_ACTIVE_INST_LDS SQ_WAIT_INST_LDS"),
    "waves": ("SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CU_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY "
              "SQ_ACTIVE_INST_VMEM SQ_INSTS_VMEM_RD TA_TA_BUSY_sum TA_ADDR_STALLED_BY_TC_CYCLES_sum "
              "TCP_TCC_READ_REQ_LATENCY_sum TCP_TCC_READ_REQ_sum"),
    "latency": "TCC_EA0_RDREQ_LEVEL_sum TCC_EA0_RDREQ_sum GRBM_GUI_ACTIVE",
}
STATS_COMMAND = ("rocprofv3 --kernel-trace --stats -f csv -d <dir> -- python3 bench.py --steps 20 --warmup 3 "
                 "--no-cpu-baseline --no-tall --no-batch --no-precision --no-serving --no-partition --no-solver --no-small")
SOLVER_STATS_FILE = os.path.join(ROOT, "profiles", "kernel_stats_cgls_wide_2e8.txt")
SERVING_BUSY_FILE = os.path.join(ROOT, "profiles", "serving_busy_64_matrices.txt")
SERVING_BUSY_COMMAND = ("rocprofv3 --kernel-trace -f csv -d <dir> -- python3 bench.py --serving-only "
                        "--serving-requests 4000 --serving-loads 1.5")
SOLVER_STATS_COMMAND = ("rocprofv3 --kernel-trace --stats -f csv -d <dir> -- python3 bench.py --steps 3 --warmup 1 "
                        "--no-cpu-baseline --no-tall --no-batch --no-precision --no-serving --no-partition --no-small")


def model_bytes(m: int, n: int, nnz: int, k: int = 1, sv: int = 8, sx: int = 8, si: int = 4, sp: int = 4) -> int:
    """Algorithmic bytes of one product (either direction; they move the same amount)."""
    return nnz * (sv + si) + sp * (n + 1) + k * sx * n + k * sx * m


def kernel_hash(extra=()) -> str:
    """Hash of the device sources of the product kernels (and of `extra`
    sources): a counter summary is used only while it matches."""
    h = hashlib.sha256()
    for p in list(KERNEL_SRCS) + list(extra):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic():
    """Per-kernel HBM bytes per launch from the committed counter summary, if it
    was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        line = line.strip()
        if "=" in line and not line.startswith("#"):
            a, b = line.split("=", 1)
            kv[a.strip()] = b.strip()
    if kv.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return kv


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def host_cpu():
    """Model name of this host's CPU and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def cpu_baseline(A, x, v, budget_s: float = 20.0):
    """The oracle, untuned, single-threaded and pinned to one core of this
    host: as many full mv+vtm pairs over the same matrix as fit about
    `budget_s` seconds (at least one)."""
    import oracle
    model, ncpu, allowed = host_cpu()
    keep = os.sched_getaffinity(0)
    core = min(keep)
    os.sched_setaffinity(0, {core})
    try:
        t_pairs = []
        t0 = time.perf_counter()
        while True:
            t = time.perf_counter()
            oracle.mv_csc(A.m, A.n, A.ptr, A.idx, A.val, x)
            oracle.vtm_csc(A.m, A.n, A.ptr, A.idx, A.val, v)
            t_pairs.append(time.perf_counter() - t)
            if time.perf_counter() - t0 + t_pairs[-1] > budget_s or len(t_pairs) >= 20:
                break
    finally:
        os.sched_setaffinity(0, keep)
    t_med = sorted(t_pairs)[len(t_pairs) // 2]
    pair_bytes = 2 * model_bytes(A.m, A.n, A.nnz)
    return {"value": round(pair_bytes / t_med / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "%d full y=Ax + u^T=v^T A pairs over the same %d-nonzero matrix, single thread pinned to "
                      "core %d, median pair %.3f s" % (len(t_pairs), A.nnz, core, t_med),
            "host_cpu": model, "host_nproc": ncpu, "host_cores_allowed": allowed}


def read_stream_ceiling(dev, gib: int = 4, reps: int = 5):
    """The library's bandwidth probe over `gib` GiB: read-only stream and copy."""
    import torch
    from paper_1812_00904_amd.spw import spw_probe_bandwidth
    n = (gib << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    r_ms, c_ms = spw_probe_bandwidth(src, dst, reps)
    nbytes = n * 8
    del src, dst
    torch.cuda.empty_cache()
    return {"kernel": "bw_probe_read / bw_probe_copy", "bytes": nbytes, "read_ms": round(r_ms, 4),
            "read_GBps": round(nbytes / (r_ms * 1e-3) / 1e9, 1), "copy_ms": round(c_ms, 4),
            "copy_GBps_read_plus_write": round(2 * nbytes / (c_ms * 1e-3) / 1e9, 1)}


def profile_probe(dev):
    """Known traffic for the counter runs: the probe's read-only stream over
    exactly 1 GiB (1 GiB read) and its copy of 1 GiB (1 GiB read, 1 GiB
    written), each launched twice."""
    import torch
    from paper_1812_00904_amd.spw import spw_probe_bandwidth
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    spw_probe_bandwidth(src, dst, 1)
    torch.cuda.synchronize()
    del src, dst


def profile_batched(args):
    """Launches for the counter runs on the batching matrix (m=20,000, n=5e6,
    ~5e7 nonzeros): binary64 at k = 4 (column passes), 16 and 64 (tiles; the
    scatter direction over the kept transpose), binary32 at k = 16 and 64,
    three calls of each direction, then the probe's known traffic."""
    import torch
    import synth
    from paper_1812_00904_amd import (SPW_CSC, SPW_F32, SPW_F64, SPW_OP_MV, SPW_OP_VTM, SPW_PLAN_PASSES,
                                      SPW_PLAN_TILE, SpwMatrix)
    A = synth.config_matrix("c2", scale=args.scale)
    for dtype, vdt, ks in ((torch.float64, SPW_F64, (4, 16, 64)), (torch.float32, SPW_F32, (16, 64))):
        M = SpwMatrix(SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val, transpose=1,
                      **({} if vdt == SPW_F64 else {"value_storage": SPW_F32}))
        for k in ks:
            plan = SPW_PLAN_PASSES if k <= 8 else SPW_PLAN_TILE
            M.set_batch_plan(SPW_OP_MV, vdt, k, plan)
            M.set_batch_plan(SPW_OP_VTM, vdt, k, plan)
            X = torch.rand((A.n, k), dtype=dtype, device="cuda") * 2 - 1
            V = torch.rand((A.m, k), dtype=dtype, device="cuda") * 2 - 1
            Y = torch.empty((A.m, k), dtype=dtype, device="cuda")
            U = torch.empty((A.n, k), dtype=dtype, device="cuda")
            for _ in range(3):
                M.mv_batch(X, Y)
                M.vtm_batch(V, U)
            torch.cuda.synchronize()
            print("[bench] profiled %s k=%d" % (dtype, k), file=sys.stderr, flush=True)
            del X, V, Y, U
        M.close()
        torch.cuda.empty_cache()
    profile_probe("cuda")
    print("[bench] profile run done", file=sys.stderr, flush=True)


def time_pairs(M, xd, vd, yd, ud, steps, warmup, per_step=True):
    """Event-timed y=Ax / u^T=v^T A pairs.  xd and vd may be lists of vectors,
    which step i takes in turn (i mod len): inputs whose total exceeds the
    256 MB Infinity Cache are then read from HBM on every step, as they are in
    a solver whose vectors change from step to step.  per_step adds events
    around each product (for latency percentiles), which cost time of their
    own; without it only the whole loop is bracketed."""
    import torch
    xs = xd if isinstance(xd, (list, tuple)) else [xd]
    vs = vd if isinstance(vd, (list, tuple)) else [vd]
    for i in range(warmup):
        M.mv(xs[i % len(xs)], yd)
        M.vtm(vs[i % len(vs)], ud)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps if per_step else 0)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for i in range(steps):
        if per_step:
            ev[i][0].record()
        M.mv(xs[i % len(xs)], yd)
        if per_step:
            ev[i][1].record()
        M.vtm(vs[i % len(vs)], ud)
        if per_step:
            ev[i][2].record()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(stop)
    mv_ms = [a.elapsed_time(b) for a, b, _ in ev]
    vtm_ms = [b.elapsed_time(c) for _, b, c in ev]
    return total_ms, wall, mv_ms, vtm_ms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workload (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tall", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the multi-RHS section")
    ap.add_argument("--no-precision", action="store_true", help="skip the reduced-precision storage section")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--no-partition", action="store_true", help="skip the column-partitioning comparison")
    ap.add_argument("--no-solver", action="store_true", help="skip the CGLS loop")
    ap.add_argument("--no-small", action="store_true", help="skip the small-matrix latency section")
    ap.add_argument("--solver-iters", type=int, default=20)
    ap.add_argument("--serving-requests", type=int, default=10000)
    ap.add_argument("--serving-loads", default="0.25,0.5,0.9,1.2,1.5",
                    help="comma-separated offered loads, as fractions of the plain path's capacity")
    ap.add_argument("--profile-run", action="store_true",
                    help="a few pairs plus a calibration copy, for rocprofv3 counter runs")
    ap.add_argument("--profile-batched", action="store_true",
                    help="only launch the batched products for rocprofv3 counter runs and exit")
    ap.add_argument("--counter-summary", metavar="ARG", nargs="+",
                    help="WORKLOAD (wide or batched) and the rocprofv3 --pmc output directories of its "
                         "passes -> counter summary")
    ap.add_argument("--batched-stats-summary", metavar="DIR",
                    help="summarize a rocprofv3 --kernel-trace --stats run of --batched-only and exit")
    ap.add_argument("--solver-stats-summary", metavar="DIR",
                    help="summarize a rocprofv3 --kernel-trace --stats run of SOLVER_STATS_COMMAND and exit")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the multi-RHS section and print its result")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving section (for a kernel trace of the server) and print its result")
    ap.add_argument("--serving-busy-summary", metavar="DIR",
                    help="rocprofv3 --kernel-trace output of SERVING_BUSY_COMMAND -> GPU busy time of the server")
    ap.add_argument("--stats-summary", metavar="DIR",
                    help="rocprofv3 --kernel-trace --stats output directory -> kernel statistics summary")
    args = ap.parse_args()

    if args.counter_summary:
        return summarize_counters(args.counter_summary[0], args.counter_summary[1:])
    if args.stats_summary:
        return summarize_stats(args.stats_summary)
    if args.solver_stats_summary:
        return summarize_stats(args.solver_stats_summary, solver=True)
    if args.batched_stats_summary:
        return summarize_stats(args.batched_stats_summary, batched=True)
    if args.serving_busy_summary:
        return summarize_serving_busy(args.serving_busy_summary)
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus %d is not supported (sharding a matrix "
              "over several GPUs is not implemented)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1812_00904_amd import SPW_CSC, SPW_CSR, SpwMatrix, spw_profile_enable, spw_profile_read, \
        spw_profile_reset, spw_profile_select

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.serving_only:
        print(json.dumps({"serving": bench_serving(args)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": bench_batched(args)}), flush=True)
        return
    if args.profile_batched:
        return profile_batched(args)
    t = time.perf_counter()
    A = synth.config_matrix("c1", scale=args.scale)
    x, v = synth.config_vectors("c1", A.m, A.n)
    gen_s = time.perf_counter() - t
    print("[bench] generated m=%d n=%d nnz=%d in %.1fs" % (A.m, A.n, A.nnz, gen_s), file=sys.stderr, flush=True)

    t = time.perf_counter()
    M = SpwMatrix(SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val)
    create_s = time.perf_counter() - t
    info = M.info()
    xd = torch.from_numpy(x).to(dev)
    vd = torch.from_numpy(v).to(dev)
    yd = torch.empty(A.m, dtype=torch.float64, device=dev)
    ud = torch.empty(A.n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    print("[bench] created in %.1fs: %s" % (create_s, info), file=sys.stderr, flush=True)

    if args.profile_run:
        for _ in range(3):
            M.mv(xd, yd)
            M.vtm(vd, ud)
        # binary32 and bfloat16 value storage, binary32 vectors
        x32, v32 = xd.float(), vd.float()
        y32 = torch.empty(A.m, dtype=torch.float32, device=dev)
        u32 = torch.empty(A.n, dtype=torch.float32, device=dev)
        for code in (1, 2):
            S = SpwMatrix(SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val, value_storage=code, transpose=0)
            for _ in range(3):
                S.mv(x32, y32)
                S.vtm(v32, u32)
            torch.cuda.synchronize()
            S.close()
        profile_probe(dev)
        print("[bench] profile run done", file=sys.stderr, flush=True)
        return

    # the timed pairs take four different x and v in turn (4 x 160 MB of x), so
    # that no input stays in the Infinity Cache from one step to the next
    xrot = [xd] + [xd * (1.0 + 0.25 * i) for i in range(1, NROT)]
    vrot = [vd] + [vd * (1.0 + 0.25 * i) for i in range(1, NROT)]
    # 1. a profiled pass with events around every kernel and every product:
    #    per-kernel figures, latency percentiles, and the dominant kernel
    spw_profile_reset()
    spw_profile_select(None)
    spw_profile_enable(True)
    _, _, mv_ms, vtm_ms = time_pairs(M, xrot, vrot, yd, ud, args.steps, args.warmup)
    spw_profile_enable(False)
    prof = spw_profile_read()
    spw_profile_reset()
    dom = max(("mv_bucket", "vtm_wave"), key=lambda k: prof.get(k, (1, 0.0))[1] / max(prof.get(k, (1, 0.0))[0], 1))
    # 2. the timed steps: events only around the dominant kernel's launches
    spw_profile_select(dom)
    spw_profile_enable(True)
    total_ms, wall, _, _ = time_pairs(M, xrot, vrot, yd, ud, args.steps, 2, per_step=False)
    spw_profile_enable(False)
    prof_dom = spw_profile_read()
    spw_profile_reset()
    spw_profile_select(None)
    # 3. the same with one fixed x and v, no events
    same_ms, _, _, _ = time_pairs(M, xd, vd, yd, ud, args.steps, 2, per_step=False)
    del xrot, vrot
    ms_per_step = total_ms / args.steps
    pair_bytes = 2 * model_bytes(A.m, A.n, A.nnz)
    value = pair_bytes / (ms_per_step * 1e-3) / 1e9
    print("[bench] %d pairs in %.3f ms (%.3f ms/pair, wall %.3f s): %.1f GB/s"
          % (args.steps, total_ms, ms_per_step, wall, value), file=sys.stderr, flush=True)

    # per-kernel figures (average launch duration from events on the launch stream)
    kernels = {}
    for name, (launches, tot) in prof.items():
        avg = tot / max(launches, 1)
        kernels[name] = {"launches": launches, "avg_us": round(avg * 1e3, 2)}
    one_op = model_bytes(A.m, A.n, A.nnz)
    for name, op in (("mv_bucket", "mv"), ("vtm_wave", "vtm")):
        if name in kernels:
            gbs = one_op / (kernels[name]["avg_us"] * 1e-6) / 1e9
            kernels[name]["achieved_GBps"] = round(gbs, 1)
            kernels[name]["op"] = op
    traffic = read_traffic()
    tr_val = None
    if traffic and ("%s_bytes_per_launch" % dom) in traffic:
        tr_val = float(traffic["%s_bytes_per_launch" % dom])
    launches, tot = prof_dom[dom]
    dom_us = tot / max(launches, 1) * 1e3
    achieved = round(one_op / (dom_us * 1e-6) / 1e9, 1)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr_val,
                "algorithmic_bytes_per_launch": one_op, "avg_launch_us": round(dom_us, 2),
                "launches_timed": launches}
    # the same launches against the bytes the stored format has to move (the
    # 60 % target is stated on the algorithmic model above)
    if dom == "vtm_wave":
        stored = (A.nnz * (8 + info["index_bytes"]) + info["n_chunks"] * (64 * 2 + 16)
                  + 8 * (A.m + A.n))
        roofline["stored_format_bytes_per_launch"] = stored
        roofline["stored_format_frac"] = round(stored / (dom_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
        roofline["target_basis"] = "algorithmic byte model (ABI: 4-byte indices and pointers)"
    ceiling = read_stream_ceiling(dev)
    roofline["read_stream_ceiling_GBps"] = ceiling["read_GBps"]
    roofline["frac_of_read_ceiling"] = round(achieved / ceiling["read_GBps"], 4)
    print("[bench] read-stream ceiling %s" % ceiling, file=sys.stderr, flush=True)

    extra = {"kernels": kernels, "kernels_from": "a profiled pass of the same steps before the timed one",
             "latency_ms": {"mv_p50": round(percentile(mv_ms, 50), 4), "mv_p99": round(percentile(mv_ms, 99), 4),
                            "vtm_p50": round(percentile(vtm_ms, 50), 4),
                            "vtm_p99": round(percentile(vtm_ms, 99), 4)},
             "mv_GBps": round(one_op / (percentile(mv_ms, 50) * 1e-3) / 1e9, 1),
             "vtm_GBps": round(one_op / (percentile(vtm_ms, 50) * 1e-3) / 1e9, 1),
             "plan": {k: info[k] for k in ("n_chunks", "n_zones", "n_panels", "panel_rows", "mv_workgroups",
                                          "index_bytes", "relabeled", "device_bytes")},
             "generate_s": round(gen_s, 2), "create_s": round(create_s, 2),
             "inputs": "%d different x and v taken in turn" % NROT,
             "pair_same_vectors_GBps": round(pair_bytes / (same_ms / args.steps * 1e-3) / 1e9, 1),
             "read_stream_ceiling": ceiling}
    if traffic:
        extra["traffic_summary"] = os.path.relpath(TRAFFIC_FILE, ROOT)

    if not args.no_tall:
        # the tall mirror: the same arrays as CSR of the n x m transpose
        T = SpwMatrix(SPW_CSR, A.n, A.m, A.ptr, A.idx, A.val)
        xt = vd          # the tall x has the short side's 50,000 entries
        yt = torch.empty(A.n, dtype=torch.float64, device=dev)
        vt = [xd] + [xd * (1.0 + 0.25 * i) for i in range(1, NROT)]   # the long v, taken in turn
        ut = torch.empty(A.m, dtype=torch.float64, device=dev)
        tot, _, tmv, tvtm = time_pairs(T, xt, vt, yt, ut, max(args.steps // 2, 5), 2)
        del vt
        extra["tall"] = {"workload": "CSR m=%d n=%d (same arrays)" % (A.n, A.m),
                         "pair_GBps": round(pair_bytes / (tot / max(args.steps // 2, 5) * 1e-3) / 1e9, 1),
                         "mv_GBps": round(one_op / (percentile(tmv, 50) * 1e-3) / 1e9, 1),
                         "vtm_GBps": round(one_op / (percentile(tvtm, 50) * 1e-3) / 1e9, 1)}
        T.close()
        del yt, ut

    if not args.no_precision:
        extra["precision"] = bench_precision(args, A, M, xd, vd)

    if not args.no_solver:
        extra["solver"] = bench_solver(args, A, M, vd, ms_per_step)

    if not args.no_small:
        extra["small"] = bench_small(args)

    if not args.no_batch:
        M.close()
        del xd, vd, yd, ud
        torch.cuda.empty_cache()
        extra["batched"] = bench_batched(args)

    if not args.no_partition:
        torch.cuda.empty_cache()
        extra["partition"] = bench_partition(args)

    if not args.no_serving:
        torch.cuda.empty_cache()
        extra["serving"] = bench_serving(args)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(A, x, v)

    out = {"metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "wide CSC m=%d n=%d nnz=%d (Zipf(1.1) column lengths + 100 half-dense "
                                  "columns, Zipf(0.8) rows, lognormal values); step = y=Ax then u^T=v^T A"
                                  % (A.m, A.n, A.nnz),
                      "m": A.m, "n": A.n, "nnz": A.nnz, "pair_model_bytes": pair_bytes,
                      "peak_GBps": HBM_PEAK_GBS, "pct_of_peak": round(100 * value / HBM_PEAK_GBS, 2)},
           "roofline": roofline, "cpu_baseline": cpu, "extra": extra}
    print(json.dumps(out), flush=True)
    if args.no_batch:
        M.close()


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _time_each(fn, reps):
    """Median and p99 of `reps` event-timed calls (ms)."""
    import torch
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ts = [a.elapsed_time(b) for a, b in ev]
    return percentile(ts, 50), percentile(ts, 99)


def _err_stats(got, ref, d):
    """max / p99 / median of |got - ref| / d over the entries with d > 0, and the
    number of entries with d == 0 that are not exactly zero."""
    import torch
    got = got.double()
    pos = d > 0
    r = ((got - ref).abs()[pos] / d[pos]).float()
    bad_zero = int(((got != 0) & ~pos).sum().item())
    if r.numel() == 0:
        return {"max": 0.0, "p99": 0.0, "median": 0.0, "nonzero_where_d_is_0": bad_zero}
    q = torch.quantile(r[torch.randperm(r.numel(), device=r.device)[:1 << 24]],
                       torch.tensor([0.5, 0.99], device=r.device))
    return {"max": float(r.max().item()), "p99": float(q[1].item()), "median": float(q[0].item()),
            "nonzero_where_d_is_0": bad_zero}


def bench_precision(args, A, M, xd, vd):
    """Binary32 and bfloat16 value storage on the 2e8-nonzero wide matrix with
    binary32 vectors: effective GB/s of each product (values 4 or 2 bytes, vector
    entries 4 bytes in the byte model) and the error of its output, per entry
    relative to d = sum |a| |x|, against (i) binary64 products with the original
    values and (ii) binary64 products with the stored values (both run by the
    binary64 path of this library, whose parity with the CPU oracle is tested
    to 1e-13 * d)."""
    import torch
    from paper_1812_00904_amd import SPW_CSC, SpwMatrix, spw_round_values
    x32, v32 = xd.float(), vd.float()
    xw, vw = x32.double(), v32.double()
    reps = max(args.steps // 2, 10)
    Mabs = SpwMatrix(SPW_CSC, A.m, A.n, A.ptr, A.idx, abs(A.val), transpose=0)
    dy, du = Mabs.mv(xw.abs()), Mabs.vtm(vw.abs())
    Mabs.close()
    y_o, u_o = M.mv(xw), M.vtm(vw)
    res = {"workload": "same wide CSC matrix, binary32 vectors", "rows": []}
    for name, code, sv in (("f32", 1, 4), ("bf16", 2, 2)):
        t = time.perf_counter()
        S = SpwMatrix(SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val, value_storage=code, transpose=0)
        create_s = time.perf_counter() - t
        y = torch.empty(A.m, dtype=torch.float32, device="cuda")
        u = torch.empty(A.n, dtype=torch.float32, device="cuda")
        mv50, mv99 = _time_each(lambda: S.mv(x32, y), reps)
        vt50, vt99 = _time_each(lambda: S.vtm(v32, u), reps)
        S.mv(x32, y)
        S.vtm(v32, u)
        R = SpwMatrix(SPW_CSC, A.m, A.n, A.ptr, A.idx, spw_round_values(code, A.val), transpose=0)
        y_r, u_r = R.mv(xw), R.vtm(vw)
        R.close()
        by = model_bytes(A.m, A.n, A.nnz, sv=sv, sx=4)
        row = {"values": name, "vectors": "f32", "device_bytes": S.info()["device_bytes"],
               "create_s": round(create_s, 2),
               "mv_ms_p50": round(mv50, 4), "mv_ms_p99": round(mv99, 4),
               "vtm_ms_p50": round(vt50, 4), "vtm_ms_p99": round(vt99, 4),
               "model_bytes": by, "mv_GBps": round(by / (mv50 * 1e-3) / 1e9, 1),
               "vtm_GBps": round(by / (vt50 * 1e-3) / 1e9, 1),
               "mv_err_vs_stored_values": _err_stats(y, y_r, dy),
               "vtm_err_vs_stored_values": _err_stats(u, u_r, du),
               "mv_err_vs_original_values": _err_stats(y, y_o, dy),
               "vtm_err_vs_original_values": _err_stats(u, u_o, du)}
        S.close()
        del y, u, y_r, u_r
        torch.cuda.empty_cache()
        res["rows"].append(row)
        print("[bench] precision %s" % row, file=sys.stderr, flush=True)
    return res


def bench_small(args):
    """The 1e6-nonzero matrix (1,000 x 100,000; 13 MB of model bytes per
    product, fits any cache), where a call is bound by latency: event-timed
    kernel time of single calls warm (back to back) and cold (a 512 MiB write
    between calls pushes the matrix out of the 256 MB Infinity Cache and the
    L2s), and the host wall clock from the call to the end of a stream
    synchronize over 1,000 calls."""
    import torch
    import synth
    from paper_1812_00904_amd import SPW_CSC, SpwMatrix
    A = synth.config_matrix("c0")
    x, v = synth.config_vectors("c0", A.m, A.n)
    M = SpwMatrix(SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val)
    xd, vd = torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda()
    yd = torch.empty(A.m, dtype=torch.float64, device="cuda")
    ud = torch.empty(A.n, dtype=torch.float64, device="cuda")
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    by = model_bytes(A.m, A.n, A.nnz)
    res = {"workload": "wide CSC m=%d n=%d nnz=%d (Zipf(1.1) lengths + 5 dense columns)" % (A.m, A.n, A.nnz),
           "model_bytes": by}
    for name, fn in (("mv", lambda: M.mv(xd, yd)), ("vtm", lambda: M.vtm(vd, ud))):
        w50, w99 = _time_each(fn, 200)
        cold = []
        for _ in range(50):
            flush.fill_(1)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            cold.append(a.elapsed_time(b))
        wall = []
        for _ in range(1000):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            wall.append((time.perf_counter() - t) * 1e3)
        res[name] = {"warm_ms_p50": round(w50, 4), "warm_ms_p99": round(w99, 4),
                     "cold_ms_p50": round(percentile(cold, 50), 4), "cold_ms_p99": round(percentile(cold, 99), 4),
                     "host_ms_p50": round(percentile(wall, 50), 4), "host_ms_p99": round(percentile(wall, 99), 4),
                     "warm_GBps": round(by / (w50 * 1e-3) / 1e9, 1)}
    M.close()
    del flush
    torch.cuda.empty_cache()
    print("[bench] small %s" % res, file=sys.stderr, flush=True)
    return res


def bench_solver(args, A, M, bd, pair_ms):
    """CGLS on the same matrix (spw_cgls, binary64): time per iteration from a
    K-iteration and a 0-iteration call (the difference removes the start-up
    product pair), against the plain product pair.  Byte model per iteration:
    the two products plus the vector passes (q = t + beta q with ||q||^2, and
    r -= alpha q, on the m-vectors: 48 m bytes; ||s||^2, then p = s + beta p
    and x += alpha p on the n-vectors: 48 n bytes)."""
    import numpy as np
    import torch
    K = max(args.solver_iters, 1)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    M.cgls(bd, x, 2, hist=False)
    torch.cuda.synchronize()

    def timed(iters):
        ts = []
        for _ in range(3):
            x.zero_()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            M.cgls(bd, x, iters, hist=False)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return sorted(ts)[1]

    t0, tk = timed(0), timed(K)
    it_ms = (tk - t0) / K
    x.zero_()
    gamma, rho = M.cgls(bd, x, K)
    by = 2 * model_bytes(A.m, A.n, A.nnz) + 48 * A.m + 48 * A.n
    res = {"workload": "CGLS, min ||b - A x||_2 on the same matrix, x0 = 0, binary64",
           "iterations": K, "ms_per_iteration": round(it_ms, 4), "pair_ms": round(pair_ms, 4),
           "vector_overhead_pct": round(100.0 * (it_ms - pair_ms) / pair_ms, 1),
           "model_bytes_per_iteration": by, "GBps": round(by / (it_ms * 1e-3) / 1e9, 1),
           "iterations_per_s": round(1e3 / it_ms, 1), "startup_ms": round(t0, 4),
           "residual_reduction": float(np.sqrt(rho[-1] / rho[0])) if rho[0] > 0 else 0.0,
           "normal_residual_reduction": float(np.sqrt(gamma[-1] / gamma[0])) if gamma[0] > 0 else 0.0}
    del x
    print("[bench] solver %s" % res, file=sys.stderr, flush=True)
    return res


def bench_batched(args):
    """Multi-RHS blocks on the batching matrix (m=20,000, n=5e6, ~5e7 nonzeros):
    one fused pass for k right-hand sides against k plain single-vector calls,
    binary64 (values and vectors) and binary32 (values and vectors), both
    directions.  The matrix is created with the autotuner on: creation times
    the column-dot chunk size and workgroup size, and the first call of each
    (direction, k) times the multi-RHS plans on its own buffers (that call is
    not in the timings).  Each row names the tuned choices."""
    import torch
    import synth
    from paper_1812_00904_amd import SPW_CSC, SPW_F32, SPW_F64, SPW_OP_MV, SPW_OP_VTM, SpwMatrix
    A = synth.config_matrix("c2", scale=args.scale)
    res = {"workload": "wide CSC m=%d n=%d nnz=%d (Zipf(1.1) lengths + 100 half-dense columns, Zipf(0.8) rows)"
                       % (A.m, A.n, A.nnz), "rows": []}
    for dtype, sx in ((torch.float64, 8), (torch.float32, 4)):
        t_create = time.perf_counter()
        M = SpwMatrix(SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val, autotune=1, transpose=1,
                      **({} if sx == 8 else {"value_storage": SPW_F32}))
        t_create = time.perf_counter() - t_create
        info = M.info()
        vdt = SPW_F64 if sx == 8 else SPW_F32
        for k in (1, 4, 16, 64):
            X = torch.rand((A.n, k), dtype=dtype, device="cuda") * 2 - 1
            V = torch.rand((A.m, k), dtype=dtype, device="cuda") * 2 - 1
            Y = torch.empty((A.m, k), dtype=dtype, device="cuda")
            U = torch.empty((A.n, k), dtype=dtype, device="cuda")
            xs = [X[:, c].contiguous() for c in range(k)]
            vs = [V[:, c].contiguous() for c in range(k)]
            ys = [torch.empty(A.m, dtype=dtype, device="cuda") for _ in range(k)]
            us = [torch.empty(A.n, dtype=dtype, device="cuda") for _ in range(k)]
            reps = 3
            t_tune = time.perf_counter()
            M.mv_batch(X, Y)          # first calls: the plans are timed here
            M.vtm_batch(V, U)
            torch.cuda.synchronize()
            t_tune = time.perf_counter() - t_tune
            t_mv = _time(lambda: M.mv_batch(X, Y), reps)
            t_vtm = _time(lambda: M.vtm_batch(V, U), reps)

            def plain_mv():
                for c in range(k):
                    M.mv(xs[c], ys[c])

            def plain_vtm():
                for c in range(k):
                    M.vtm(vs[c], us[c])
            t_pmv = _time(plain_mv, reps)
            t_pvtm = _time(plain_vtm, reps)
            by = model_bytes(A.m, A.n, A.nnz, k=k, sv=sx, sx=sx)
            by1 = model_bytes(A.m, A.n, A.nnz, k=1, sv=sx, sx=sx)
            pmv, _ = M.batch_plan(SPW_OP_MV, vdt, k)
            pvtm, _ = M.batch_plan(SPW_OP_VTM, vdt, k)
            row = {"dtype": "f64" if sx == 8 else "f32", "k": k,
                   "plan": batch_plan(info, k, pmv, pvtm, sx), "create_with_tuning_s": round(t_create, 2),
                   "first_calls_with_tuning_s": round(t_tune, 3),
                   "mv_batch_ms": round(t_mv, 4), "vtm_batch_ms": round(t_vtm, 4),
                   "mv_plain_k_calls_ms": round(t_pmv, 4), "vtm_plain_k_calls_ms": round(t_pvtm, 4),
                   "mv_batch_GBps": round(by / (t_mv * 1e-3) / 1e9, 1),
                   "vtm_batch_GBps": round(by / (t_vtm * 1e-3) / 1e9, 1),
                   "mv_plain_GBps": round(k * by1 / (t_pmv * 1e-3) / 1e9, 1),
                   "vtm_plain_GBps": round(k * by1 / (t_pvtm * 1e-3) / 1e9, 1),
                   "mv_speedup": round(t_pmv / t_mv, 2), "vtm_speedup": round(t_pvtm / t_vtm, 2)}
            res["rows"].append(row)
            print("[bench] batched %s" % row, file=sys.stderr, flush=True)
            del X, V, Y, U, xs, vs, ys, us
            torch.cuda.empty_cache()
        M.close()
    return res


def bench_partition(args):
    """Nonzero partitioning (the paper's method) against column partitioning
    (its Section VI comparison) on one GPU: the same kernels and results, only
    the assignment of work to workers differs.  Three 5e7-nonzero matrices:
    the batching matrix in generated order, the same with columns in
    descending length (the worst case for column partitioning), and a
    2,000 x 100,000 matrix with uniform column lengths (the best case).
    Then the same comparison on a stand-in for the paper's document-term data
    set (19,996 x 1,355,191, 9,097,916 nonzeros, its published heavy-column
    statistics), ingested from coordinate triples as the paper's driver reads
    it, in random column order and in descending column length (the order of
    the paper's first experiment).
    Reports median kernel times of single-vector products and the column
    partition's imbalance Delta = P (max - min) / nnz over its P workers."""
    import numpy as np
    import torch
    import synth
    from paper_1812_00904_amd import SPW_CSC, SPW_PART_COLUMN, SpwMatrix
    base = synth.config_matrix("c2", scale=args.scale)
    mats = [("batching matrix, generated order", base),
            ("batching matrix, columns by descending length", synth.sort_columns_by_length(base)),
            ("uniform lengths 2000 x 100000", synth.uniform_lengths(2000, max(int(100000 * args.scale), 1), 0.274,
                                                                    100, 100, synth.SEED_BASE + 5))]
    news = synth.news20_shaped(scale=min(args.scale, 1.0))
    mats += [("document-term stand-in 19996 x 1355191, random column order", news),
             ("document-term stand-in, columns by descending length", synth.sort_columns_by_length(news))]
    reps = max(args.steps // 2, 10)
    out = []
    for name, A in mats:
        x = torch.rand(A.n, dtype=torch.float64, device="cuda") * 2 - 1
        v = torch.rand(A.m, dtype=torch.float64, device="cuda") * 2 - 1
        y = torch.empty(A.m, dtype=torch.float64, device="cuda")
        u = torch.empty(A.n, dtype=torch.float64, device="cuda")
        row = {"matrix": name, "m": A.m, "n": A.n, "nnz": A.nnz}
        coo = name.startswith("document-term")
        if coo:
            rows_t = A.idx.astype(np.int32)
            cols_t = np.repeat(np.arange(A.n, dtype=np.int32), np.diff(A.ptr))
        for label, opts in (("nonzero", {}), ("column", {"partition": SPW_PART_COLUMN})):
            t_create = time.perf_counter()
            if coo:
                M = SpwMatrix.from_coo(SPW_CSC, A.m, A.n, rows_t, cols_t, A.val, transpose=0, **opts)
            else:
                M = SpwMatrix(SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val, transpose=0, **opts)
            t_create = time.perf_counter() - t_create
            info = M.info()
            mv50, _ = _time_each(lambda: M.mv(x, y), reps)
            vt50, _ = _time_each(lambda: M.vtm(v, u), reps)
            P = info["workers"]
            row[label] = {"mv_ms": round(mv50, 4), "vtm_ms": round(vt50, 4), "workers": P,
                          "worker_max_nnz": info["worker_max_nnz"], "worker_min_nnz": info["worker_min_nnz"],
                          "imbalance_pct": round(100.0 * P * (info["worker_max_nnz"] - info["worker_min_nnz"])
                                                 / max(A.nnz, 1), 2),
                          "zones": info["n_zones"], "pair_GBps": round(2 * model_bytes(A.m, A.n, A.nnz) /
                                                                      ((mv50 + vt50) * 1e-3) / 1e9, 1),
                          "create_s": round(t_create, 2), "created_from": "triples" if coo else "CSC"}
            M.close()
        row["vtm_column_over_nonzero"] = round(row["column"]["vtm_ms"] / row["nonzero"]["vtm_ms"], 2)
        row["mv_column_over_nonzero"] = round(row["column"]["mv_ms"] / row["nonzero"]["mv_ms"], 2)
        out.append(row)
        print("[bench] partition %s" % row, file=sys.stderr, flush=True)
        del x, v, y, u
        torch.cuda.empty_cache()
    return {"rows": out}


def bench_serving(args):
    """64 resident matrices (32 wide CSC, 32 tall CSR; shapes log-uniform) and a
    stream of requests (k = 1..8 columns, A x or v^T A, binary64 or binary32
    vectors) with Poisson arrivals.  The plain path runs each request as k
    single-vector calls on one stream in arrival order; its capacity (requests
    per second back to back) sets the offered loads.  The server runs the same
    arrivals with continuous batching over 4 streams.  Latency is host time
    from submission to completion as seen by a host thread."""
    import threading
    import numpy as np
    import torch
    import synth
    from paper_1812_00904_amd import SPW_CSC, SPW_CSR, SPW_OP_MV, Server, SpwMatrix
    t0 = time.perf_counter()
    specs = synth.serving_specs()
    mats, io = [], []
    for sp in specs:
        A = synth.serving_matrix(sp)
        if sp["tall"]:
            M = SpwMatrix(SPW_CSR, A.n, A.m, A.ptr, A.idx, A.val, transpose=0)
        else:
            M = SpwMatrix(SPW_CSC, A.m, A.n, A.ptr, A.idx, A.val, transpose=0)
        mats.append(M)
        bufs = {}
        for dt in (torch.float64, torch.float32):
            # row-major 8-column blocks (server) and contiguous columns (plain path)
            bufs[dt] = {
                "x_blk": torch.rand((M.n, 8), dtype=dt, device="cuda") * 2 - 1,
                "v_blk": torch.rand((M.m, 8), dtype=dt, device="cuda") * 2 - 1,
                "y_blk": torch.empty((M.m, 8), dtype=dt, device="cuda"),
                "u_blk": torch.empty((M.n, 8), dtype=dt, device="cuda")}
            b = bufs[dt]
            b["x_col"] = [b["x_blk"][:, c].contiguous() for c in range(8)]
            b["v_col"] = [b["v_blk"][:, c].contiguous() for c in range(8)]
            b["y_col"] = [torch.empty(M.m, dtype=dt, device="cuda") for _ in range(8)]
            b["u_col"] = [torch.empty(M.n, dtype=dt, device="cuda") for _ in range(8)]
        io.append(bufs)
        del A
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    nreq = args.serving_requests
    R = synth.serving_requests(nreq, len(mats))
    dts = [torch.float32 if f else torch.float64 for f in R["f32"]]
    model = []
    for i in range(nreq):
        M = mats[R["matrix"][i]]
        info = M.info()
        sx = 4 if dts[i] == torch.float32 else 8
        model.append(info["nnz"] * 12 + 4 * (info["inner_cols"] + 1) + int(R["k"][i]) * sx * (M.m + M.n))
    total_bytes = float(sum(model))
    print("[bench] serving: %d matrices (%.2e nonzeros) ready in %.1fs" %
          (len(mats), sum(M.info()["nnz"] for M in mats), setup_s), file=sys.stderr, flush=True)

    def plain_issue(i, stream):
        M, b, k = mats[R["matrix"][i]], io[R["matrix"][i]][dts[i]], int(R["k"][i])
        for c in range(k):
            if R["op"][i] == SPW_OP_MV:
                M.mv(b["x_col"][c], b["y_col"][c], stream)
            else:
                M.vtm(b["v_col"][c], b["u_col"][c], stream)

    stream = torch.cuda.Stream()
    # capacity of the plain path: every request back to back
    with torch.cuda.stream(stream):
        for i in range(min(200, nreq)):
            plain_issue(i, stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(nreq):
        plain_issue(i, stream)
    torch.cuda.synchronize()
    cap_s = time.perf_counter() - t
    capacity = nreq / cap_s
    res = {"workload": "64 resident matrices (32 wide CSC + 32 tall CSR), %d requests" % nreq,
           "total_nnz": int(sum(M.info()["nnz"] for M in mats)), "setup_s": round(setup_s, 1),
           "plain_back_to_back_s": round(cap_s, 3), "plain_capacity_req_per_s": round(capacity, 1),
           "plain_back_to_back_GBps": round(total_bytes / cap_s / 1e9, 1), "loads": []}

    def run_plain(gaps):
        events = [torch.cuda.Event() for _ in range(nreq)]
        t_sub = [0.0] * nreq
        t_done = [0.0] * nreq

        def completer():
            for i in range(nreq):
                while t_sub[i] == 0.0:
                    time.sleep(0)
                events[i].synchronize()
                t_done[i] = time.perf_counter()
        th = threading.Thread(target=completer)
        th.start()
        start = time.perf_counter()
        due = start
        for i in range(nreq):
            due += gaps[i]
            while time.perf_counter() < due:
                pass
            now = time.perf_counter()
            plain_issue(i, stream)
            events[i].record(stream)
            t_sub[i] = now
        th.join()
        lat = [(t_done[i] - t_sub[i]) * 1e6 for i in range(nreq)]
        span = max(t_done) - start
        return lat, span

    def run_server(gaps):
        S = Server(streams=4, hbm_budget_bytes=64 << 30)
        hs = [S.register(M) for M in mats]
        tickets = []
        start = time.perf_counter()
        due = start
        for i in range(nreq):
            due += gaps[i]
            while time.perf_counter() < due:
                pass
            b, k = io[R["matrix"][i]][dts[i]], int(R["k"][i])
            if R["op"][i] == SPW_OP_MV:
                X, Y = b["x_blk"][:, :k], b["y_blk"][:, :k]
            else:
                X, Y = b["v_blk"][:, :k], b["u_blk"][:, :k]
            tickets.append(S.submit(hs[R["matrix"][i]], int(R["op"][i]), X, Y))
        for tk in tickets:
            S.wait(tk)
        st = S.stats()
        S.close()
        return st

    for load in [float(x) for x in args.serving_loads.split(",") if x]:
        gaps = R["gap"] / (load * capacity)
        lat, span = run_plain(gaps)
        st = run_server(gaps)
        row = {"offered_load": load, "rate_req_per_s": round(load * capacity, 1),
               "plain": {"p50_us": round(percentile(lat, 50), 1), "p99_us": round(percentile(lat, 99), 1),
                         "GBps": round(total_bytes / span / 1e9, 1)},
               "server": {"p50_us": round(st["latency_p50_us"], 1), "p99_us": round(st["latency_p99_us"], 1),
                          "GBps": round(st["gbps"], 1), "groups": st["groups"],
                          "merged_requests": st["merged_requests"], "passes": st["passes"],
                          "hbm_used_GB": round(st["hbm_used_bytes"] / 1e9, 2)}}
        res["loads"].append(row)
        print("[bench] serving %s" % row, file=sys.stderr, flush=True)
    for M in mats:
        M.close()
    return res


def batch_plan(info, k, plan_mv, plan_vtm, sx):
    """The kernel configuration a k-wide block runs with (the tuned plan per
    direction, the tuned column-dot chunk and workgroup sizes)."""
    L = 2
    while L < k:
        L *= 2
    chunk = info["chunk_nnz"]
    wg = info["wg_size_f64"] if sx == 8 else info["wg_size_f32"]
    def tile(ch):
        return ("tiled column dots: chunks of %d nonzeros, one chunk per wave, %d column lanes x %d position "
                "sub-groups of %d nonzeros, batches of 8, 256-thread workgroups" % (ch, L, 64 // L, (ch // 64) * L))
    scatter = ("scatter product: %d row panel(s) of %d rows in LDS, %d workgroup ranges x 4 waves per column, "
               "blocks of 1024 nonzeros" % (info["n_panels"], info["panel_rows"], info["mv_workgroups"]))
    names = {1: "single", 2: "passes", 3: "tile"}
    if k == 1:
        mv, vtm = scatter, ("column dots: chunks of %d nonzeros, one wave per chunk, %d-thread workgroups"
                            % (chunk, wg))
    else:
        mv = {1: "%d single-column passes of the " % k + scatter,
              2: "passes of up to 8 columns of the " + scatter,
              3: tile(1024) + ", over the kept transpose"}[plan_mv]
        vtm = {1: "%d single-column passes of the column dots (chunks of %d)" % (k, chunk),
               2: "column-dot passes of up to 8 columns, each chunk (of %d) loaded once per pass" % chunk,
               3: tile(chunk)}[plan_vtm]
    return {"mv": mv, "vtm": vtm, "mv_plan": names.get(plan_mv, "single"), "vtm_plan": names.get(plan_vtm, "single"),
            "chunk_nnz": chunk, "coldot_wg_size": wg, "tuned": bool(info["tuned"])}


def kernel_label(name: str) -> str:
    """Short kernel name with its template arguments, types abbreviated."""
    n = name.replace("spw::(anonymous namespace)::", "").replace("spw::", "").replace("void ", "").strip()
    depth, end = 0, len(n)
    for i, ch in enumerate(n):              # cut the parameter list after the template arguments
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            end = i
            break
    n = n[:end].replace(" ", "")
    for a, b in (("unsignedshort", "u16"), ("unsignedint", "u32"), ("__hip_bfloat16", "bf16"),
                 ("hip_bfloat16", "bf16"), ("double", "f64"), ("float", "f32")):
        n = n.replace(a, b)
    n = n.replace("<int,", "<i32,")
    return n


COUNTER_WORKLOADS = {
    "wide": ("`bench.py --profile-run`: the wide CSC matrix m=50000 n=2e7 nnz=200201679 (k=1): three y=Ax / "
             "u^T=v^T A pairs with binary64 values and vectors, three with binary32 and three with bfloat16 "
             "storage (binary32 vectors); then the probe's known traffic", "--profile-run"),
    "batched": ("`bench.py --profile-batched`: the batching matrix m=20000 n=5e6 nnz=50425484, three calls of "
                "each direction at binary64 k=4 (column passes), k=16 and 64 (tiles, the scatter direction over "
                "the kept transpose) and binary32 k=16 and 64; then the probe's known traffic",
                "--profile-batched"),
}


def summarize_counters(workload: str, dirs):
    """Fold the rocprofv3 --pmc runs of one profiling mode (one run per pass
    of PMC_PASSES, in any order) into per-kernel figures, each the median over
    that kernel's dispatches:
    - HBM-side bytes: reads = 32 B x TCC_EA0_RDREQ_32B + 64 B x _64B + 128 B x
      _128B, writes = 64 B x TCC_EA0_WRREQ_64B + 32 B x the rest of
      TCC_EA0_WRREQ; the request totals check the split, and the probe's
      read stream and copy of exactly 1 GiB check the byte count;
    - the share of those requests sent to DRAM, the L2 hit rate, the share
      of L1 accesses sent on to L2, LDS bank-conflict cycles per LDS-active
      cycle;
    - wave-state ratios (all in quad-cycles: waiting / resident, VMEM issue /
      resident; resident wave-cycles per busy CU-cycle, which reads as waves
      per SIMD: 1.00 for a launch of one 4-wave workgroup per CU), the
      average L1-to-L2 and L2-to-memory read latencies in cycles.  The DRAM
      request counters see the Infinity Cache as memory: they do not split
      its hits from HBM reads."""
    if workload not in COUNTER_WORKLOADS:
        raise SystemExit("workload must be one of %s" % sorted(COUNTER_WORKLOADS))
    vals = {}
    for d in dirs:
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit("no counter_collection.csv under %s" % d)
        for f in files:
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    key = (kernel_label(r["Kernel_Name"]), r["Counter_Name"].replace("_sum", ""))
                    vals.setdefault(key, {})[r.get("Dispatch_Id", str(len(vals)))] = float(r["Counter_Value"])
    per = {}
    for (kern, cn), by_dispatch in vals.items():
        xs = sorted(by_dispatch.values())
        per.setdefault(kern, {})[cn] = (xs[len(xs) // 2], len(xs))
    desc, mode = COUNTER_WORKLOADS[workload]
    cmds = ["rocprofv3 --pmc %s -f csv -d <dir_%s> -- python3 bench.py %s" % (c, name, mode)
            for name, c in PMC_PASSES.items()]
    out = ["# rocprofv3 counters per kernel launch (median over launches), from %s." % desc,
           "# Bytes come from the request counts by size (32, 64, 128 B); no scale factor is applied.",
           "# commands: " + " ; ".join(cmds) + " ; python3 bench.py --counter-summary %s %s"
           % (workload, " ".join("<dir_%s>" % n for n in PMC_PASSES)),
           "kernel_source_sha256_16=%s" % kernel_hash(TILE_SRCS if workload == "batched" else ())]

    def g(c, name):
        v = c.get(name)
        return None if v is None else v[0]

    order = sorted(per, key=lambda k: (not k.startswith(("vtm_wave", "mv_bucket", "cdot_tile")), k))
    for kern in order:
        c = per[kern]
        if kern.startswith(("at::", "__amd")):
            continue
        launches = max(n for _, n in c.values())
        out.append("# %s (%d launches)" % (kern, launches))
        line = lambda key, v, fmt="%.0f": out.append(("%s.%s=" + fmt) % (kern, key, v))
        r32, r64, r128, rq = (g(c, "TCC_EA0_RDREQ_32B"), g(c, "TCC_EA0_RDREQ_64B"), g(c, "TCC_EA0_RDREQ_128B"),
                              g(c, "TCC_EA0_RDREQ"))
        rd = wr = None
        if None not in (r32, r64, r128):
            rd = 32 * r32 + 64 * r64 + 128 * r128
            line("read_bytes", rd)
            line("read_requests_32_64_128", "%d/%d/%d" % (r32, r64, r128), "%s")
            if rq:
                line("read_size_split_covers", (r32 + r64 + r128) / rq, "%.4f")
        w64, wq = g(c, "TCC_EA0_WRREQ_64B"), g(c, "TCC_EA0_WRREQ")
        if None not in (w64, wq):
            wr = 64 * w64 + 32 * (wq - w64)
            line("write_bytes", wr)
        if rd is not None and wr is not None:
            line("bytes_per_launch", rd + wr)
        if rq and g(c, "TCC_EA0_RDREQ_DRAM") is not None:
            line("read_requests_to_dram_pct", 100.0 * g(c, "TCC_EA0_RDREQ_DRAM") / rq, "%.1f")
        if wq and g(c, "TCC_EA0_WRREQ_DRAM") is not None:
            line("write_requests_to_dram_pct", 100.0 * g(c, "TCC_EA0_WRREQ_DRAM") / wq, "%.1f")
        hit, miss = g(c, "TCC_HIT"), g(c, "TCC_MISS")
        if hit is not None and miss is not None and hit + miss > 0:
            line("L2_hit_pct", 100.0 * hit / (hit + miss), "%.1f")
        acc, req = g(c, "TCP_TOTAL_CACHE_ACCESSES"), g(c, "TCP_TCC_READ_REQ")
        if acc and req is not None:
            line("L1_accesses_sent_to_L2_pct", 100.0 * req / acc, "%.1f")
        bc, act = g(c, "SQ_LDS_BANK_CONFLICT"), g(c, "SQ_LDS_IDX_ACTIVE")
        if act and bc is not None:
            line("LDS_bank_conflict_pct_of_active", 100.0 * bc / act, "%.1f")
        for raw in ("SQ_INSTS_LDS", "SQ_INSTS_LDS_ATOMIC", "SQ_INSTS_VMEM_RD", "SQ_WAVES"):
            if g(c, raw) is not None:
                line(raw, g(c, raw))
        wc = g(c, "SQ_WAVE_CYCLES")
        if wc:
            for num, key in (("SQ_WAIT_ANY", "waiting_pct_of_resident"),
                             ("SQ_WAIT_INST_ANY", "waiting_on_issue_pct_of_resident"),
                             ("SQ_ACTIVE_INST_ANY", "issuing_pct_of_resident"),
                             ("SQ_ACTIVE_INST_VMEM", "vmem_issue_pct_of_resident"),
                             ("SQ_ACTIVE_INST_LDS", "lds_issue_pct_of_resident")):
                if g(c, num) is not None:
                    line(key, 100.0 * g(c, num) / wc, "%.1f")
            if g(c, "SQ_BUSY_CU_CYCLES"):
                line("resident_waves_per_simd", wc / g(c, "SQ_BUSY_CU_CYCLES"), "%.2f")
        lat, lreq = g(c, "TCP_TCC_READ_REQ_LATENCY"), g(c, "TCP_TCC_READ_REQ")
        if lat is not None and lreq:
            line("L1_to_L2_read_latency_cycles", lat / lreq, "%.0f")
        lev = g(c, "TCC_EA0_RDREQ_LEVEL")
        if lev is not None and rq:
            line("L2_to_memory_read_latency_cycles", lev / rq, "%.0f")
        if lev is not None and g(c, "GRBM_GUI_ACTIVE"):
            line("L2_to_memory_reads_in_flight", lev / g(c, "GRBM_GUI_ACTIVE"), "%.0f")
        if g(c, "TA_TA_BUSY") is not None and g(c, "TA_ADDR_STALLED_BY_TC_CYCLES") is not None and g(c, "TA_TA_BUSY"):
            line("TA_addr_stalled_by_L1_pct_of_busy", 100.0 * g(c, "TA_ADDR_STALLED_BY_TC_CYCLES")
                 / g(c, "TA_TA_BUSY"), "%.1f")
    # the probe's known traffic: reads 1 GiB (read stream), reads and writes 1 GiB (copy)
    for kern, want_rd, want_wr in (("bw_probe_read", 1 << 30, 0), ("bw_probe_copy", 1 << 30, 1 << 30)):
        got = [line for line in out if line.startswith(kern + ".read_bytes=")]
        if got:
            rd = float(got[0].split("=")[1])
            out.append("check.%s_read_bytes_over_1GiB=%.4f" % (kern, rd / want_rd))
        gw = [line for line in out if line.startswith(kern + ".write_bytes=")]
        if gw and want_wr:
            out.append("check.%s_write_bytes_over_1GiB=%.4f" % (kern, float(gw[0].split("=")[1]) / want_wr))
    if workload == "wide":
        # the headline kernels (binary64 values and vectors, one right-hand side)
        for base in ("vtm_wave", "mv_bucket", "mv_reduce", "zone_fixup", "gather_vec"):
            for kern in order:
                if kern.startswith(base + "<") and "f64" in kern and not kern.endswith(",true>") \
                        and "f32" not in kern and "bf16" not in kern:
                    hit = [line for line in out if line.startswith(kern + ".bytes_per_launch=")]
                    if hit:
                        out.append("%s_bytes_per_launch=%s" % (base, hit[0].split("=")[1]))
                    break
    path = COUNTER_FILES[workload]
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


def summarize_serving_busy(trace_dir: str):
    """From the kernel trace of a serving-only run (SERVING_BUSY_COMMAND): the
    span of the last offered load (the server's run follows the plain path's),
    the share of it during which at least one kernel ran, and the idle gaps
    between kernels.  A persistent kernel pulling work from a device ring can
    only remove the idle share, so this bounds what it would gain."""
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit("no kernel_trace.csv under %s" % trace_dir)
    ev = []
    with open(files[0]) as fh:
        for r in csv.DictReader(fh):
            ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    ev.sort()
    # the plain path's run and the server's run are separated by the largest
    # idle gap of the trace's second half (setup and the plain run come first)
    half = ev[len(ev) // 2:]
    cut, gap = 0, -1
    for (s0, e0, _), (s1, e1, _) in zip(half, half[1:]):
        if s1 - e0 > gap:
            gap, cut = s1 - e0, s1
    served = [e for e in ev if e[0] >= cut]
    start, end = served[0][0], max(e[1] for e in served)
    busy, cur_s, cur_e = 0, served[0][0], served[0][1]
    gaps = []
    for s_, e_, _ in served[1:]:
        if s_ > cur_e:
            busy += cur_e - cur_s
            gaps.append(s_ - cur_e)
            cur_s, cur_e = s_, e_
        else:
            cur_e = max(cur_e, e_)
    busy += cur_e - cur_s
    span = end - start
    gaps.sort()
    pick = lambda q: gaps[min(len(gaps) - 1, int(q * (len(gaps) - 1)))] / 1e3 if gaps else 0.0
    out = ["# GPU busy time of the server at 1.5x the plain path's capacity (64 resident matrices, the",
           "# serving workload's request stream), from a rocprofv3 kernel trace of the serving section alone.",
           "# command: %s ; python3 bench.py --serving-busy-summary <dir>" % SERVING_BUSY_COMMAND,
           "kernel_source_sha256_16=%s" % kernel_hash(),
           "server_kernels %d" % len(served),
           "server_span_ms %.3f" % (span / 1e6),
           "gpu_busy_ms %.3f" % (busy / 1e6),
           "gpu_busy_fraction %.4f" % (busy / max(span, 1)),
           "idle_gaps %d" % len(gaps),
           "idle_gap_us p50 %.2f p90 %.2f p99 %.2f max %.2f" % (pick(0.5), pick(0.9), pick(0.99), pick(1.0)),
           "idle_total_ms %.3f" % (sum(gaps) / 1e6)]
    with open(SERVING_BUSY_FILE, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


def summarize_stats(stats_dir: str, solver: bool = False, batched: bool = False):
    """Fold the kernel_stats.csv of a `rocprofv3 --kernel-trace --stats` run of
    the main benchmark (STATS_COMMAND), or of the run that adds the solver
    section (SOLVER_STATS_COMMAND), into its kernel statistics summary."""
    files = glob.glob(os.path.join(stats_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit("no kernel_stats.csv under %s" % stats_dir)
    rows = []
    with open(files[0]) as fh:
        for r in csv.DictReader(fh):
            rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                         float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    rows.sort(key=lambda t: -t[5])
    if batched:
        head = ["# rocprofv3 kernel statistics for `bench.py --batched-only`: the batching matrix m=20000 n=5e6",
                "# nnz=50425484 with the autotuner on (creation and the first call of each (direction, k) time",
                "# candidates), binary64 then binary32, k = 1, 4, 16, 64: 3 timed fused calls and 3 x k plain",
                "# calls per direction and k.",
                "# command: %s ; python3 bench.py --batched-stats-summary <dir>" % BATCHED_STATS_COMMAND]
    elif solver:
        head = ["# rocprofv3 kernel statistics for the CGLS loop on the wide CSC matrix m=50000 n=2e7",
                "# nnz=200201679, binary64: 1 + 3 profiled and 2 + 3 timed pairs on rotating x and v, 2 + 3 on one",
                "# x and v, then spw_cgls calls of 2, 3 x 0, 4 x 20 iterations (90 of the 104 product pairs).",
                "# command: %s ; python3 bench.py --solver-stats-summary <dir>" % SOLVER_STATS_COMMAND]
    else:
        head = ["# rocprofv3 kernel statistics for one benchmark run on the wide CSC matrix m=50000 n=2e7",
                "# nnz=200201679, binary64 values and vectors, y=Ax / u^T=v^T A pairs on 4 rotating x and v:",
                "# 3 + 20 profiled, 2 + 20 timed; then 2 + 20 on one x and v.",
                "# command: %s ; python3 bench.py --stats-summary <dir>" % STATS_COMMAND]
    out = head + ["kernel_source_sha256_16=%s" % kernel_hash(TILE_SRCS if batched else ()),
                  "# columns: kernel | calls | average us | min us | max us | share of GPU time"]
    for name, calls, avg, mn, mx, pct in rows:
        out.append("%-56s %5d %10.2f %10.2f %10.2f %7.2f%%" % (kernel_label(name)[:56], calls, avg, mn, mx, pct))
    with open(BATCHED_STATS_FILE if batched else SOLVER_STATS_FILE if solver else STATS_FILE, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


if __name__ == "__main__":
    main()
