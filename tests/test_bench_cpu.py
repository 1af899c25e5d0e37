"""Host logic of bench.py (no GPU): the byte model, the kernel-name labels and
the counter summary that turns rocprofv3 request counts by size into bytes.

The counter summary is fed CSV files laid out as rocprofv3 writes them, with
counts whose bytes are known: a read stream of exactly 1 GiB in 128-byte
requests, a copy of 1 GiB, and a kernel with a mix of 32-, 64- and 128-byte
reads and 32- / 64-byte writes.
"""
import csv
import os

import pytest

import bench

GiB = 1 << 30
PROBE_READ = "spw::(anonymous namespace)::bw_probe_read(HIP_vector_type<unsigned int, 4u> const*, long, unsigned int*)"
PROBE_COPY = ("spw::(anonymous namespace)::bw_probe_copy(HIP_vector_type<unsigned int, 4u> const*, "
              "HIP_vector_type<unsigned int, 4u>*, long)")
VTM = ("void spw::(anonymous namespace)::vtm_wave<512, 16, unsigned short, double, double, false>"
       "(unsigned short const*, double const*)")


def write_pass(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "1_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_model_bytes_matches_the_stated_formula():
    m, n, nnz = 50_000, 20_000_000, 200_201_679
    assert bench.model_bytes(m, n, nnz) == nnz * 12 + 4 * (n + 1) + 8 * n + 8 * m
    assert bench.model_bytes(m, n, nnz, k=4, sv=4, sx=4) == nnz * 8 + 4 * (n + 1) + 16 * n + 16 * m


def test_kernel_label():
    assert bench.kernel_label(VTM) == "vtm_wave<512,16,u16,f64,f64,false>"
    assert bench.kernel_label(PROBE_READ) == "bw_probe_read"
    assert bench.kernel_label("void spw::(anonymous namespace)::cdot_tile<int, float, float, 16, 16, 4, double, 8>"
                              "(int const*)") == "cdot_tile<i32,f32,f32,16,16,4,f64,8>"


def test_counter_summary_bytes_by_request_size(tmp_path, monkeypatch):
    out = tmp_path / "summary.txt"
    monkeypatch.setitem(bench.COUNTER_FILES, "wide", str(out))
    read_rows, write_rows = [], []
    d = 0
    for launch in range(3):
        # the read stream: 1 GiB in 128-byte requests, nothing written
        d += 1
        for c, v in (("TCC_EA0_RDREQ_sum", GiB // 128), ("TCC_EA0_RDREQ_32B_sum", 0),
                     ("TCC_EA0_RDREQ_64B_sum", 0), ("TCC_EA0_RDREQ_128B_sum", GiB // 128)):
            read_rows.append(dict(Dispatch_Id=d, Kernel_Name=PROBE_READ, Counter_Name=c, Counter_Value=v))
        for c, v in (("TCC_EA0_WRREQ_sum", 0), ("TCC_EA0_WRREQ_64B_sum", 0), ("TCC_EA0_RDREQ_DRAM_sum", GiB // 128),
                     ("TCC_EA0_WRREQ_DRAM_sum", 0)):
            write_rows.append(dict(Dispatch_Id=d, Kernel_Name=PROBE_READ, Counter_Name=c, Counter_Value=v))
        # the copy: 1 GiB read in 128-byte requests, 1 GiB written in 64-byte requests
        d += 1
        for c, v in (("TCC_EA0_RDREQ_sum", GiB // 128), ("TCC_EA0_RDREQ_32B_sum", 0),
                     ("TCC_EA0_RDREQ_64B_sum", 0), ("TCC_EA0_RDREQ_128B_sum", GiB // 128)):
            read_rows.append(dict(Dispatch_Id=d, Kernel_Name=PROBE_COPY, Counter_Name=c, Counter_Value=v))
        for c, v in (("TCC_EA0_WRREQ_sum", GiB // 64), ("TCC_EA0_WRREQ_64B_sum", GiB // 64),
                     ("TCC_EA0_RDREQ_DRAM_sum", GiB // 128), ("TCC_EA0_WRREQ_DRAM_sum", GiB // 64)):
            write_rows.append(dict(Dispatch_Id=d, Kernel_Name=PROBE_COPY, Counter_Name=c, Counter_Value=v))
        # a kernel with mixed sizes: 10 x 32 B + 40 x 64 B + 50 x 128 B read (the median launch), 5 x 32 B + 15 x 64 B written
        d += 1
        extra = launch          # launches differ in the total only: the median is taken per counter
        for c, v in (("TCC_EA0_RDREQ_sum", 100 + extra), ("TCC_EA0_RDREQ_32B_sum", 10),
                     ("TCC_EA0_RDREQ_64B_sum", 40), ("TCC_EA0_RDREQ_128B_sum", 50)):
            read_rows.append(dict(Dispatch_Id=d, Kernel_Name=VTM, Counter_Name=c, Counter_Value=v))
        for c, v in (("TCC_EA0_WRREQ_sum", 20), ("TCC_EA0_WRREQ_64B_sum", 15), ("TCC_EA0_RDREQ_DRAM_sum", 90),
                     ("TCC_EA0_WRREQ_DRAM_sum", 20)):
            write_rows.append(dict(Dispatch_Id=d, Kernel_Name=VTM, Counter_Name=c, Counter_Value=v))
    write_pass(str(tmp_path / "read"), read_rows)
    write_pass(str(tmp_path / "write"), write_rows)
    bench.summarize_counters("wide", [str(tmp_path / "read"), str(tmp_path / "write")])
    kv = {}
    for line in out.read_text().splitlines():
        if "=" in line and not line.startswith("#"):
            a, b = line.split("=", 1)
            kv[a] = b
    assert kv["kernel_source_sha256_16"] == bench.kernel_hash()
    assert float(kv["check.bw_probe_read_read_bytes_over_1GiB"]) == 1.0
    assert float(kv["check.bw_probe_copy_read_bytes_over_1GiB"]) == 1.0
    assert float(kv["check.bw_probe_copy_write_bytes_over_1GiB"]) == 1.0
    lab = "vtm_wave<512,16,u16,f64,f64,false>"
    assert int(kv[lab + ".read_bytes"]) == 10 * 32 + 40 * 64 + 50 * 128
    assert int(kv[lab + ".write_bytes"]) == 15 * 64 + 5 * 32
    assert int(kv[lab + ".bytes_per_launch"]) == 10 * 32 + 40 * 64 + 50 * 128 + 15 * 64 + 5 * 32
    assert kv[lab + ".read_requests_32_64_128"] == "10/40/50"
    assert float(kv[lab + ".read_size_split_covers"]) == pytest.approx(100 / 101, abs=1e-4)
    assert float(kv[lab + ".read_requests_to_dram_pct"]) == pytest.approx(100 * 90 / 101, abs=0.05)
    # the headline key the roofline reads
    assert kv["vtm_wave_bytes_per_launch"] == kv[lab + ".bytes_per_launch"]


def test_counter_summary_rejects_unknown_workload(tmp_path):
    with pytest.raises(SystemExit):
        bench.summarize_counters("nonsense", [str(tmp_path)])


def test_traffic_is_read_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    f = tmp_path / "counters.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.read_traffic() is None                      # no summary at all
    f.write_text("# header\nkernel_source_sha256_16=%s\nvtm_wave_bytes_per_launch=1234\n" % bench.kernel_hash())
    kv = bench.read_traffic()
    assert kv is not None and kv["vtm_wave_bytes_per_launch"] == "1234"
    # a summary taken on another kernel source is not used
    f.write_text("kernel_source_sha256_16=0000000000000000\nvtm_wave_bytes_per_launch=1234\n")
    assert bench.read_traffic() is None

