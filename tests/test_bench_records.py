"""Host-side checks of the benchmark's bookkeeping: the committed counter records are read
only for the workload and kernel source they were taken with, and the algorithmic byte
count is the state plus the CSR."""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_traffic_records_match_workload_and_source():
    cases = [("step_kernel_traffic.json", bench.DEVICE_SOURCES),
             ("slice_step_traffic.json", bench.SLICE_SOURCES),
             ("compact_step_traffic.json", bench.COMPACT_SOURCES),
             ("dense_tile128_kernel_traffic.json", bench.DENSE_SOURCES),
             ("slot_step_traffic.json", bench.SLOT_SOURCES),
             ("resident_traffic.json", bench.RESIDENT_SOURCES)]
    for name, sources in cases:
        recs = json.load(open(os.path.join(ROOT, "profiles", name)))
        for rec in recs if isinstance(recs, list) else [recs]:
            assert rec["workload"] in bench.WORKLOADS or rec["workload"] == bench.BATCH_WORKLOAD, (name, rec["workload"])
            got = bench.traffic_from_profiles(name, sources, rec["workload"])
            if rec["kernel_source_sha256"] == bench.source_hash(sources):
                assert got == rec["bytes_per_launch"]
                # FETCH_SIZE scaled by what a plain copy reads back, WRITE_SIZE as counted (KiB)
                f = rec.get("fetch_kib_per_dispatch", rec.get("fetch_kib_per_dispatch_raw"))
                w = rec.get("write_kib_per_dispatch", rec.get("write_kib_per_dispatch_raw"))
                per = rec.get("updates_per_dispatch", 1)
                assert abs(1024 * (f * rec["fetch_scale"] + w * rec["write_scale"]) / per - got) < 2.0, name
            else:
                assert got is None
        # another workload never borrows a record
        other = [w for w in bench.WORKLOADS if w not in
                 {r["workload"] for r in (recs if isinstance(recs, list) else [recs])}][0]
        assert bench.traffic_from_profiles(name, sources, other) is None
        # a record is void once its kernel source changes
        assert bench.traffic_from_profiles(name, ["qqa_color.hip"], recs[0]["workload"] if isinstance(recs, list)
                                           else recs["workload"]) is None


def test_algorithmic_bytes():
    # 24 B of state per replica-variable, plus the CSR: 4 (n + 1) + 4 nnz, and 4 nnz of weights
    n, nnz, S = 20000, 100560, 256
    assert bench.algorithmic_bytes_per_update_launch(n, nnz, S, S, False) == 24 * n * S + 4 * (n + 1) + 4 * nnz
    assert bench.algorithmic_bytes_per_update_launch(n, nnz, S, S, True) == 24 * n * S + 4 * (n + 1) + 8 * nnz


def test_default_line_records_are_current():
    # the counter records the default bench line reports were taken with the kernel sources
    # in the tree (a kernel change leaves its traffic unmeasured until the counters are retaken)
    for name, sources, workload in [
            ("slice_step_traffic.json", bench.SLICE_SOURCES, "mis_er_n20000_d5_S256_K3000"),
            ("slice_step_traffic.json", bench.SLICE_SOURCES, "maxcut_ba_n100000_m4_pm1_S128_K3000"),
            ("dense_tile128_kernel_traffic.json", bench.DENSE_SOURCES, "maxcut_dense_n4096_gauss_S256_K3000"),
            ("resident_traffic.json", bench.RESIDENT_SOURCES, bench.BATCH_WORKLOAD)]:
        assert bench.traffic_from_profiles(name, sources, workload) is not None, (name, workload)
