"""Host logic of bench.py (CPU): the byte model, the traffic record's guards
and the one-GPU contract."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("n,nnz", [(4096, 20_224), (2_097_152, 14_581_760), (1_000_000, 27_009_777)])
def test_iteration_bytes_are_the_sum_of_launch_bytes(n, nnz):
    """Each schedule's per-iteration model is the sum of its launches: p-BiCGSafe runs one
    product of each class and, with the separate pass, one inner-product pass."""
    for sched, classes in ((0, ("spmv", "dots", "update", "spmv_fused")),
                           (1, ("spmv", "update", "spmv_fused")),
                           (2, ("spmv", "update", "spmv_fused")),
                           (3, ("spmv", "update", "spmv_fused"))):
        per_launch = sum(bench.bytes_per_launch(c, n, nnz, sched) for c in classes)
        for variant in ("pbicgsafe", "pbicgsafe_rr"):
            assert bench.bytes_per_iteration(variant, n, nnz, sched) == per_launch, (sched, variant)
    # the fused schedules skip the 40n pass: 8n (schedule 1) and 32n (schedule 2) fewer bytes
    b0, b1, b2, b3 = (bench.bytes_per_iteration("pbicgsafe", n, nnz, s) for s in (0, 1, 2, 3))
    assert b0 - b1 == 8 * n and b0 - b2 == 32 * n
    assert b3 == b2  # the same vector traffic on one stream
    # p-BiCGStab on one stream: the dot passes' 56n gone, r0* read by both passes (16n)
    assert bench.bytes_per_iteration("pbicgstab", n, nnz, 0) - \
        bench.bytes_per_iteration("pbicgstab", n, nnz, 3) == 40 * n
    # the device layout's own matrix bytes replace the CSR estimate when known
    info = {"matrix_bytes": 123_456}
    assert bench.bytes_per_iteration("pbicgsafe", n, nnz, 2, info) == 2 * 123_456 + 248 * n


def test_recorded_traffic_is_refused_when_it_does_not_apply():
    t = json.load(open(bench.TRAFFIC_FILE))
    assert bench.load_traffic("spmv_fused", "rand_band_1m", t.get("schedule")) is None
    assert bench.load_traffic("spmv_fused", t.get("workload"), 99) is None
    assert bench.load_traffic("no_such_class", t.get("workload"), t.get("schedule")) is None
    # the digest covers the solver's sources: it is a stable function of them
    assert bench.source_digest() == bench.source_digest() and len(bench.source_digest()) == 16
    # every solver source (all of csrc but the warm-start network's) is in the digest
    csrc = os.path.join(os.path.dirname(bench.__file__), "paper_2108_10591_amd", "csrc")
    assert sorted(bench.SOLVER_SOURCES) == sorted(f for f in os.listdir(csrc)
                                                  if not f.startswith("wsnet"))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_batch_bytes_use_the_layout_that_ran():
    """A system's share of a batch iteration: rows padded to 512, entries at the layout's
    bytes per slot and padding ratio (not the CSR int32 estimate)."""
    from paper_2108_10591_amd import workloads as W
    A = W.cd2d(40, 10.0)  # 1600 rows -> 2048 padded
    sell = {"format": "sell", "index_bits": 16, "slots": 2 * 1000, "nnz": 1000, "gather_sort": 0}
    got = bench.batch_bytes_per_iteration(sell, A, 2)
    assert got == 2 * (10 * 2 * A.nnz + 4 * (2048 / 64 + 1)) + 248 * 2048
    csr = {"format": "csr", "index_bits": 32, "slots": 1000, "nnz": 1000, "gather_sort": 1}
    got = bench.batch_bytes_per_iteration(csr, A, 0)
    assert got == 2 * (14 * A.nnz + 4 * (2048 + 1)) + 280 * 2048


def test_cpu_baseline_reports_both_legs_and_the_host():
    from paper_2108_10591_amd import workloads as W
    A = W.cd2d(32, 10.0)
    r = bench.cpu_baseline(A, 3, 5)
    assert r["kind"] == "oracle" and r["unit"] == "GB/s" and r["value"] > 0
    assert r["one_core"]["threads"] == 1 and r["one_core"]["iterations"] == 3
    assert r["all_cores"]["iterations"] == 5 and r["cores"] == r["all_cores"]["threads"] >= 1
    assert r["nproc"] == os.cpu_count() and "cpu_model" in r
    assert r["bytes_per_iteration"] == 2 * (12 * A.nnz + 4 * (A.n + 1)) + 288 * A.n
