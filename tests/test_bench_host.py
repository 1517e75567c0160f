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
                           (2, ("spmv", "update", "spmv_fused"))):
        per_launch = sum(bench.bytes_per_launch(c, n, nnz, sched) for c in classes)
        for variant in ("pbicgsafe", "pbicgsafe_rr"):
            assert bench.bytes_per_iteration(variant, n, nnz, sched) == per_launch, (sched, variant)
    # the fused schedules skip the 40n pass: 8n (schedule 1) and 32n (schedule 2) fewer bytes
    b0, b1, b2 = (bench.bytes_per_iteration("pbicgsafe", n, nnz, s) for s in (0, 1, 2))
    assert b0 - b1 == 8 * n and b0 - b2 == 32 * n
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


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
