"""bench.py's host-side contract: one GPU only, and its byte models."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_traffic_is_reported_only_for_the_measured_kernels(monkeypatch):
    """bench.py reports the committed HBM traffic of a kernel class only
    while the kernel sources carry the digest the counters were taken with."""
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    assert rec
    for key, ent in rec.items():
        wl, cls = key.split(":")
        monkeypatch.setattr(bench, "kernel_source_digest", lambda: ent["kernel_digest"])
        assert bench.measured_traffic(wl, cls) == ent["bytes_per_unit"] > 0
        monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 16)
        assert bench.measured_traffic(wl, cls) is None


def test_method_bytes_follow_the_byte_model():
    """The algorithmic bytes bench.py divides by time: SpMV 76 nnzb + 52 N,
    application 76 nnzb + 100 N (FP64 factors) or 40 nnzb + 100 N (FP32),
    one iteration 304 nnzb + 712 N resp. 232 nnzb + 712 N, factorisation
    148 nnzb."""
    sys.path.insert(0, ROOT)
    import bench
    n, nnzb = 1_000_000, 6_940_000
    m = bench.method_bytes(n, nnzb, "fp64")
    assert m["spmv"] == 76 * nnzb + 52 * n and m["apply"] == 76 * nnzb + 100 * n and m["factor"] == 148 * nnzb
    assert m["iteration"] == 304 * nnzb + 712 * n
    m = bench.method_bytes(n, nnzb, "fp32")
    assert m["apply"] == 40 * nnzb + 100 * n and m["iteration"] == 232 * nnzb + 712 * n


def test_default_run_is_the_large_grid_in_fp64():
    """With no flags bench.py measures the 100^3 grid with plain FP64 factors
    at a reduction of 1e-2 (the mixed-precision and 1e-6 runs ride along)."""
    sys.path.insert(0, ROOT)
    import bench
    a = bench.parse([])
    assert a.workload == "c3" and a.precision is None and a.reduction is None and a.steps == 20
    wl = bench.WORKLOADS["c3"]
    assert wl["precision"] == "fp64" and wl["reduction"] == 1e-2 and "100x100x100" in wl["desc"]


def test_host_cpu_is_described():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and h["usable_cpus"] >= 1


@pytest.mark.parametrize("workload", ["c1", "c2", "c3", "c4", "c5"])
def test_workload_descriptions(workload):
    sys.path.insert(0, ROOT)
    import bench
    assert workload in bench.WORKLOADS and bench.WORKLOADS[workload]["desc"]
