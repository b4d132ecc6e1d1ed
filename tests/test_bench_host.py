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
    assert {"c2:lsweep", "c3:spmv", "c4:factor"} <= set(rec)
    key = "c2:lsweep"
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: rec[key]["kernel_digest"])
    assert bench.measured_traffic("c2", "lsweep") == rec[key]["bytes_per_unit"] > 0
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 16)
    assert bench.measured_traffic("c2", "lsweep") is None


@pytest.mark.parametrize("workload", ["c1", "c2", "c3", "c4", "c5"])
def test_workload_descriptions(workload):
    sys.path.insert(0, ROOT)
    import bench
    assert workload in bench.WORKLOADS and bench.WORKLOADS[workload]["desc"]


def test_rcm_renumbering_is_a_similarity():
    """bench.py --pre rcm hands the solver P A P^T and P b (P from reverse
    Cuthill-McKee): products with the renumbered matrix are the original's,
    renumbered."""
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    sys.path.insert(0, ROOT)
    import bench
    import oracle
    from synth import make_grid_system

    s = make_grid_system(9, 8, 6, active_frac=0.9, nnc_frac=0.03, seed=21, n_rhs=2)
    r = bench.rcm_renumbered(s)
    perm = reverse_cuthill_mckee(sp.csr_matrix((np.ones(s.nnzb), s.colidx, s.rowptr), shape=(s.n, s.n)),
                                 symmetric_mode=True)
    assert r.nnzb == s.nnzb and np.all(np.diff(r.rowptr) >= 1)
    for i in range(r.n):
        row = r.colidx[r.rowptr[i]:r.rowptr[i + 1]]
        assert np.all(np.diff(row) > 0)
    x = np.random.default_rng(22).standard_normal((s.n, 3))
    y = oracle.spmv(s.rowptr, s.colidx, s.vals[0], x)
    y2 = oracle.spmv(r.rowptr, r.colidx, r.vals[0], x[perm])
    assert np.allclose(y2, y[perm], rtol=1e-13, atol=1e-12)
    assert np.array_equal(r.b, s.b[:, :, perm])
