#!/usr/bin/env python
"""Throughput benchmark of the BCSR 3x3 BiCGStab-ILU0 path on one MI355X.

Default workload: the 100x100x100 grid (1M cells, 7-point stencil, 3x3 FP64
blocks, log-normal permeability with sigma = 2), the size class of the
paper's largest benchmark model.  One step = one block-ILU0 factorisation
from values already in HBM + one BiCGStab solve at a residual reduction of
1e-2 (max 200 iterations), plain FP64; `value` is solves per second.  The
same JSON line also carries, on the same workload: the solve with FP32-stored
ILU0 factors inside the FP64 BiCGStab at the same reduction (`mixed`), both
precisions at a reduction of 1e-6 (`reduction_1e6`), the device time of each
phase from the library's HIP events (`phases`), the achievable device copy
rate measured in the same run (`copy`), a bounded request stream of mixed
sizes with p50/p99 latency (`serving`), and the CPU oracle on the host
(`cpu_baseline`, with the CPU model and core count).

Prints ONE JSON line on stdout (progress goes to stderr).  The roofline
object is for the dominant kernel class: an untimed pre-pass step times
every class and picks the one with the most device time (a preconditioner
application counts as one class: both triangular sweeps).  During the timed
steps the units of that class are timed with HIP events on the solve
stream while the rest of each iteration replays as graph segments.
Algorithmic bytes per unit are the method's minimum (SpMV 76 nnzb + 52 N;
application (9 tb + 4) nnzb + 100 N with tb = 8 for FP64 factors, 4 for
FP32; factorisation 148 nnzb), not counting the work the kernels fuse.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# The paper's only throughput-like figure for this path (Results section): the
# linear solves of the refined NORNE model took 685 s on an AMD MI210 with
# rocSPARSE and 150 Jacobi blocks against 3832 s on one dual-threaded MPI
# process of an AMD EPYC 7763.  Other hardware and another workload: context,
# never a target.
PAPER_CONTEXT = {
    "figure": "5.6x linear-solve speedup (3832 s -> 685 s)",
    "gpu": "AMD MI210, rocSPARSE BiCGStab-ILU0 with 150 Block-Jacobi partitions",
    "cpu": "one dual-threaded MPI process on an AMD EPYC 7763",
    "workload": "NORNE refined (355 407 rows, 2 530 093 3x3 blocks), whole simulation",
    "section": "Results",
}

WORKLOADS = {
    "c1": dict(desc="20x20x10 grid (4000 cells), 7-point, 3x3 FP64 blocks, lognormal sigma=1; "
                    "1 ILU0 factorisation + 1 solve per step", rhs=1, precision="fp64", reduction=1e-2),
    "c2": dict(desc="46x112x22 grid, 85% active cells (96549), 2% non-neighbour connections, 3x3 FP64 "
                    "blocks, lognormal sigma=1; 1 ILU0 factorisation + 10 sequential right-hand sides per step",
               rhs=10, precision="fp64", reduction=1e-2),
    "c3": dict(desc="100x100x100 grid (1M cells), 7-point, 3x3 FP64 blocks, lognormal sigma=2; "
                    "1 ILU0 factorisation + 1 solve per step", rhs=1, precision="fp64", reduction=1e-2),
    "c4": dict(desc="64 same-pattern realisations of a 40x40x30 grid (48000 cells each), lognormal sigma=1; "
                    "1 batched ILU0 factorisation + 1 batched solve of all 64 per step", rhs=1, precision="fp32",
               reduction=1e-2),
    "c5": dict(desc="request stream: Poisson arrivals of single solves, sizes uniform over 10k (25x20x20), "
                    "50k (50x50x20), 200k (100x100x20) and 1M (100x100x100) cells, lognormal sigma=1, 5% of "
                    "requests also carry 2% non-neighbour connections; each request = upload values + ILU0 "
                    "factorisation + 1 solve; FP32 factors in FP64 BiCGStab; HBM budget 200 GB",
               rhs=1, precision="fp32", reduction=1e-2),
}
ORDER = {"natural": 0, "level": 1, "colour": 2, "rcm_level": 3}
PREC = {"fp64": 0, "fp32": 1}
CLASS = {"factor": 0, "lsweep": 1, "usweep": 2, "spmv": 3, "vec": 4, "spmv_t": 5, "gm": 6, "apply": 7}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--ordering", default="colour", choices=sorted(ORDER))
    ap.add_argument("--precision", default=None, choices=sorted(PREC))
    ap.add_argument("--reduction", type=float, default=None)
    ap.add_argument("--roofline", default="auto", choices=["auto", "off"] + sorted(CLASS),
                    help="kernel class of the roofline object (auto: the class with the most device time in a "
                         "profiled pre-pass step)")
    ap.add_argument("--solver", default="bicgstab", choices=["bicgstab", "gmres"],
                    help="Krylov solver on the same factors (gmres: restarted, --restart m)")
    ap.add_argument("--restart", type=int, default=30, help="GMRES restart length (1..32)")
    ap.add_argument("--jacobi", type=int, default=0, metavar="P",
                    help="Block-Jacobi-ILU0 with P transmissibility-weighted partitions (0: plain ILU0)")
    ap.add_argument("--wells", type=int, default=0, metavar="W",
                    help="standard wells kept separate (Algorithm 5): W vertical wells on the workload's grid, "
                         "drawn by synth/wells.py (seed 11); the SpMVs and the true residual subtract them")
    ap.add_argument("--no-extras", action="store_true",
                    help="1M-cell grid: skip the mixed-precision and 1e-6 runs")
    ap.add_argument("--no-serving", action="store_true", help="1M-cell grid: skip the bounded request stream")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="requests of the bounded request stream at half the saturated rate")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-configuration autotuner")
    ap.add_argument("--fuse", type=int, default=1, choices=[0, 1],
                    help="RS_OPT_FUSE_SPMV: the upper launch of the rows without lower blocks also forms their "
                         "rows of the following SpMV (where the pattern allows it)")
    ap.add_argument("--y-input", type=int, default=1, choices=[0, 1],
                    help="RS_OPT_Y_INPUT: the applications read the y of the rows without lower blocks from their "
                         "input and store no y (where the pattern allows it)")
    ap.add_argument("--factor-async", type=int, default=1, choices=[0, 1],
                    help="RS_OPT_FACTOR_ASYNC: each step's ilu0_factor only queues the factorisation (a singular "
                         "pivot shows in the solve's statuses); 0: it waits for it")
    ap.add_argument("--slots", type=int, default=8, help="request stream: concurrent worker slots")
    ap.add_argument("--requests", type=int, default=2000, help="request stream (c5): requests per arrival rate")
    ap.add_argument("--loads", default="0.5,0.8,1.0",
                    help="request stream (c5): arrival rates as fractions of the measured saturated rate")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-sized buffer with torch (a kernel of known traffic, "
                         "used to scale rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args(argv)


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2309_11488_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key, cls):
    """HBM bytes per unit from committed rocprofv3 counter runs, only while the
    kernel source is unchanged since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec.get(f"{key}:{cls}")
    if not ent or ent.get("kernel_digest") != kernel_source_digest():
        return None
    return ent.get("bytes_per_unit")


def host_cpu():
    """CPU model and core counts of the host that runs the oracle."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def method_bytes(n, nnzb, precision):
    """Algorithmic bytes of the method per unit (int32 indices, each vector
    entry read or written once): SpMV, one preconditioner application, the
    factorisation, and one BiCGStab iteration (2 SpMVs, 2 applications and
    the vector updates, 408 N)."""
    tb = 8 if precision == "fp64" else 4
    spmv = 76 * nnzb + 52 * n
    apply = (9 * tb + 4) * nnzb + 100 * n
    return {"spmv": spmv, "apply": apply, "factor": 148 * nnzb, "iteration": 2 * spmv + 2 * apply + 408 * n}


def cpu_baseline(s, rhs, ordering, precision, reduction, budget_s, part=None, restart=0):
    """The oracle as it stands, single-threaded, on whole steps of the same workload."""
    import numpy as np

    import oracle
    prec = oracle.PREC_ILU_F64 if precision == "fp64" else oracle.PREC_ILU_F32
    t0 = time.perf_counter()
    solves = 0
    while True:
        for sysk in range(s.batch):
            if part is None:
                perm = oracle.ordering_perm(s.rowptr, s.colidx, ordering)
                prow, pcol, pv = oracle.permute(s.rowptr, s.colidx, s.vals[sysk], perm)
                mrow, mcol, mv = prow, pcol, pv
            else:        # Block-Jacobi: ordering and ILU0 on the Jacobi matrix
                jrow, jcol, jv = oracle.jacobi_matrix(s.rowptr, s.colidx, s.vals[sysk], part)
                perm = oracle.ordering_perm(jrow, jcol, ordering)
                prow, pcol, pv = oracle.permute(s.rowptr, s.colidx, s.vals[sysk], perm)
                mrow, mcol, mv = oracle.permute(jrow, jcol, jv, perm)
            st, _, lu, dinv = oracle.ilu0(mrow, mcol, mv)
            for j in range(rhs):
                if restart:
                    x, info = oracle.gmres(prow, pcol, pv, lu, dinv, s.b[sysk, j][perm], precond=prec,
                                           restart=restart, reduction=reduction)
                else:
                    x, info = oracle.bicgstab(prow, pcol, pv, lu, dinv, s.b[sysk, j][perm], precond=prec,
                                              reduction=reduction, mrow=mrow, mcol=mcol)
                xo = np.empty_like(x)
                xo[perm] = x
                solves += 1
            if time.perf_counter() - t0 > budget_s:
                break
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return solves / dt, solves, dt


def copy_rate(torch, dev, mib=2048, reps=5):
    """Achievable device copy rate: a torch copy of a `mib` MiB FP64 buffer,
    (bytes read + bytes written) / kernel time, best of `reps` after one
    untimed copy."""
    src = torch.ones(mib << 17, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    byts = 2 * src.numel() * 8
    del src, dst
    torch.cuda.empty_cache()
    return {"gbs": byts / (best / 1e3) / 1e9, "bytes": byts, "ms": best,
            "what": f"torch copy of a {mib} MiB FP64 buffer, read + written bytes / kernel time, best of {reps}"}


class Problem:
    """One workload on the device: the caller's matrix handle and the
    right-hand sides; preconditioner handles per precision share one
    analysis and keep their own factors, tuned options and graphs."""

    def __init__(self, args, s, rhs, ordering, part):
        import numpy as np
        import torch

        import paper_2309_11488_amd as rs
        self.rs, self.np, self.torch = rs, np, torch
        self.args, self.s, self.rhs, self.ordering, self.part = args, s, rhs, ordering, part
        dev = torch.device("cuda:0")
        rowptr = torch.from_numpy(s.rowptr).to(dev)
        colidx = torch.from_numpy(s.colidx).to(dev)
        vals = torch.from_numpy(s.vals).to(dev)
        self.b = torch.from_numpy(np.ascontiguousarray(s.b.transpose(1, 0, 2, 3))).to(dev)  # (rhs, batch, n, 3)
        self.x = torch.zeros_like(self.b)
        self.A = rs.bcsr_create(rowptr, colidx, vals)
        # value upload from host memory (PCIe-inclusive, the paper's copy_to_GPU), timed apart
        hv = np.ascontiguousarray(s.vals)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rs.bcsr_set_values(self.A, hv)
        torch.cuda.synchronize()
        self.upload_ms = (time.perf_counter() - t) * 1e3
        self.n_perf = 0
        if args.wells:
            from synth import make_wells
            w = make_wells(s, args.wells, seed=11, batch=s.batch)
            rs.bcsr_set_wells(self.A, w.well_ptr, w.perf_row, w.B, w.C, w.Dinv)
            self.n_perf = w.n_perf
        self.handles = {}
        t = time.perf_counter()
        self.base = self._analyse()
        self.analyse_ms = (time.perf_counter() - t) * 1e3
        self.nl, self.nu = rs.ilu0_get_sweep_levels(self.base)
        _, self.n_sets, _ = rs.ilu0_get_schedule(self.base, s.n)
        self.fused_rows = rs.ilu0_get_option(self.base, rs.OPT_FUSED_ROWS)
        self.y_input_pattern = rs.ilu0_get_option(self.base, rs.OPT_Y_INPUT_PATTERN)

    def _analyse(self):
        rs = self.rs
        if self.part is not None:
            return rs.ilu0_analyse_jacobi(self.A, self.ordering, self.part)
        return rs.ilu0_analyse(self.A, self.ordering)

    def handle(self, precision, reduction):
        """Factored, autotuned preconditioner handle for `precision`."""
        rs = self.rs
        if precision in self.handles:
            return self.handles[precision]
        M = self.base if not self.handles else rs.ilu0_analyse_shared(self.A, self.base)
        st, bad = rs.ilu0_factor(M, self.A, PREC[precision])
        assert st == rs.OK, (st, bad)
        rs.ilu0_set_option(M, rs.OPT_FUSE_SPMV, self.args.fuse)
        rs.ilu0_set_option(M, rs.OPT_Y_INPUT, self.args.y_input)
        # the first factorisation above waited and was checked; the steps' own are queued
        rs.ilu0_set_option(M, rs.OPT_FACTOR_ASYNC, self.args.factor_async)
        tune = None
        if not self.args.no_tune:
            t = time.perf_counter()
            tune = rs.ilu0_autotune(M, self.A, self.b[0], reduction, reps=3)
            log(f"autotune {precision}: {tune} in {time.perf_counter() - t:.2f}s")
        self.handles[precision] = (M, tune)
        return self.handles[precision]

    def close(self):
        for M, _ in self.handles.values():
            self.rs.ilu0_destroy(M)
        if self.base is not None and not self.handles:
            self.rs.ilu0_destroy(self.base)
        self.handles = {}
        self.base = None
        self.rs.bcsr_destroy(self.A)


def measure(P, precision, reduction, steps, warmup, roofline="auto", key=None, label=""):
    """Time `steps` steps (one factorisation + the right-hand sides) after
    `warmup` untimed ones; returns solves/s, iteration counts, residuals,
    phase times from the library's events and (unless roofline is "off") the
    roofline object of the timed kernel class."""
    rs, np, torch = P.rs, P.np, P.torch
    args, s, rhs = P.args, P.s, P.rhs
    gmres = args.solver == "gmres"
    M, tune = P.handle(precision, reduction)
    prec = PREC[precision]
    rec = {"half": [], "res": [], "status": [], "factor_ms": [], "solve_ms": []}
    # when a solve class is timed, one solve in every `period` records its
    # events: two of the timed steps' solves (the sampled solves launch
    # eagerly, with events between kernels)
    period = max((steps * rhs + 1) // 2, 1)
    sample = {"mask": 0, "count": 0}

    def solve(j):
        if gmres:
            return rs.gmres_solve(M, P.A, P.b[j], P.x[j], args.restart, reduction, 200)
        return rs.bicgstab_solve(M, P.A, P.b[j], P.x[j], reduction, 200)

    def step(record=False):
        if sample["mask"]:
            rs.rsolve_profile_set_mask(sample["mask"])      # every factorisation
        st, bad = rs.ilu0_factor(M, P.A, prec)
        assert st == rs.OK, (st, bad)
        for j in range(rhs):
            if sample["mask"]:
                rs.rsolve_profile_set_mask(sample["mask"] if sample["count"] % period == 0 else 0)
                sample["count"] += 1
            _, st, info = solve(j)
            if record:
                for i in info:
                    rec["half"].append(i["half_steps"])
                    rec["res"].append(i["true_rel_residual"])
                    rec["status"].append(i["status"])
                    rec["solve_ms"].append(i["solve_ms"])
                rec["factor_ms"].append(info[0]["factor_ms"])

    for _ in range(warmup):
        step()
    class_times, dominant, chosen = {}, None, None
    if roofline != "off":
        # pre-pass (untimed): one step with every kernel class timed
        classes = ["factor", "lsweep", "usweep", "spmv", "spmv_t", "vec"] + (["gm"] if gmres else [])
        rs.rsolve_profile_enable(sum(1 << CLASS[c] for c in classes))
        step()
        torch.cuda.synchronize()
        for c in classes:
            ms, units, byts = rs.rsolve_profile_get(CLASS[c])
            if units:
                class_times[c] = {"ms": ms, "units": units, "us_per_unit": ms * 1e3 / units,
                                  "gbs": byts / (ms / 1e3) / 1e9 if ms > 0 else None}
        if "lsweep" in class_times and "usweep" in class_times:
            # one application = one lower and one upper sweep
            lo, up = class_times["lsweep"], class_times["usweep"]
            ms = lo["ms"] + up["ms"]
            byts = lo["gbs"] * 1e9 * lo["ms"] / 1e3 + up["gbs"] * 1e9 * up["ms"] / 1e3
            class_times["apply"] = {"ms": ms, "units": lo["units"], "us_per_unit": ms * 1e3 / lo["units"],
                                    "gbs": byts / (ms / 1e3) / 1e9, "note": "lower + upper sweep"}
        main = [c for c in class_times if c not in ("lsweep", "usweep")]
        total_ms = sum(class_times[c]["ms"] for c in main)
        for c, v in class_times.items():
            v["share"] = v["ms"] / total_ms if total_ms else None
        dominant = max(main, key=lambda c: class_times[c]["ms"])
        log(f"{label} pre-pass device time per class: " + ", ".join(
            f"{c} {v['share'] * 100:.1f}% ({v['us_per_unit']:.2f} us/unit, {v['gbs'] or 0:.0f} GB/s)"
            for c, v in sorted(class_times.items(), key=lambda kv: -kv[1]["ms"])))
        chosen = dominant if roofline == "auto" else roofline
        # the timed class's units record events between graph segments,
        # which one more warm-up step captures
        tmask = 1 << CLASS[chosen]
        sample.update(mask=tmask, count=0)
        rs.rsolve_profile_enable(tmask)
        step()
        torch.cuda.synchronize()
        rs.rsolve_profile_enable(tmask)
        sample["count"] = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(record=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    roof = None
    if chosen:
        ms, units, byts = rs.rsolve_profile_get(CLASS[chosen])
        rs.rsolve_profile_enable(0)
        sample.update(mask=0, count=0)
        per_unit_bytes = byts / max(units, 1)
        per_unit_s = ms / 1e3 / max(units, 1)
        achieved = per_unit_bytes / per_unit_s / 1e9 if units else None
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": measured_traffic(key, chosen) if key else None,
                "kernel": chosen, "units_timed": units, "us_per_unit": per_unit_s * 1e6,
                "algorithmic_bytes_per_unit": per_unit_bytes, "dominant_in_prepass": dominant,
                "sampling": f"every factorisation; for the solve classes one solve in every {period}"}
        log(f"{label} roofline {chosen}: {units} units, {per_unit_s * 1e6:.2f} us/unit, "
            f"{per_unit_bytes / 1e6:.2f} MB/unit -> {achieved or 0:.1f} GB/s")
    n_solves = steps * rhs * s.batch
    value = n_solves / elapsed
    fms = float(np.median(rec["factor_ms"]))
    sms = float(np.median(rec["solve_ms"]))
    out = {"solves_per_s": value, "ms_per_step": elapsed / steps * 1e3, "steps": steps, "precision": precision,
           "reduction": reduction, "mean_half_steps": float(np.mean(rec["half"])),
           "max_true_rel_residual": float(max(rec["res"])), "statuses": sorted(set(rec["status"])),
           "phases": {"factor_ms": fms, "solve_ms": sms,
                      "solves_per_s_without_factor": s.batch * 1e3 / sms if sms > 0 else None,
                      "source": "median over the timed steps of the library's HIP-event times "
                                "(solve_info.factor_ms, solve_info.solve_ms)"},
           "launch_config": tune, "roofline": roof, "kernel_classes": class_times or None}
    log(f"{label}: {n_solves} solves in {elapsed:.3f}s: {value:.1f} solves/s; half steps mean "
        f"{out['mean_half_steps']:.2f}; max true residual {out['max_true_rel_residual']:.3e}; statuses "
        f"{out['statuses']}; device factor {fms:.3f} ms, solve {sms:.3f} ms")
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py measures one GPU only: the solver runs on a single MI355X "
                                   "(a system or request per GPU is how it would spread); run it with --gpus 1"}),
              flush=True)
        sys.exit(2)

    if args.workload == "c5":
        serve_main(args)
        return

    import numpy as np
    import torch

    import paper_2309_11488_amd as rs
    from synth import config_system

    wl = WORKLOADS[args.workload]
    gmres = args.solver == "gmres"
    if gmres and args.jacobi:
        sys.exit("bench.py: --solver gmres runs on the plain ILU0 preconditioner only")
    precision = args.precision or wl["precision"]
    reduction = args.reduction if args.reduction is not None else wl["reduction"]
    ordering = ORDER[args.ordering]
    rhs = wl["rhs"]
    t = time.perf_counter()
    s = config_system(args.workload, seed=0)
    log(f"workload {args.workload}: n={s.n} nnzb={s.nnzb} batch={s.batch} rhs={rhs} "
        f"(generated in {time.perf_counter() - t:.1f}s)")
    part = None
    if args.jacobi > 0:
        part = rs.bcsr_partition(s.rowptr, s.colidx, args.jacobi, weights=s.trans)
    P = Problem(args, s, rhs, ordering, part)
    log(f"ordering {args.ordering}: {P.n_sets} sets, sweep levels lower {P.nl} upper {P.nu}; analysis "
        f"{P.analyse_ms:.1f} ms; value upload from host {P.upload_ms:.2f} ms")
    # key of the committed counter runs (profiles/traffic.json) for this configuration
    key = f"c3_{precision}" if args.workload == "c3" else args.workload
    if args.jacobi or gmres or args.ordering != "colour" or args.wells:
        key = None
    head = measure(P, precision, reduction, args.steps, args.warmup, args.roofline, key=key, label=precision)
    extras = args.workload == "c3" and not args.no_extras and not gmres and args.precision is None \
        and args.reduction is None and not args.wells
    mixed = red6 = None
    if extras:
        # the same workload with FP32-stored factors at the same reduction,
        # then both precisions at a reduction of 1e-6
        mixed = measure(P, "fp32", reduction, args.steps, args.warmup, args.roofline, key="c3_fp32",
                        label="fp32 factors")
        mixed["speedup_vs_fp64"] = mixed["solves_per_s"] / head["solves_per_s"]
        red6 = {}
        for pr in ("fp64", "fp32"):
            red6["fp64" if pr == "fp64" else "mixed"] = measure(P, pr, 1e-6, max(5, args.steps // 2), 1, "off",
                                                                label=f"{pr} at 1e-6")
        red6["mixed"]["speedup_vs_fp64"] = red6["mixed"]["solves_per_s"] / red6["fp64"]["solves_per_s"]
    P.close()
    torch.cuda.synchronize()
    copy = copy_rate(torch, torch.device("cuda:0"))
    log(f"copy: {copy['gbs']:.0f} GB/s")
    serving = None
    if args.workload == "c3" and not args.no_serving:
        serving = serve(args, requests=args.serve_requests, loads=[0.5], burst=100,
                        plain_seeds={10_000: 2, 50_000: 2, 200_000: 1, 1_000_000: 1}, cpu=False)
    cpu = None
    if args.wells and not args.no_cpu:
        log("cpu oracle: not timed with wells (the baseline leg times the plain oracle solve)")
    elif not args.no_cpu:
        v, nsol, dt = cpu_baseline(s, rhs, ordering, precision, reduction, args.cpu_seconds, part,
                                   args.restart if gmres else 0)
        hc = host_cpu()
        cpu = {"value": v, "unit": "solves/s", "cores": 1, "kind": "oracle", "cpu_model": hc["model"],
               "nproc": hc["nproc"], "usable_cpus": hc["usable_cpus"],
               "sample": f"{nsol} solves of the same workload (ordering, reordered copy, ILU0 per step, "
                         f"then {'GMRES' if gmres else 'BiCGStab'} per right-hand side) in {dt:.1f}s, "
                         f"single-threaded C oracle, {precision} factors"}
        log(f"cpu oracle: {v:.3f} solves/s ({nsol} solves in {dt:.1f}s) on {hc}")
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 17, dtype=torch.float64, device=torch.device("cuda:0"))
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy} MiB read + {args.calibrate_copy} MiB written, 3 times")
    mb = method_bytes(s.n, s.nnzb, precision)
    it_gb = mb["iteration"] * head["mean_half_steps"] / 2 / 1e9
    out = {
        "metric": (f"GMRES({args.restart})-ILU0" if gmres else "BiCGStab-ILU0") +
                  " solves/sec at 1e-2 reduction, HBM GB/s vs roofline, p50/p99 latency of a request stream",
        "value": head["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if precision == "fp64" else "f64+f32-factors", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "ordering": args.ordering,
                   "precision": precision,
                   "solver": f"gmres({args.restart})" if gmres else "bicgstab",
                   "reduction": reduction, "max_iter": 200, "n_brows": s.n, "nnzb": s.nnzb, "batch": s.batch,
                   "rhs_per_step": rhs, "sets": P.n_sets, "sweep_levels": [P.nl, P.nu],
                   "fuse_spmv": args.fuse, "fused_rows": P.fused_rows,
                   "y_input": args.y_input, "y_input_pattern": P.y_input_pattern,
                   "factor_async": args.factor_async,
                   "jacobi_partitions": args.jacobi or None,
                   "wells": args.wells or None, "perforations": P.n_perf or None,
                   "mean_half_steps": head["mean_half_steps"],
                   "max_true_rel_residual": head["max_true_rel_residual"], "statuses": head["statuses"],
                   "launch_config": head["launch_config"],
                   "method_bytes": mb,
                   "whole_solve_gbs": (it_gb * s.batch * rhs) / (head["phases"]["solve_ms"] / 1e3)
                   if head["phases"]["solve_ms"] else None},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "phases": dict(head["phases"], upload_ms=P.upload_ms, analyse_ms=P.analyse_ms,
                       upload_note="values copied from host memory with bcsr_set_values (PCIe), "
                                   "outside the timed region"),
        "copy": copy,
        "mixed": mixed,
        "reduction_1e6": red6,
        "serving": serving,
        "kernel_classes": head["kernel_classes"],
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(out), flush=True)


# ----------------------------------------------------------------- serving

def solve_bytes(n, nnzb, half_steps, precision):
    """Algorithmic HBM bytes of one request (approximate): value upload
    (device copy), the factorisation's minimum, BiCGStab half-steps and the
    true-residual SpMV."""
    mb = method_bytes(n, nnzb, "fp64" if precision == "fp64" else "fp32")
    upload = 144 * nnzb
    return upload + mb["factor"] + half_steps * mb["iteration"] / 2 + mb["spmv"]


def serve(args, requests, loads, burst, plain_seeds, cpu):
    """Request stream: a warm-up that meets every pattern, a saturated burst,
    then Poisson arrivals at fractions of the saturated rate; p50 / p99
    latency from arrival to result.  Returns a dict."""
    import threading

    import numpy as np
    import torch

    import paper_2309_11488_amd as rs
    from synth import make_grid_system, serving_classes

    wl = WORKLOADS["c5"]
    precision = "fp32"
    reduction = 1e-2
    ordering = ORDER[args.ordering]
    dev = torch.device("cuda:0")
    classes = serving_classes()
    # per class: plain realisations (one pattern per class) and one with NNCs
    pool = {}
    t = time.perf_counter()
    for cells, shape in classes.items():
        sysl = []
        for k in range(plain_seeds[cells]):
            sysl.append(make_grid_system(*shape, seed=1000 + 10 * k, n_rhs=2))
        nnc = make_grid_system(*shape, nnc_frac=0.02, seed=7777, n_rhs=2)
        pool[cells] = (sysl, nnc)
        log(f"class {cells}: n={sysl[0].n} nnzb={sysl[0].nnzb} (+NNC nnzb={nnc.nnzb}); "
            f"{time.perf_counter() - t:.1f}s")

    def on_device(s):
        return (torch.from_numpy(s.vals[0]).to(dev), torch.from_numpy(np.ascontiguousarray(s.b[0])).to(dev))

    budget = 200 * 10**9
    srv = rs.Server(hbm_budget_bytes=budget, max_slots=args.slots, ordering=ordering, precision=PREC[precision],
                    autotune=not args.no_tune)
    entries = {}      # cells -> ([(pattern, s, vals_d, b_d)], nnc entry)
    for cells, (sysl, nnc) in pool.items():
        p = srv.add_pattern(sysl[0].rowptr, sysl[0].colidx)
        plain = [(p, s) + on_device(s) for s in sysl]
        q = srv.add_pattern(nnc.rowptr, nnc.colidx)
        entries[cells] = (plain, (q, nnc) + on_device(nnc))
    torch.cuda.synchronize()
    sizes = sorted(entries)

    def draw(rng, count):
        out = []
        for _ in range(count):
            cells = sizes[int(rng.integers(0, len(sizes)))]
            plain, nnc = entries[cells]
            e = nnc if rng.random() < 0.05 else plain[int(rng.integers(0, len(plain)))]
            out.append((cells, e, int(rng.integers(0, 2))))
        return out

    def run_stream(reqs, rate):
        """Submit at Poisson times (rate None: all at once); returns per-request records and the makespan."""
        rng = np.random.default_rng(12345)
        gaps = rng.exponential(1.0 / rate, len(reqs)) if rate else np.zeros(len(reqs))
        arrivals = np.cumsum(gaps) - gaps[0]
        done = []
        tickets = []
        lock = threading.Condition()

        def collector():
            k = 0
            while True:
                with lock:
                    while k >= len(tickets):
                        lock.wait()
                    item = tickets[k]
                    tickets[k] = 0           # drop the result buffer once collected
                if item is None:
                    return
                ticket, t_arr, t_sub, cells, e, _ = item
                _, st, info, tm = srv.wait(ticket)
                # latency from the scheduled arrival: submission lag + submission to completion
                t_end = t_sub + tm["total_ms"] / 1e3
                done.append(dict(cells=cells, n=e[1].n, nnzb=e[1].nnzb, status=st, half=info["half_steps"],
                                 res=info["true_rel_residual"], lat_ms=(t_end - t_arr) * 1e3, t_end=t_end,
                                 resident=tm["resident"], queue_ms=tm["queue_ms"], solve_ms=tm["solve_ms"],
                                 factor_ms=tm["factor_ms"], dev_solve_ms=info["solve_ms"],
                                 dev_factor_ms=info["factor_ms"]))
                k += 1

        th = threading.Thread(target=collector)
        th.start()
        t0 = time.perf_counter()
        for (cells, e, j), a in zip(reqs, arrivals):
            now = time.perf_counter() - t0
            if a > now:
                time.sleep(a - now)
            pid, s, vals_d, b_d = e
            x = torch.empty_like(b_d[j])
            t_sub = time.perf_counter()
            ticket = srv.submit(pid, vals_d, b_d[j], x, reduction=reduction)
            with lock:
                tickets.append((ticket, t0 + a, t_sub, cells, e, x))
                lock.notify()
        with lock:
            tickets.append(None)
            lock.notify()
        th.join()
        makespan = max(d["t_end"] for d in done) - t0
        return done, makespan

    def summarise(done, makespan, offered=None):
        lat = np.array([d["lat_ms"] for d in done])
        byts = sum(solve_bytes(d["n"], d["nnzb"], d["half"], precision) for d in done)
        per_class = {}
        for c in sizes:
            lc = np.array([d["lat_ms"] for d in done if d["cells"] == c])
            if len(lc):
                per_class[str(c)] = {"count": int(len(lc)), "p50_ms": float(np.percentile(lc, 50)),
                                     "p99_ms": float(np.percentile(lc, 99))}
        return {"offered_per_s": offered, "solves_per_s": len(done) / makespan, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "makespan_s": makespan, "requests": len(done),
                "hbm_gbs": byts / makespan / 1e9, "statuses": sorted({d["status"] for d in done}),
                "max_true_rel_residual": max(d["res"] for d in done),
                "mean_half_steps": float(np.mean([d["half"] for d in done])), "per_class": per_class}

    rng = np.random.default_rng(2024)
    t = time.perf_counter()
    # the warm-up meets every pattern (each size with and without NNCs), so
    # the measured phases see a server whose analyses are all done, as in
    # steady serving; analysis is a once-per-pattern cost
    every = [(c, entries[c][1], 0) for c in sizes] + [(c, entries[c][0][0], 0) for c in sizes]
    warm, wspan = run_stream(every + draw(rng, max(4 * args.slots * len(sizes), 100)), None)
    W = summarise(warm, wspan)
    log(f"warm-up: {len(warm)} requests in {time.perf_counter() - t:.1f}s, statuses {W['statuses']}, max true "
        f"residual {W['max_true_rel_residual']:.3e}; stats {srv.stats()}")
    recs, span = run_stream(draw(rng, burst), None)
    sat = summarise(recs, span)
    log(f"saturated burst: {sat['requests']} requests, {sat['solves_per_s']:.1f} solves/s, "
        f"{sat['hbm_gbs']:.0f} GB/s algorithmic, statuses {sat['statuses']}, max true residual "
        f"{sat['max_true_rel_residual']:.3e}")
    by_load = {}
    for f in loads:
        rate = f * sat["solves_per_s"]
        recs, span = run_stream(draw(rng, requests), rate)
        by_load[f"{f:g}"] = summarise(recs, span, offered=rate)
        L = by_load[f"{f:g}"]
        log(f"load {f:g} ({rate:.1f}/s offered): {L['solves_per_s']:.1f} solves/s, p50 {L['p50_ms']:.2f} ms, "
            f"p99 {L['p99_ms']:.2f} ms, statuses {L['statuses']}, max true residual "
            f"{L['max_true_rel_residual']:.3e}")
    stats = srv.stats()
    srv.close()
    log(f"server stats {stats}")

    cpu_rec = None
    if cpu and not args.no_cpu:
        import oracle
        prec = oracle.PREC_ILU_F32
        sample = draw(np.random.default_rng(99), 64)
        t0 = time.perf_counter()
        nsol = 0
        for cells, e, j in sample:
            s = e[1]
            oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, j], ordering=ordering, reduction=reduction,
                         precond=prec)
            nsol += 1
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        hc = host_cpu()
        cpu_rec = {"value": nsol / dt, "unit": "solves/s", "cores": 1, "kind": "oracle", "cpu_model": hc["model"],
                   "nproc": hc["nproc"], "usable_cpus": hc["usable_cpus"],
                   "sample": f"the first {nsol} requests of a seeded draw from the same mix, one after another "
                             f"(ordering, ILU0, BiCGStab, true residual), in {dt:.1f}s, single-threaded C oracle"}
        log(f"cpu oracle: {nsol / dt:.3f} solves/s ({nsol} requests in {dt:.1f}s)")

    top = by_load[f"{loads[0]:g}"] if loads else sat
    return {"workload": f"c5: {wl['desc']}", "slots": args.slots, "hbm_budget_bytes": budget,
            "pool": {str(c): {"n": entries[c][0][0][1].n, "nnzb": entries[c][0][0][1].nnzb,
                              "realisations": len(entries[c][0])} for c in sizes},
            "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"], "load_of_p50_p99": loads[0] if loads else None,
            "saturated": sat, "loads": by_load, "warmup_requests": len(warm), "server_stats": stats,
            "cpu_baseline": cpu_rec}


def serve_main(args):
    """The full request-stream study (--workload c5): one JSON line."""
    loads = [float(v) for v in args.loads.split(",") if v]
    r = serve(args, requests=args.requests, loads=loads, burst=max(args.requests // 4, 50),
              plain_seeds={10_000: 4, 50_000: 4, 200_000: 3, 1_000_000: 2}, cpu=True)
    sat = r["saturated"]
    top = r["loads"].get("1", sat)
    out = {
        "metric": "BiCGStab-ILU0 solves/sec with p50/p99 latency at 1e-2 reduction (request stream)",
        "value": sat["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": sat["requests"],
        "warmup": r["warmup_requests"], "ms_per_step": 1e3 / sat["solves_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32-factors", "data": "synthetic",
        "config": {"workload": r["workload"], "ordering": args.ordering, "precision": "fp32", "reduction": 1e-2,
                   "slots": args.slots, "hbm_budget_bytes": r["hbm_budget_bytes"],
                   "requests_per_load": args.requests, "pool": r["pool"], "p50_ms": top["p50_ms"],
                   "p99_ms": top["p99_ms"], "saturated": sat, "loads": r["loads"],
                   "server_stats": r["server_stats"]},
        "roofline": {"bound": "hbm", "achieved": sat["hbm_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": sat["hbm_gbs"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole request stream: algorithmic bytes of upload, factorisation, BiCGStab "
                               "half-steps and true residual per request over the burst makespan"},
        "cpu_baseline": r["cpu_baseline"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
