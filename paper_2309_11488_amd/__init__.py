"""Python binding of librsolve.so: BCSR (3x3 FP64 blocks) BiCGStab with block-ILU0 on MI355X.

Argument marshalling only: every step of the solver runs in the HIP library.
The functions carry the C names (``bcsr_create``, ``ilu0_analyse``,
``ilu0_factor``, ``bicgstab_solve`` ...).  Arrays may be NumPy arrays (host
memory) or torch CUDA tensors (device memory; PyTorch supplies memory and the
current stream only).  There is no CPU fallback: when the library is missing
the import of a function fails loudly.
"""

from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsolve.so")

OK, NOT_CONVERGED, BREAKDOWN, PENDING = 0, 1, 2, 3
INVALID_ARG, UNSUPPORTED_BLOCK_SIZE, BAD_PATTERN, MISSING_DIAGONAL = -1, -2, -3, -4
ZERO_PIVOT, NON_FINITE, OUT_OF_MEMORY, HIP_ERROR, PATTERN_MISMATCH, NOT_FACTORED = -5, -6, -7, -8, -9, -10
ORDER_NATURAL, ORDER_LEVEL_SET, ORDER_GRAPH_COLOUR, ORDER_RCM_LEVEL_SET = 0, 1, 2, 3
PREC_FP64, PREC_FP32_FACTORS = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
OPT_SWEEP_TILES, OPT_SWEEP_GRID, OPT_POLL_CHUNK, OPT_USE_GRAPH, OPT_PREDICT_POLL = 0, 1, 2, 3, 4
OPT_SPMV_VARIANT, OPT_SWEEP_VARIANT, OPT_REDUCE_SPLIT, OPT_SPIN_LIMIT, OPT_FUSE_SPMV, OPT_FUSED_ROWS = 5, 6, 7, 8, 9, 10
OPT_Y_INPUT, OPT_Y_INPUT_PATTERN, OPT_FACTOR_ASYNC, OPT_LOWER_PARTS = 11, 12, 13, 14
N_ROW_VARIANTS = 9

EXPORTS = (
    "bcsr_create", "bcsr_set_values", "bcsr_set_wells", "bcsr_get_dims", "bcsr_spmv", "bcsr_set_option", "bcsr_destroy", "ilu0_analyse",
    "ilu0_get_schedule", "ilu0_get_sweep_levels", "ilu0_set_option", "ilu0_get_option", "ilu0_autotune",
    "ilu0_factor", "ilu0_factor_status", "ilu0_get_factors", "ilu0_apply", "ilu0_apply_noalloc",
    "bicgstab_solve", "gmres_solve", "ilu0_destroy", "ilu0_analyse_host", "rsolve_profile_enable", "rsolve_profile_set_mask", "rsolve_profile_get",
    "ilu0_analyse_shared", "ilu0_analyse_jacobi", "bcsr_partition", "server_create", "server_request_bytes", "server_analysis_bytes", "server_add_pattern",
    "server_submit", "server_poll", "server_wait", "server_get_stats",
    "server_destroy", "rsolve_status_string", "rsolve_last_error",
)
PROF_FACTOR, PROF_LSWEEP, PROF_USWEEP, PROF_SPMV_V, PROF_VEC, PROF_SPMV_T, PROF_GM, PROF_APPLY = 0, 1, 2, 3, 4, 5, 6, 7
GMRES_MAX_RESTART = 32


class SolveInfo(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("half_steps", ct.c_int32), ("r0_norm", ct.c_double),
                ("final_norm", ct.c_double), ("true_rel_residual", ct.c_double), ("factor_ms", ct.c_double),
                ("solve_ms", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneResult(ct.Structure):
    _fields_ = [("spmv_variant", ct.c_int32), ("sweep_variant", ct.c_int32), ("sweep_tiles", ct.c_int32),
                ("sweep_grid", ct.c_int32), ("us_per_solve", ct.c_double), ("candidates", ct.c_int32),
                ("from_cache", ct.c_int32), ("reduce_split", ct.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(ct.Structure):
    _fields_ = [("hbm_budget_bytes", ct.c_size_t), ("max_slots", ct.c_int32), ("ordering", ct.c_int32),
                ("precision", ct.c_int32), ("autotune", ct.c_int32)]


class ServerTiming(ct.Structure):
    _fields_ = [("queue_ms", ct.c_double), ("analyse_ms", ct.c_double), ("factor_ms", ct.c_double),
                ("tune_ms", ct.c_double), ("solve_ms", ct.c_double), ("total_ms", ct.c_double),
                ("slot", ct.c_int32), ("resident", ct.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(ct.Structure):
    _fields_ = [("queued", ct.c_int64), ("running", ct.c_int64), ("completed", ct.c_int64),
                ("instances", ct.c_int64), ("created", ct.c_int64), ("evicted", ct.c_int64),
                ("analyses", ct.c_int64), ("reserved_bytes", ct.c_size_t), ("peak_reserved_bytes", ct.c_size_t),
                ("device_used_bytes", ct.c_size_t), ("device_total_bytes", ct.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RsolveError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib().rsolve_last_error().decode()
        super().__init__(f"{where}: {status_string(status)} ({status}): {msg}")


_lib = None


def lib():
    """Load librsolve.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime; loading it first makes librsolve.so
        # bind to that same runtime (by soname), so one HIP runtime serves
        # the process and torch's streams and pointers are valid here
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover - host-only callers
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2309_11488_amd.build`")
        L = ct.CDLL(LIB_PATH)
        i32, vp, dbl = ct.c_int32, ct.c_void_p, ct.c_double
        P = ct.POINTER
        L.bcsr_create.argtypes = [i32, i32, i32, i32, vp, vp, vp, i32, vp, P(vp), P(i32)]
        L.bcsr_set_values.argtypes = [vp, vp, i32, i32, i32, vp]
        L.bcsr_set_wells.argtypes = [vp, i32, vp, vp, vp, vp, vp, i32, vp]
        L.bcsr_get_dims.argtypes = [vp, P(i32), P(i32), P(i32)]
        L.bcsr_spmv.argtypes = [vp, vp, vp, i32, i32, i32, vp]
        L.bcsr_destroy.argtypes = [vp]
        L.bcsr_set_option.argtypes = [vp, i32, i32]
        L.ilu0_analyse.argtypes = [vp, i32, P(vp)]
        L.ilu0_analyse_shared.argtypes = [vp, vp, P(vp)]
        L.ilu0_analyse_jacobi.argtypes = [vp, i32, vp, P(vp)]
        L.bcsr_partition.argtypes = [i32, i32, vp, vp, vp, i32, vp]
        L.ilu0_get_schedule.argtypes = [vp, vp, P(i32), vp]
        L.ilu0_get_sweep_levels.argtypes = [vp, P(i32), P(i32)]
        L.ilu0_set_option.argtypes = [vp, i32, i32]
        L.ilu0_get_option.argtypes = [vp, i32, P(i32)]
        L.ilu0_factor.argtypes = [vp, vp, i32, vp, vp]
        L.ilu0_factor_status.argtypes = [vp, vp]
        L.ilu0_autotune.argtypes = [vp, vp, vp, i32, dbl, i32, vp, ct.POINTER(TuneResult)]
        L.ilu0_get_factors.argtypes = [vp, i32, vp, vp]
        L.ilu0_apply.argtypes = [vp, vp, vp, i32, i32, i32, vp]
        L.ilu0_apply_noalloc.argtypes = [vp, vp, vp, i32, i32, vp]
        L.bicgstab_solve.argtypes = [vp, vp, vp, vp, dbl, i32, i32, vp, vp]
        L.gmres_solve.argtypes = [vp, vp, vp, vp, i32, dbl, i32, i32, vp, vp]
        L.ilu0_destroy.argtypes = [vp]
        L.ilu0_analyse_host.argtypes = [i32, vp, vp, i32, vp, P(i32), P(i32)]
        L.rsolve_profile_enable.argtypes = [i32]
        L.rsolve_profile_set_mask.argtypes = [i32]
        L.rsolve_profile_get.argtypes = [i32, P(dbl), P(ct.c_int64), P(dbl)]
        L.server_create.argtypes = [P(ServerConfig), P(vp)]
        L.server_request_bytes.argtypes = [i32, i32, i32, P(ct.c_size_t)]
        L.server_analysis_bytes.argtypes = [i32, i32, P(ct.c_size_t)]
        L.server_add_pattern.argtypes = [vp, i32, i32, vp, vp, P(i32), P(i32)]
        L.server_submit.argtypes = [vp, i32, vp, vp, vp, dbl, i32, i32, P(ct.c_int64)]
        L.server_poll.argtypes = [vp, ct.c_int64, P(SolveInfo), P(ServerTiming)]
        L.server_wait.argtypes = [vp, ct.c_int64, P(SolveInfo), P(ServerTiming)]
        L.server_get_stats.argtypes = [vp, P(ServerStats)]
        L.server_destroy.argtypes = [vp]
        L.rsolve_status_string.argtypes = [ct.c_int]
        L.rsolve_status_string.restype = ct.c_char_p
        L.rsolve_last_error.restype = ct.c_char_p
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().rsolve_status_string(int(status)).decode()


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _mem_ptr(*arrays):
    """(mem, [pointers]) for arrays that are all host NumPy or all CUDA torch tensors."""
    kinds = {_is_torch(a) for a in arrays if a is not None}
    if len(kinds) > 1:
        raise TypeError("mix of host and device arrays")
    if kinds == {True}:
        for a in arrays:
            if a is not None and (not a.is_cuda or not a.is_contiguous()):
                raise TypeError("torch tensors must be contiguous CUDA tensors")
        return MEM_DEVICE, [a.data_ptr() if a is not None else None for a in arrays]
    ptrs = []
    for a in arrays:
        if a is None:
            ptrs.append(None)
        else:
            if not a.flags["C_CONTIGUOUS"]:
                raise TypeError("NumPy arrays must be C-contiguous")
            ptrs.append(a.ctypes.data)
    return MEM_HOST, ptrs


def _stream(stream):
    if stream is not None:
        return stream
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:  # pragma: no cover - torch is optional for host callers
        pass
    return None


def _check(st, where, ok=(OK,)):
    if st not in ok:
        raise RsolveError(st, where)
    return st


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------- C names

def bcsr_create(rowptr, colidx, vals=None, *, batch=None, stream=None):
    """Create a BCSR handle.  vals: (batch, nnzb, 3, 3) or (nnzb, 3, 3) FP64."""
    if not _is_torch(rowptr):
        rowptr, colidx = _host(rowptr, np.int32), _host(colidx, np.int32)
    n = len(rowptr) - 1
    nnzb = len(colidx)
    if vals is not None:
        if not _is_torch(vals):
            vals = _host(vals, np.float64)
        if batch is None:
            batch = 1 if vals.ndim == 3 else int(vals.shape[0])
    batch = 1 if batch is None else batch
    mem, (rp, ci) = _mem_ptr(rowptr, colidx)
    vmem, (vp,) = _mem_ptr(vals)
    if vals is not None and vmem != mem:
        raise TypeError("pattern and values must live in the same memory")
    h = ct.c_void_p()
    bad = ct.c_int32(-1)
    st = lib().bcsr_create(n, nnzb, 3, batch, rp, ci, vp, mem, _stream(stream), ct.byref(h), ct.byref(bad))
    if st != OK:
        err = RsolveError(st, "bcsr_create")
        err.bad_row = bad.value
        raise err
    return h


def bcsr_set_values(A, vals, first_sys=0, n_sys=None, *, stream=None):
    if not _is_torch(vals):
        vals = _host(vals, np.float64)
    if n_sys is None:
        n_sys = 1 if vals.ndim == 3 else int(vals.shape[0])
    mem, (vp,) = _mem_ptr(vals)
    return _check(lib().bcsr_set_values(A, vp, first_sys, n_sys, mem, _stream(stream)), "bcsr_set_values")


def bcsr_set_wells(A, well_ptr=None, perf_row=None, B=None, C=None, Dinv=None, *, stream=None):
    """Standard wells kept separate (see rsolve.h); no arguments removes them.
    B, C: (batch, n_perf, 4, 3) or (n_perf, 4, 3); Dinv: (batch, n_wells, 4, 4)."""
    if well_ptr is None:
        return _check(lib().bcsr_set_wells(A, 0, None, None, None, None, None, MEM_HOST, _stream(stream)),
                      "bcsr_set_wells")
    well_ptr, perf_row = _host(well_ptr, np.int32), _host(perf_row, np.int32)
    if not _is_torch(B):
        B, C, Dinv = _host(B, np.float64), _host(C, np.float64), _host(Dinv, np.float64)
    mem, (bp, cp, dp) = _mem_ptr(B, C, Dinv)
    return _check(lib().bcsr_set_wells(A, len(well_ptr) - 1, well_ptr.ctypes.data, perf_row.ctypes.data, bp, cp, dp,
                                       mem, _stream(stream)), "bcsr_set_wells")


def bcsr_get_dims(A):
    n, nnzb, b = ct.c_int32(), ct.c_int32(), ct.c_int32()
    _check(lib().bcsr_get_dims(A, ct.byref(n), ct.byref(nnzb), ct.byref(b)), "bcsr_get_dims")
    return n.value, nnzb.value, b.value


def bcsr_spmv(A, x, y=None, first_sys=0, n_sys=None, *, stream=None):
    n, _, batch = bcsr_get_dims(A)
    if n_sys is None:
        n_sys = batch - first_sys
    if not _is_torch(x):
        x = _host(x, np.float64)
        if y is None:
            y = np.zeros((n_sys, n, 3))
    mem, (xp, yp) = _mem_ptr(x, y)
    _check(lib().bcsr_spmv(A, xp, yp, first_sys, n_sys, mem, _stream(stream)), "bcsr_spmv")
    return y


def bcsr_set_option(A, option, value):
    return _check(lib().bcsr_set_option(A, int(option), int(value)), "bcsr_set_option")


def bcsr_destroy(A):
    if A:
        lib().bcsr_destroy(A)


def ilu0_analyse(A, ordering=ORDER_LEVEL_SET):
    h = ct.c_void_p()
    _check(lib().ilu0_analyse(A, ordering, ct.byref(h)), "ilu0_analyse")
    return h


def ilu0_analyse_jacobi(A, ordering, part):
    """Block-Jacobi-ILU0 analysis: ``part`` gives every row a partition id."""
    n, _, _ = bcsr_get_dims(A)
    part = _host(part, np.int32)
    if part.shape != (n,):
        raise ValueError("part must hold one partition id per block row")
    h = ct.c_void_p()
    _check(lib().ilu0_analyse_jacobi(A, ordering, part.ctypes.data, ct.byref(h)), "ilu0_analyse_jacobi")
    return h


def bcsr_partition(rowptr, colidx, n_parts, weights=None):
    """Coupling-weighted partition of the rows into n_parts near-equal parts (host only)."""
    rowptr, colidx = _host(rowptr, np.int32), _host(colidx, np.int32)
    n = len(rowptr) - 1
    part = np.zeros(max(n, 1), np.int32)
    w = None if weights is None else _host(weights, np.float64)
    if w is not None and w.shape != (len(colidx),):
        raise ValueError("weights must hold one value per stored block")
    _check(lib().bcsr_partition(n, len(colidx), rowptr.ctypes.data, colidx.ctypes.data,
                                None if w is None else w.ctypes.data, int(n_parts), part.ctypes.data),
           "bcsr_partition")
    return part[:n]


def ilu0_analyse_shared(A, like):
    """A further preconditioner for A sharing the analysis of ``like`` (same pattern)."""
    h = ct.c_void_p()
    _check(lib().ilu0_analyse_shared(A, like, ct.byref(h)), "ilu0_analyse_shared")
    return h


def ilu0_get_schedule(M, n):
    perm = np.zeros(max(n, 1), np.int32)
    ns = ct.c_int32()
    _check(lib().ilu0_get_schedule(M, perm.ctypes.data, ct.byref(ns), None), "ilu0_get_schedule")
    sp = np.zeros(ns.value + 1, np.int32)
    lib().ilu0_get_schedule(M, None, ct.byref(ns), sp.ctypes.data)
    return perm[:n], ns.value, sp


def ilu0_get_sweep_levels(M):
    a, b = ct.c_int32(), ct.c_int32()
    _check(lib().ilu0_get_sweep_levels(M, ct.byref(a), ct.byref(b)), "ilu0_get_sweep_levels")
    return a.value, b.value


def ilu0_set_option(M, option, value):
    return _check(lib().ilu0_set_option(M, int(option), int(value)), "ilu0_set_option")


def ilu0_get_option(M, option):
    v = ct.c_int32()
    _check(lib().ilu0_get_option(M, int(option), ct.byref(v)), "ilu0_get_option")
    return v.value


def ilu0_autotune(M, A, b, reduction=1e-2, reps=3, *, stream=None):
    """Time launch configurations on solves of b and apply the fastest (see rsolve.h)."""
    if not _is_torch(b):
        b = _host(b, np.float64)
    mem, (bp,) = _mem_ptr(b)
    r = TuneResult()
    _check(lib().ilu0_autotune(M, A, bp, mem, float(reduction), int(reps), _stream(stream), ct.byref(r)),
           "ilu0_autotune")
    return r.as_dict()


def ilu0_factor(M, A, precision=PREC_FP64, *, stream=None):
    """Factor every system; returns (status, bad_row per system)."""
    _, _, batch = bcsr_get_dims(A)
    bad = np.full(batch, -1, np.int32)
    st = lib().ilu0_factor(M, A, precision, _stream(stream), bad.ctypes.data)
    _check(st, "ilu0_factor", ok=(OK, ZERO_PIVOT))
    return st, bad


def ilu0_factor_status(M, batch):
    """Status and bad_row per system of the last factorisation (waits for a
    queued one)."""
    bad = np.full(batch, -1, np.int32)
    st = lib().ilu0_factor_status(M, bad.ctypes.data)
    _check(st, "ilu0_factor_status", ok=(OK, ZERO_PIVOT))
    return st, bad


def ilu0_get_factors(M, sys, n, nnzb):
    lu = np.zeros((max(nnzb, 1), 3, 3))
    dinv = np.zeros((max(n, 1), 3, 3))
    _check(lib().ilu0_get_factors(M, sys, lu.ctypes.data, dinv.ctypes.data), "ilu0_get_factors")
    return lu[:nnzb], dinv[:n]


def ilu0_apply(M, v, z=None, first_sys=0, n_sys=1, *, stream=None):
    if not _is_torch(v):
        v = _host(v, np.float64)
        if z is None:
            z = np.zeros_like(v)
    mem, (vp, zp) = _mem_ptr(v, z)
    _check(lib().ilu0_apply(M, vp, zp, first_sys, n_sys, mem, _stream(stream)), "ilu0_apply")
    return z


def ilu0_apply_noalloc(M, v, z, first_sys=0, n_sys=1, *, stream=None):
    """ilu0_apply with every intermediate in the library's fixed per-GPU
    workspace (no device allocation): v and z are device tensors."""
    if not (_is_torch(v) and _is_torch(z)):
        raise TypeError("ilu0_apply_noalloc: v and z must be CUDA tensors")
    _, (vp, zp) = _mem_ptr(v, z)
    _check(lib().ilu0_apply_noalloc(M, vp, zp, first_sys, n_sys, _stream(stream)), "ilu0_apply_noalloc")
    return z


def bicgstab_solve(M, A, b, x=None, reduction=1e-2, max_iter=200, *, stream=None):
    """Solve every system of A.  Returns (x, status, [info dict per system])."""
    _, _, batch = bcsr_get_dims(A)
    if not _is_torch(b):
        b = _host(b, np.float64)
        if x is None:
            x = np.zeros_like(b)
    mem, (bp, xp) = _mem_ptr(b, x)
    info = (SolveInfo * batch)()
    st = lib().bicgstab_solve(M, A, bp, xp, float(reduction), int(max_iter), mem, _stream(stream), info)
    _check(st, "bicgstab_solve", ok=(OK, NOT_CONVERGED, BREAKDOWN, NON_FINITE, ZERO_PIVOT))
    return x, st, [i.as_dict() for i in info]


def gmres_solve(M, A, b, x=None, restart=30, reduction=1e-2, max_iter=200, *, stream=None):
    """Restarted GMRES on every system of A (max_iter counts Arnoldi steps).
    Returns (x, status, [info dict per system]); half_steps = Arnoldi steps."""
    _, _, batch = bcsr_get_dims(A)
    if not _is_torch(b):
        b = _host(b, np.float64)
        if x is None:
            x = np.zeros_like(b)
    mem, (bp, xp) = _mem_ptr(b, x)
    info = (SolveInfo * batch)()
    st = lib().gmres_solve(M, A, bp, xp, int(restart), float(reduction), int(max_iter), mem, _stream(stream), info)
    _check(st, "gmres_solve", ok=(OK, NOT_CONVERGED, NON_FINITE, ZERO_PIVOT))
    return x, st, [i.as_dict() for i in info]


def ilu0_destroy(M):
    if M:
        lib().ilu0_destroy(M)


def ilu0_analyse_host(rowptr, colidx, ordering=ORDER_LEVEL_SET):
    """Host-only analysis: (status, perm, n_sets, bad_row); needs no GPU."""
    rowptr, colidx = _host(rowptr, np.int32), _host(colidx, np.int32)
    n = len(rowptr) - 1
    perm = np.zeros(max(n, 1), np.int32)
    ns, bad = ct.c_int32(), ct.c_int32()
    st = lib().ilu0_analyse_host(n, rowptr.ctypes.data, colidx.ctypes.data, ordering, perm.ctypes.data,
                                 ct.byref(ns), ct.byref(bad))
    return st, perm[:n], ns.value, bad.value


def rsolve_profile_enable(mask):
    return _check(lib().rsolve_profile_enable(int(mask)), "rsolve_profile_enable")


def rsolve_profile_set_mask(mask):
    """Change the timed classes without clearing the counters."""
    return _check(lib().rsolve_profile_set_mask(int(mask)), "rsolve_profile_set_mask")


def rsolve_profile_get(cls):
    """(device ms, units, algorithmic bytes) accumulated for a kernel class."""
    ms, units, byt = ct.c_double(), ct.c_int64(), ct.c_double()
    _check(lib().rsolve_profile_get(int(cls), ct.byref(ms), ct.byref(units), ct.byref(byt)), "rsolve_profile_get")
    return ms.value, units.value, byt.value


# ------------------------------------------------------------ convenience

class Solver:
    """Owns a matrix handle and its ILU0 handle: create -> analyse -> factor -> solve."""

    def __init__(self, rowptr, colidx, vals, *, ordering=ORDER_LEVEL_SET, precision=PREC_FP64, stream=None,
                 part=None):
        self.A = bcsr_create(rowptr, colidx, vals, stream=stream)
        self.n, self.nnzb, self.batch = bcsr_get_dims(self.A)
        self.M = ilu0_analyse(self.A, ordering) if part is None else ilu0_analyse_jacobi(self.A, ordering, part)
        self.precision = precision
        self.stream = stream

    def factor(self, vals=None):
        if vals is not None:
            bcsr_set_values(self.A, vals, stream=self.stream)
        return ilu0_factor(self.M, self.A, self.precision, stream=self.stream)

    def solve(self, b, x=None, reduction=1e-2, max_iter=200):
        return bicgstab_solve(self.M, self.A, b, x, reduction, max_iter, stream=self.stream)

    def solve_gmres(self, b, x=None, restart=30, reduction=1e-2, max_iter=200):
        return gmres_solve(self.M, self.A, b, x, restart, reduction, max_iter, stream=self.stream)

    def close(self):
        ilu0_destroy(self.M)
        bcsr_destroy(self.A)
        self.M = self.A = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """A request server (see ``server_create`` in rsolve.h).

    ``submit`` borrows its arrays until the request is collected with
    ``poll``/``wait``; the binding keeps references to them until then.
    """

    def __init__(self, hbm_budget_bytes=200 << 30, max_slots=4, ordering=ORDER_GRAPH_COLOUR,
                 precision=PREC_FP32_FACTORS, autotune=False):
        cfg = ServerConfig(int(hbm_budget_bytes), int(max_slots), int(ordering), int(precision), int(autotune))
        h = ct.c_void_p()
        _check(lib().server_create(ct.byref(cfg), ct.byref(h)), "server_create")
        self.h = h
        self.precision = precision
        self._held = {}

    def add_pattern(self, rowptr, colidx):
        """Register a pattern (copied by the server); returns its id."""
        rowptr, colidx = _host(rowptr, np.int32), _host(colidx, np.int32)
        pid, bad = ct.c_int32(), ct.c_int32(-1)
        st = lib().server_add_pattern(self.h, len(rowptr) - 1, len(colidx), rowptr.ctypes.data, colidx.ctypes.data,
                                      ct.byref(pid), ct.byref(bad))
        if st != OK:
            err = RsolveError(st, "server_add_pattern")
            err.bad_row = bad.value
            raise err
        return pid.value

    def submit(self, pattern, vals, b, x=None, reduction=1e-2, max_iter=200):
        """Queue a solve of a registered pattern; returns a ticket."""
        if not _is_torch(vals):
            vals, b = _host(vals, np.float64), _host(b, np.float64)
            if x is None:
                x = np.zeros_like(b)
        mem, (vp, bp, xp) = _mem_ptr(vals, b, x)
        t = ct.c_int64()
        _check(lib().server_submit(self.h, int(pattern), vp, bp, xp, float(reduction), int(max_iter), mem,
                                   ct.byref(t)), "server_submit")
        self._held[t.value] = (vals, b, x)
        return t.value

    def _finish(self, fn, ticket):
        info, tm = SolveInfo(), ServerTiming()
        if ticket not in self._held:
            raise RsolveError(INVALID_ARG, "server: unknown or already collected ticket")
        st = fn(self.h, int(ticket), ct.byref(info), ct.byref(tm))
        if st == PENDING:
            return None
        x = self._held.pop(ticket)[2]
        return x, st, info.as_dict(), tm.as_dict()

    def poll(self, ticket):
        """None while pending, else (x, status, info, timing)."""
        return self._finish(lib().server_poll, ticket)

    def wait(self, ticket):
        return self._finish(lib().server_wait, ticket)

    def stats(self):
        st = ServerStats()
        _check(lib().server_get_stats(self.h, ct.byref(st)), "server_get_stats")
        return st.as_dict()

    @staticmethod
    def request_bytes(n, nnzb, precision=PREC_FP32_FACTORS):
        v = ct.c_size_t()
        _check(lib().server_request_bytes(int(n), int(nnzb), int(precision), ct.byref(v)), "server_request_bytes")
        return v.value

    @staticmethod
    def analysis_bytes(n, nnzb):
        v = ct.c_size_t()
        _check(lib().server_analysis_bytes(int(n), int(nnzb), ct.byref(v)), "server_analysis_bytes")
        return v.value

    def close(self):
        if self.h:
            lib().server_destroy(self.h)
            self.h = None
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
