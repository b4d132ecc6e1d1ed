"""CPU FP64 oracle of block-ILU0-preconditioned BiCGStab (ctypes over liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the HIP library never imports, links or calls it.
It shares no code with the HIP path.  The C source (``oracle.c``) documents
which passage of the paper each function follows.

Status codes follow the documented C-ABI convention (0 ok, 1 not converged,
2 breakdown, negative = error) but are defined here independently.
"""

from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
INVALID, BAD_PATTERN, MISSING_DIAG, ZERO_PIVOT, NON_FINITE = -1, -3, -4, -5, -6
ORDER_NATURAL, ORDER_LEVEL, ORDER_COLOUR, ORDER_RCM_LEVEL = 0, 1, 2, 3
PREC_ILU_F64, PREC_ILU_F32, PREC_NONE = 0, 1, 2


class Info(ct.Structure):
    _fields_ = [("status", ct.c_int), ("half_steps", ct.c_int), ("r0_norm", ct.c_double),
                ("final_norm", ct.c_double), ("true_rel_residual", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no contraction of multiply-adds)."""
    src = os.path.join(HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None

_I32P = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_F64P = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_F32P = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = ct.CDLL(LIB_PATH)
        ci, cd, vp = ct.c_int, ct.c_double, ct.c_void_p
        L.orc_validate.argtypes = [ci, _I32P, _I32P, ct.POINTER(ci)]
        L.orc_level_sets.argtypes = [ci, _I32P, _I32P, _I32P, _I32P]
        L.orc_dsatur_colour.argtypes = [ci, _I32P, _I32P, _I32P, _I32P]
        L.orc_rcm_levels.argtypes = [ci, _I32P, _I32P, _I32P, _I32P]
        L.orc_permute.argtypes = [ci, _I32P, _I32P, _F64P, _I32P, _I32P, _I32P, _F64P]
        L.orc_permute.restype = None
        L.orc_ilu0.argtypes = [ci, _I32P, _I32P, _F64P, _F64P, ct.POINTER(ci)]
        L.orc_ilu0_kij.argtypes = [ci, _I32P, _I32P, _F64P, _F64P, ct.POINTER(ci)]
        L.orc_apply.argtypes = [ci, _I32P, _I32P, _F64P, _F64P, _F64P, _F64P]
        L.orc_apply.restype = None
        L.orc_apply_f32.argtypes = [ci, _I32P, _I32P, _F32P, _F32P, _F64P, _F64P]
        L.orc_apply_f32.restype = None
        L.orc_spmv.argtypes = [ci, _I32P, _I32P, _F64P, _F64P, _F64P]
        L.orc_spmv.restype = None
        L.orc_inv3.argtypes = [_F64P, _F64P]
        L.orc_bicgstab.argtypes = [ci, _I32P, _I32P, _F64P, _F64P, _F64P, ci, _F64P, cd, ci, _F64P,
                                   ct.POINTER(Info), vp]
        L.orc_bicgstab_split.argtypes = [ci, _I32P, _I32P, _F64P, _I32P, _I32P, _F64P, _F64P, ci, _F64P, cd, ci,
                                         _F64P, ct.POINTER(Info), vp]
        L.orc_solve.argtypes = [ci, _I32P, _I32P, _F64P, _F64P, ci, ci, cd, ci, _F64P, ct.POINTER(Info),
                                _I32P, ct.POINTER(ci), ct.POINTER(ci)]
        L.orc_solve_jacobi.argtypes = [ci, _I32P, _I32P, _F64P, vp, _F64P, ci, ci, cd, ci, _F64P,
                                       ct.POINTER(Info), _I32P, ct.POINTER(ci), ct.POINTER(ci)]
        L.orc_jacobi_matrix.argtypes = [ci, _I32P, _I32P, _F64P, _I32P, _I32P, _I32P, _F64P]
        L.orc_wells_apply.argtypes = [ci, _I32P, _I32P, _F64P, _F64P, _F64P, _F64P, _F64P]
        L.orc_gmres.argtypes = [ci, _I32P, _I32P, _F64P, _F64P, _F64P, ci, _F64P, ci, cd, ci, _F64P,
                                ct.POINTER(Info), vp]
        L.orc_gmres_wells.argtypes = [ci, _I32P, _I32P, _F64P, ci, vp, vp, vp, vp, vp, _F64P, _F64P, ci, _F64P,
                                      ci, cd, ci, _F64P, ct.POINTER(Info), vp]
        L.orc_wells_apply.restype = None
        L.orc_bicgstab_wells.argtypes = [ci, _I32P, _I32P, _F64P, ci, vp, vp, vp, vp, vp, _F64P, _F64P, ci, _F64P,
                                         cd, ci, _F64P, ct.POINTER(Info), vp]
        L.orc_solve_wells.argtypes = [ci, _I32P, _I32P, _F64P, vp, ci, vp, vp, vp, vp, vp, _F64P, ci, ci, cd, ci,
                                      _F64P, ct.POINTER(Info), _I32P, ct.POINTER(ci), ct.POINTER(ci)]
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def validate(rowptr, colidx):
    """(status, bad_row) of the structural check."""
    bad = ct.c_int(-1)
    st = lib().orc_validate(len(rowptr) - 1, _i32(rowptr), _i32(colidx), ct.byref(bad))
    return st, bad.value


def level_sets(rowptr, colidx):
    """(n_levels, level[n], perm[n]) of level scheduling on lower dependencies."""
    n = len(rowptr) - 1
    level = np.zeros(n, np.int32)
    perm = np.zeros(n, np.int32)
    nl = lib().orc_level_sets(n, _i32(rowptr), _i32(colidx), level, perm)
    return nl, level, perm


def dsatur_colour(rowptr, colidx):
    """(n_colours, colour[n], perm[n]) of the DSatur colouring (Brelaz 1979;
    ties by degree, then by the smaller index)."""
    n = len(rowptr) - 1
    col = np.zeros(n, np.int32)
    perm = np.zeros(n, np.int32)
    nc = lib().orc_dsatur_colour(n, _i32(rowptr), _i32(colidx), col, perm)
    return nc, col, perm


def rcm_levels(rowptr, colidx):
    """(n_levels, level[n], perm[n]) of level scheduling after a reverse
    Cuthill-McKee renumbering (rows by level, then RCM position)."""
    n = len(rowptr) - 1
    level = np.zeros(max(n, 1), np.int32)
    perm = np.zeros(max(n, 1), np.int32)
    nl = lib().orc_rcm_levels(n, _i32(rowptr), _i32(colidx), level, perm)
    return nl, level[:n], perm[:n]


def ordering_perm(rowptr, colidx, ordering):
    n = len(rowptr) - 1
    if ordering == ORDER_LEVEL:
        return level_sets(rowptr, colidx)[2]
    if ordering == ORDER_COLOUR:
        return dsatur_colour(rowptr, colidx)[2]
    if ordering == ORDER_RCM_LEVEL:
        return rcm_levels(rowptr, colidx)[2]
    return np.arange(n, dtype=np.int32)


def permute(rowptr, colidx, vals, perm):
    """(rowptr', colidx', vals') of P A P^T with perm[new] = old."""
    n = len(rowptr) - 1
    nnz = len(colidx)
    prow = np.zeros(n + 1, np.int32)
    pcol = np.zeros(nnz, np.int32)
    pv = np.zeros((nnz, 3, 3), np.float64)
    lib().orc_permute(n, _i32(rowptr), _i32(colidx), _f64(vals), _i32(perm), prow, pcol, pv)
    return prow, pcol, pv


def ilu0(rowptr, colidx, vals, kij=False):
    """(status, bad_row, lu[nnzb,3,3], dinv[n,3,3]) of block ILU0 on the given order."""
    n = len(rowptr) - 1
    lu = _f64(vals).copy()
    dinv = np.zeros((n, 3, 3), np.float64)
    bad = ct.c_int(-1)
    fn = lib().orc_ilu0_kij if kij else lib().orc_ilu0
    st = fn(n, _i32(rowptr), _i32(colidx), lu, dinv, ct.byref(bad))
    return st, bad.value, lu, dinv


def apply(rowptr, colidx, lu, dinv, v):
    n = len(rowptr) - 1
    z = np.zeros((n, 3), np.float64)
    lib().orc_apply(n, _i32(rowptr), _i32(colidx), _f64(lu), _f64(dinv), _f64(v).reshape(n, 3), z)
    return z


def apply_f32(rowptr, colidx, lu, dinv, v):
    """Apply with factors rounded to FP32 and FP32 sweep arithmetic."""
    n = len(rowptr) - 1
    z = np.zeros((n, 3), np.float64)
    lib().orc_apply_f32(n, _i32(rowptr), _i32(colidx), np.ascontiguousarray(lu, np.float32),
                        np.ascontiguousarray(dinv, np.float32), _f64(v).reshape(n, 3), z)
    return z


def spmv(rowptr, colidx, vals, x):
    n = len(rowptr) - 1
    y = np.zeros((n, 3), np.float64)
    lib().orc_spmv(n, _i32(rowptr), _i32(colidx), _f64(vals), _f64(x).reshape(n, 3), y)
    return y


def inv3(a):
    out = np.zeros((3, 3), np.float64)
    ok = lib().orc_inv3(_f64(a), out)
    return ok, out


def wells_apply(well_ptr, perf_row, B, C, Dinv, x, y):
    """y -= sum over wells of C^T D^-1 B x (Algorithm 5); returns the new y."""
    y = _f64(y).copy()
    n = y.reshape(-1, 3).shape[0]
    lib().orc_wells_apply(len(well_ptr) - 1, _i32(well_ptr), _i32(perf_row), _f64(B), _f64(C), _f64(Dinv),
                          _f64(x).reshape(n, 3), y.reshape(n, 3))
    return y


def gmres(rowptr, colidx, vals, lu, dinv, b, *, precond=PREC_ILU_F64, restart=30, reduction=1e-2, max_iter=200,
          trace=False, wells=None):
    """Right-preconditioned GMRES(restart) on an already ordered system.
    ``wells`` = (well_ptr, perf_row, B, C, Dinv) in this system's numbering
    adds standard wells kept separate to every product with A.
    Returns (x, info dict[, residual estimate after every Arnoldi step])."""
    n = len(rowptr) - 1
    x = np.zeros((n, 3), np.float64)
    info = Info()
    tr = np.zeros(max(max_iter, 1), np.float64) if trace else None
    lu = _f64(lu) if lu is not None else np.zeros((max(len(colidx), 1), 3, 3))
    dinv = _f64(dinv) if dinv is not None else np.zeros((max(n, 1), 3, 3))
    trp = tr.ctypes.data if tr is not None else None
    if wells is None:
        lib().orc_gmres(n, _i32(rowptr), _i32(colidx), _f64(vals), lu, dinv, precond, _f64(b).reshape(n, 3),
                        int(restart), reduction, max_iter, x, ct.byref(info), trp)
    else:
        wp, pr, B, C, D = (_i32(wells[0]), _i32(wells[1]), _f64(wells[2]), _f64(wells[3]), _f64(wells[4]))
        lib().orc_gmres_wells(n, _i32(rowptr), _i32(colidx), _f64(vals), len(wp) - 1, wp.ctypes.data,
                              pr.ctypes.data, B.ctypes.data, C.ctypes.data, D.ctypes.data, lu, dinv, precond,
                              _f64(b).reshape(n, 3), int(restart), reduction, max_iter, x, ct.byref(info), trp)
    if trace:
        return x, info.as_dict(), tr[:info.half_steps]
    return x, info.as_dict()


def solve_gmres(rowptr, colidx, vals, b, *, ordering=ORDER_NATURAL, precond=PREC_ILU_F64, restart=30,
                reduction=1e-2, max_iter=200, wells=None):
    """The whole path with GMRES: ordering, reordered copy, ILU0, GMRES,
    x back in the original order, true residual with the original operator
    (``wells`` = (well_ptr, perf_row, B, C, Dinv) in the caller's numbering:
    standard wells kept separate)."""
    perm = ordering_perm(rowptr, colidx, ordering)
    prow, pcol, pv = permute(rowptr, colidx, vals, perm)
    lu = dinv = None
    if precond != PREC_NONE:
        st, bad, lu, dinv = ilu0(prow, pcol, pv)
        if st != OK:
            return np.zeros((len(rowptr) - 1, 3)), {"status": st, "bad_row": int(perm[bad]) if bad >= 0 else -1}
    b = _f64(b).reshape(-1, 3)
    pw = None
    if wells is not None:
        iperm = np.empty_like(perm)
        iperm[perm] = np.arange(len(perm), dtype=perm.dtype)
        pw = (wells[0], iperm[_i32(wells[1])], wells[2], wells[3], wells[4])
    xp, info = gmres(prow, pcol, pv, lu, dinv, b[perm], precond=precond, restart=restart, reduction=reduction,
                     max_iter=max_iter, wells=pw)
    x = np.empty_like(xp)
    x[perm] = xp
    ax = spmv(rowptr, colidx, vals, x)
    if wells is not None:
        ax = wells_apply(wells[0], wells[1], wells[2], wells[3], wells[4], x, ax)
    r = b - ax.reshape(-1, 3)
    info["true_rel_residual"] = float(np.linalg.norm(r) / np.linalg.norm(b)) if np.linalg.norm(b) > 0 else 0.0
    info["perm"] = perm
    return x, info


def jacobi_matrix(rowptr, colidx, vals, part):
    """(rowptr', colidx', vals') of the Jacobi matrix: blocks within one partition."""
    n = len(rowptr) - 1
    nnz = len(colidx)
    rrow = np.zeros(n + 1, np.int32)
    rcol = np.zeros(max(nnz, 1), np.int32)
    rv = np.zeros((max(nnz, 1), 3, 3), np.float64)
    k = lib().orc_jacobi_matrix(n, _i32(rowptr), _i32(colidx), _f64(vals), _i32(part), rrow, rcol, rv)
    return rrow, rcol[:k], rv[:k]


def bicgstab(rowptr, colidx, vals, lu, dinv, b, *, precond=PREC_ILU_F64, reduction=1e-2, max_iter=200,
             trace=False, mrow=None, mcol=None, wells=None):
    """BiCGStab on an already ordered system.  Returns (x, info dict[, trace (k, 8)]).

    The factors lu / dinv live on (mrow, mcol) when given (a Jacobi matrix's
    pattern), else on the matrix's own pattern.  ``wells`` = (well_ptr,
    perf_row, B, C, Dinv) in this system's numbering adds standard wells kept
    separate to every product with A (factors on the matrix's pattern).
    The trace holds, per iteration: rho, (rhat, v), alpha, ||s||, (t, s),
    (t, t), omega, ||r||."""
    n = len(rowptr) - 1
    x = np.zeros((n, 3), np.float64)
    info = Info()
    tr = np.zeros((max(max_iter, 1), 8), np.float64) if trace else None
    mrow = _i32(rowptr if mrow is None else mrow)
    mcol = _i32(colidx if mcol is None else mcol)
    lu = _f64(lu) if lu is not None else np.zeros((max(len(mcol), 1), 3, 3))
    dinv = _f64(dinv) if dinv is not None else np.zeros((max(n, 1), 3, 3))
    trp = tr.ctypes.data if tr is not None else None
    if wells is not None:
        if mrow is not None and not (np.array_equal(mrow, _i32(rowptr)) and np.array_equal(mcol, _i32(colidx))):
            raise ValueError("bicgstab with wells takes factors on the matrix's own pattern")
        wp, pr, B, C, D = (_i32(wells[0]), _i32(wells[1]), _f64(wells[2]), _f64(wells[3]), _f64(wells[4]))
        lib().orc_bicgstab_wells(n, _i32(rowptr), _i32(colidx), _f64(vals), len(wp) - 1, wp.ctypes.data,
                                 pr.ctypes.data, B.ctypes.data, C.ctypes.data, D.ctypes.data, lu, dinv, precond,
                                 _f64(b).reshape(n, 3), reduction, max_iter, x, ct.byref(info), trp)
    else:
        lib().orc_bicgstab_split(n, _i32(rowptr), _i32(colidx), _f64(vals), mrow, mcol, lu, dinv, precond,
                                 _f64(b).reshape(n, 3), reduction, max_iter, x, ct.byref(info), trp)
    if trace:
        return x, info.as_dict(), tr
    return x, info.as_dict()


def solve(rowptr, colidx, vals, b, *, ordering=ORDER_NATURAL, precond=PREC_ILU_F64, reduction=1e-2,
          max_iter=200, part=None, wells=None):
    """The whole path on one system in original order.

    ``part`` (n partition ids) selects the Block-Jacobi-ILU0 preconditioner;
    ``wells`` = (well_ptr, perf_row, B, C, Dinv) adds standard wells kept
    separate in the operator.  Returns (x[n,3], info dict with status,
    half_steps, r0_norm, final_norm, true_rel_residual, n_sets, bad_row, perm).
    """
    n = len(rowptr) - 1
    x = np.zeros((n, 3), np.float64)
    info = Info()
    perm = np.zeros(max(n, 1), np.int32)
    nsets = ct.c_int(0)
    bad = ct.c_int(-1)
    part = None if part is None else _i32(part)
    nw, wargs = 0, [None] * 5
    if wells is not None:
        wp, pr, B, C, D = wells
        keep = [_i32(wp), _i32(pr), _f64(B), _f64(C), _f64(D)]
        nw = len(wp) - 1
        wargs = [a.ctypes.data for a in keep]
    lib().orc_solve_wells(n, _i32(rowptr), _i32(colidx), _f64(vals), None if part is None else part.ctypes.data, nw,
                          *wargs, _f64(b).reshape(n, 3), ordering, precond, reduction, max_iter, x, ct.byref(info),
                          perm, ct.byref(nsets), ct.byref(bad))
    d = info.as_dict()
    d.update(n_sets=nsets.value, bad_row=bad.value, perm=perm[:n])
    return x, d
