"""Small test-side builders: hand-shaped patterns and dense expansions.

These feed both sides of a comparison; they hold no solver arithmetic.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np


def dense_pattern(n):
    rowptr = np.arange(0, n * n + 1, n, dtype=np.int32)
    colidx = np.tile(np.arange(n, dtype=np.int32), n)
    return rowptr, colidx


def chain_pattern(n):
    """Block tridiagonal (1D chain): ILU0 drops no fill on it."""
    rows, cols = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
    rowptr = np.zeros(n + 1, np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return rowptr, np.asarray(cols, np.int32)


def pattern_from_pairs(n, pairs, symmetric=True):
    s = set((i, i) for i in range(n))
    for i, j in pairs:
        s.add((i, j))
        if symmetric:
            s.add((j, i))
    ent = sorted(s)
    rowptr = np.zeros(n + 1, np.int32)
    np.cumsum(np.bincount([i for i, _ in ent], minlength=n), out=rowptr[1:])
    return rowptr, np.asarray([j for _, j in ent], np.int32)


def random_values(rowptr, colidx, seed=0, diag_boost=4.0):
    """Non-symmetric blocks with a dominant diagonal (so no zero pivots)."""
    rng = np.random.default_rng(seed)
    n = len(rowptr) - 1
    vals = rng.uniform(-1.0, 1.0, size=(len(colidx), 3, 3))
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            if colidx[p] == i:
                vals[p] += diag_boost * (rowptr[i + 1] - rowptr[i]) * np.eye(3)
    return vals


def to_dense(rowptr, colidx, vals):
    n = len(rowptr) - 1
    a = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            j = colidx[p]
            a[3 * i:3 * i + 3, 3 * j:3 * j + 3] = vals[p]
    return a


def split_lu(rowptr, colidx, lu):
    """Expand in-place factors into dense unit-lower L and upper U."""
    n = len(rowptr) - 1
    L = np.eye(3 * n)
    U = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            j = colidx[p]
            blk = slice(3 * i, 3 * i + 3), slice(3 * j, 3 * j + 3)
            if j < i:
                L[blk] = lu[p]
            else:
                U[blk] = lu[p]
    return L, U


def pattern_set(rowptr, colidx):
    n = len(rowptr) - 1
    return {(i, int(colidx[p])) for i in range(n) for p in range(rowptr[i], rowptr[i + 1])}


def read_golden(path):
    """Parse a ``NAME = a b c ; d e f ; ...`` fixture of exact rationals."""
    out = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = (t.strip() for t in line.split("=", 1))
            rows = [[float(Fraction(t)) for t in r.split()] for r in val.split(";")]
            out[key] = np.asarray(rows if len(rows) > 1 else rows[0])
    return out


TIMING_KEYS = ("factor_ms", "solve_ms")


def outcome(info):
    """A solve's per-system results (a list of info dicts, or one dict)
    without its device timings, which differ from run to run (compare these
    when results must be bitwise equal)."""
    if isinstance(info, dict):
        info = [info]
    return [{k: v for k, v in i.items() if k not in TIMING_KEYS} for i in info]


# BiCGStab breakdown cases, derived by hand in exact binary fractions (every
# quantity below is exact in FP64, so any summation order gives the same
# bits).  The operator is one 3x3 block K; a preconditioner equal to the
# identity makes the iteration plain BiCGStab on K (x0 = 0, rhat = r0 = b,
# p = b in the first iteration):
#   rhat_v: K = rotation in the (e1, e2) plane + e3, b = e1:
#           v = K b = -e2, (rhat, v) = 0 -> breakdown before alpha; x = 0,
#           no half step taken.
#   tt:     K = [[1,1,0],[0,0,0],[0,0,1]] (singular), b = (1,1,0):
#           v = (2,0,0), alpha = 2/2 = 1, s = (-1,1,0) (||s|| = ||b||),
#           t = K s = 0, (t, t) = 0 -> breakdown after the half step; x = 0.
#   omega:  K = [[2,1,0],[1,0,0],[0,0,1]], b = (1,1,0): v = (3,1,0),
#           alpha = 2/4, s = (-1/2,1/2,0), t = (-1/2,-1/2,0), (t, s) = 0 ->
#           omega = 0: breakdown, x keeps the half-step update alpha p = (1/2,1/2,0).
#   rho:    K = [[1,1,0],[-1,2,1],[-1,1,0]], b = (0,2,2): v = (2,6,2),
#           alpha = 8/16, s = (-1,-1,1), t = (-2,0,0), omega = 2/4,
#           x = alpha b + omega s = (-1/2,1/2,3/2), r = s - omega t = (0,-1,1),
#           next rho = (rhat, r) = 0 -> breakdown after the full step.
# At a reduction of 0.1 none of the norms (||s||/||b|| >= 1/2, ||r||/||b||
# = 1/2) meets the test first.
BREAKDOWN_CASES = {
    "rhat_v": dict(K=[[0, 1, 0], [-1, 0, 0], [0, 0, 1]], b=[1, 0, 0], half=0, x=[0, 0, 0]),
    "tt": dict(K=[[1, 1, 0], [0, 0, 0], [0, 0, 1]], b=[1, 1, 0], half=1, x=[0, 0, 0]),
    "omega": dict(K=[[2, 1, 0], [1, 0, 0], [0, 0, 1]], b=[1, 1, 0], half=1, x=[0.5, 0.5, 0]),
    "rho": dict(K=[[1, 1, 0], [-1, 2, 1], [-1, 1, 0]], b=[0, 2, 2], half=2, x=[-0.5, 0.5, 1.5]),
}


def breakdown_as_well(K):
    """The operator K as the identity block with one standard well kept
    separate: A = I, one well perforating row 0 with D^-1 = I4, C = [I3; 0]
    and B = [I3 - K; 0], so A x - C^T D^-1 B x = K x exactly, while ILU0 of
    A is the identity.  Returns (rowptr, colidx, vals, well_ptr, perf_row,
    B, C, Dinv) with one system."""
    rowptr = np.array([0, 1], np.int32)
    colidx = np.array([0], np.int32)
    vals = np.eye(3)[None, None]                       # (batch 1, nnzb 1, 3, 3)
    C = np.zeros((1, 1, 4, 3))
    C[0, 0, :3] = np.eye(3)
    B = np.zeros((1, 1, 4, 3))
    B[0, 0, :3] = np.eye(3) - np.asarray(K, np.float64)
    Dinv = np.eye(4)[None, None]
    return rowptr, colidx, vals, np.array([0, 1], np.int32), np.array([0], np.int32), B, C, Dinv


def fp32_apply_bound(rowptr, colidx, lu, dinv, v):
    """Element-wise bound on how far two FP32 evaluations of the ILU0 apply
    (equations 3-4 with FP32 factors and arithmetic) may differ, whatever
    their order of operations or fused multiply-adds: twice a first-order
    bound of each against the exact apply of the same rounded data.

    Forward row i (k lower blocks) rounds each entry of its accumulation at
    most 3k + 2 times, so its local error is at most g(3k + 2) (|v_i| +
    sum |L_ij| |y_j|) with g(m) = m u / (1 - m u), u = 2^-24, and errors of
    earlier rows arrive through |L_ij|; the backward sweep does the same with
    |U_ij| and then multiplies by inv(U_ii) (3 more roundings).  Magnitudes
    |y|, |z| are bounded by the same sweeps run on absolute values.  Runs
    in FP64 on the reordered system (rows in sweep order)."""
    n = len(rowptr) - 1
    u = 2.0 ** -24

    def g(m):
        return m * u / (1 - m * u)

    L = np.abs(np.asarray(lu, np.float64))
    D = np.abs(np.asarray(dinv, np.float64))
    av = np.abs(np.asarray(v, np.float64).reshape(n, 3))
    Y = np.zeros((n, 3))
    ey = np.zeros((n, 3))
    for i in range(n):
        acc, err = av[i].copy(), np.zeros(3)
        k = 0
        for p in range(rowptr[i], rowptr[i + 1]):
            j = colidx[p]
            if j < i:
                acc += L[p] @ Y[j]
                err += L[p] @ ey[j]
                k += 1
        Y[i] = acc
        ey[i] = err + g(3 * k + 2) * acc
    Z = np.zeros((n, 3))
    ez = np.zeros((n, 3))
    for i in range(n - 1, -1, -1):
        acc, err = Y[i].copy(), ey[i].copy()
        k = 0
        for p in range(rowptr[i], rowptr[i + 1]):
            j = colidx[p]
            if j > i:
                acc += L[p] @ Z[j]
                err += L[p] @ ez[j]
                k += 1
        Z[i] = D[i] @ acc
        ez[i] = D[i] @ (err + g(3 * k + 2) * acc) + g(3) * Z[i]
    return 2.0 * (1 + 1e-3) * ez


def trajectory_check(gpu_solve, oracle_run, reduction, x_tol, not_converged):
    """GPU BiCGStab against the oracle on the same trajectory, then at a
    reduction.

    gpu_solve(reduction, max_iter) -> (x, status, info of the system);
    oracle_run(reduction, max_iter) -> (x, info, trace) with the oracle's
    per-iteration trace (..., ||s|| at column 3, ..., ||r|| at column 7).

    1. Same trajectory: K full iterations on both sides (K = the oracle's
       iterations to `reduction`; at reduction 0 no test can stop either
       side early): equal status and half steps, x within x_tol, and the
       relative difference of the final residual norms `dev`.
    2. At `reduction`: x within x_tol, and equal half-step counts wherever
       the oracle's residual norms cross the threshold by more than 10 dev
       (the two sides' norms agree to dev); where a norm lies that close to
       the threshold, the GPU's count lies between the first half step whose
       oracle norm is within the band tol (1 + 3 dev) and the first one
       below tol / (1 + 3 dev) (the steps at which a norm within that factor
       of the oracle's can stop), or within two of the oracle's count.
    Returns (dev, decisive)."""
    xo, oinfo, tr = oracle_run(reduction, 200)
    m = oinfo["half_steps"]
    K = max((m + 1) // 2, 1)
    xk, stk, ik = gpu_solve(0.0, K)
    xok, oik, _ = oracle_run(0.0, K)
    assert stk == not_converged and ik["half_steps"] == oik["half_steps"] == 2 * K
    assert np.linalg.norm(xk - xok) <= x_tol * np.linalg.norm(xok)
    dev = abs(ik["final_norm"] - oik["final_norm"]) / oik["final_norm"]
    x, st, info = gpu_solve(reduction, 200)
    assert np.linalg.norm(x - xo) <= x_tol * np.linalg.norm(xo)
    h = []
    for i in range((m + 1) // 2):
        h += [tr[i, 3], tr[i, 7]]
    tol = reduction * oinfo["r0_norm"]
    margin = max(10 * dev, 1e-12)
    decisive = h[m - 1] < tol * (1 - margin) and all(hj > tol * (1 + margin) for hj in h[:m - 1])
    if decisive:
        assert info["half_steps"] == m, (info["half_steps"], m, dev)
    else:
        band = 1 + 3 * dev
        # the oracle's norms past its own stop: its trace of a longer run
        _, _, tr2 = oracle_run(0.0, (m + 1) // 2 + 8)
        h2 = []
        for i in range(tr2.shape[0]):
            h2 += [tr2[i, 3], tr2[i, 7]]
        lo = next((j + 1 for j, hj in enumerate(h2) if hj <= tol * band), len(h2))
        hi = next((j + 1 for j, hj in enumerate(h2) if hj <= tol / band), len(h2))
        ok = lo <= info["half_steps"] <= hi or abs(info["half_steps"] - m) <= 2
        assert ok, (info["half_steps"], m, dev, lo, hi)
    return dev, decisive
