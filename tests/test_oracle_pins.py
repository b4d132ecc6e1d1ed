"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test fixes one part of the oracle with an independent truth: a
hand-derived fixture, exact LU where ILU0 drops no fill, dense triangular
solves, closed-form level/colour counts, Krylov finite-termination, the
minimisation property of the BiCGStab omega step, and the agreement of the
recursive and true residuals.
"""

import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from synth import config_system, make_grid_system
from tests.helpers import (BREAKDOWN_CASES, breakdown_as_well, chain_pattern, dense_pattern, pattern_from_pairs,
                           pattern_set, random_values, read_golden, split_lu, to_dense)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- fixture

def test_golden_two_block_ilu0():
    g = read_golden(os.path.join(GOLDEN, "ilu0_two_block.txt"))
    rowptr, colidx = dense_pattern(2)
    vals = np.stack([g["A00"], g["A01"], g["A10"], g["A11"]])
    st, bad, lu, dinv = oracle.ilu0(rowptr, colidx, vals)
    assert st == oracle.OK and bad == -1
    np.testing.assert_allclose(lu[0], g["A00"], rtol=0, atol=1e-15)   # U00 = A00
    np.testing.assert_allclose(lu[1], g["A01"], rtol=0, atol=1e-15)   # U01 = A01
    np.testing.assert_allclose(lu[2], g["L10"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(lu[3], g["U11"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(dinv[0], g["DINV0"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(dinv[1], g["DINV1"], rtol=0, atol=1e-15)
    x, info = oracle.bicgstab(rowptr, colidx, vals, lu, dinv, g["B"], reduction=1e-12)
    assert info["status"] == oracle.OK and info["half_steps"] == 1
    np.testing.assert_allclose(x.ravel(), g["X"], rtol=0, atol=1e-14)


def _fp32_fixture():
    g = read_golden(os.path.join(GOLDEN, "apply_f32_two_block.txt"))
    rowptr, colidx = dense_pattern(2)
    lu = np.zeros((4, 3, 3))
    lu[1], lu[2] = g["U01"], g["L10"]          # diagonal blocks are not read by the apply
    dinv = np.stack([g["DINV0"], g["DINV1"]])
    return rowptr, colidx, lu, dinv, g["V"].reshape(2, 3), g["Z"].reshape(2, 3)


def _apply_variant(lu, dinv, v, acc_dtype, round_input, fused=False):
    """A deliberately different reading of the FP32 apply on the 2-block
    fixture: products and sums in acc_dtype, the input rounded to FP32 or
    not, or FP32 with fused multiply-adds (every value of this fixture is
    exact in FP64, so rounding the FP64 result once is the fused result)."""
    f32 = np.float32
    L, U, D0, D1 = (m.astype(f32).astype(acc_dtype) for m in (lu[2], lu[1], dinv[0], dinv[1]))
    vv = (v.astype(f32) if round_input else v).astype(acc_dtype)

    def d3(b, x):
        if fused:
            t = f32(np.float64(b[0]) * np.float64(x[0]))
            t = f32(np.float64(b[1]) * np.float64(x[1]) + np.float64(t))
            return f32(np.float64(b[2]) * np.float64(x[2]) + np.float64(t))
        return (b[0] * x[0] + b[1] * x[1]) + b[2] * x[2]

    y0 = vv[0]
    y1 = np.array([vv[1, r] - d3(L[r], y0) for r in range(3)], acc_dtype)
    z1 = np.array([d3(D1[r], y1) for r in range(3)], acc_dtype)
    acc = np.array([y0[r] - d3(U[r], z1) for r in range(3)], acc_dtype)
    z0 = np.array([d3(D0[r], acc) for r in range(3)], acc_dtype)
    return np.stack([z0, z1]).astype(np.float64)


def test_golden_fp32_apply_bit_for_bit():
    """The mixed-precision apply (FP32 factors, FP32 input, every product and
    sum of both sweeps rounded to FP32 in row order) reproduces a fixture
    derived by hand bit for bit; readings that accumulate in FP64, keep the
    input in FP64 or fuse multiply-adds all miss it."""
    rowptr, colidx, lu, dinv, v, z = _fp32_fixture()
    got = oracle.apply_f32(rowptr, colidx, lu, dinv, v)
    assert np.array_equal(got, z)
    for variant in (_apply_variant(lu, dinv, v, np.float64, True), _apply_variant(lu, dinv, v, np.float64, False),
                    _apply_variant(lu, dinv, v, np.float32, True, fused=True)):
        assert not np.array_equal(variant, z)
    assert np.array_equal(_apply_variant(lu, dinv, v, np.float32, True), z)


# ----------------------------------------------------------------- breakdown

@pytest.mark.parametrize("case", sorted(BREAKDOWN_CASES))
def test_bicgstab_breakdown_branches(case):
    """Each breakdown branch of BiCGStab ((rhat, v) = 0, (t, t) = 0,
    omega = 0, rho = 0) on hand-derived exact cases: the status, the half
    steps taken and x (after omega = 0, x keeps x + alpha phat) are exact.
    Unpreconditioned on the 3x3 operator itself, and as the identity with
    one standard well kept separate under ILU0 (the path the GPU runs)."""
    c = BREAKDOWN_CASES[case]
    K = np.asarray(c["K"], np.float64)
    b = np.asarray(c["b"], np.float64)
    rowptr, colidx = np.array([0, 1], np.int32), np.array([0], np.int32)
    x, info = oracle.bicgstab(rowptr, colidx, K[None], None, None, b, precond=oracle.PREC_NONE, reduction=0.1)
    assert info["status"] == oracle.BREAKDOWN and info["half_steps"] == c["half"]
    assert np.array_equal(x.ravel(), np.asarray(c["x"], np.float64))
    rp, ci, vals, wp, pr, B, C, Dinv = breakdown_as_well(K)
    for ordering in (oracle.ORDER_NATURAL, oracle.ORDER_LEVEL):
        xw, iw = oracle.solve(rp, ci, vals[0], b, ordering=ordering, reduction=0.1,
                              wells=(wp, pr, B[0], C[0], Dinv[0]))
        assert iw["status"] == oracle.BREAKDOWN and iw["half_steps"] == c["half"]
        assert np.array_equal(xw.ravel(), np.asarray(c["x"], np.float64))


# --------------------------------------------------------------- validation

def test_validate_errors():
    rowptr, colidx = chain_pattern(4)
    assert oracle.validate(rowptr, colidx) == (oracle.OK, -1)
    c = colidx.copy()
    c[3], c[4] = c[4], c[3]                       # unsorted row 1
    assert oracle.validate(rowptr, c) == (oracle.BAD_PATTERN, 1)
    c = colidx.copy()
    c[4] = c[3]                                   # duplicate in row 1
    assert oracle.validate(rowptr, c)[0] == oracle.BAD_PATTERN
    c = colidx.copy()
    c[-1] = 7                                     # out of range
    assert oracle.validate(rowptr, c) == (oracle.BAD_PATTERN, 3)
    rp, ci = pattern_from_pairs(3, [(0, 1), (1, 2)])
    keep = [p for p in range(len(ci)) if not (ci[p] == 2 and p >= rp[2])]  # drop (2,2)
    rows = np.repeat(np.arange(3), np.diff(rp))[keep]
    rp2 = np.zeros(4, np.int32)
    np.cumsum(np.bincount(rows, minlength=3), out=rp2[1:])
    assert oracle.validate(rp2, ci[keep]) == (oracle.MISSING_DIAG, 2)


# -------------------------------------------------------------- orderings

@pytest.mark.parametrize("shape", [(20, 20, 10), (40, 40, 30), (7, 3, 5), (1, 1, 9)])
def test_level_count_closed_form(shape):
    s = make_grid_system(*shape, seed=1)
    nl, level, perm = oracle.level_sets(s.rowptr, s.colidx)
    assert nl == sum(shape) - 2
    # level of cell (i,j,k) is its Manhattan distance from the origin
    nx, ny, nz = shape
    c = np.arange(nx * ny * nz)
    assert np.array_equal(level, c % nx + (c // nx) % ny + c // (nx * ny))
    assert np.array_equal(np.sort(perm), np.arange(s.n))


def test_level_sets_respect_dependencies():
    s = make_grid_system(12, 10, 6, active_frac=0.8, nnc_frac=0.05, seed=3)
    nl, level, perm = oracle.level_sets(s.rowptr, s.colidx)
    for i in range(s.n):
        for p in range(s.rowptr[i], s.rowptr[i + 1]):
            j = s.colidx[p]
            if j < i:
                assert level[j] < level[i]
    # each row sits one level above its deepest lower dependency
    for i in range(s.n):
        deps = [level[j] for j in s.colidx[s.rowptr[i]:s.rowptr[i + 1]] if j < i]
        assert level[i] == (max(deps) + 1 if deps else 0)
    # stable order inside a level
    assert np.all(np.diff(level[perm]) >= 0)
    for lv in range(nl):
        rows = perm[level[perm] == lv]
        assert np.all(np.diff(rows) > 0)


@pytest.mark.parametrize("shape", [(20, 20, 10), (7, 3, 5), (1, 1, 9), (12, 1, 4)])
def test_rcm_levels_of_a_full_grid(shape):
    """Reverse Cuthill-McKee on a full nx*ny*nz grid starts from cell 0 (a
    corner: fewest neighbours, lowest index), so the breadth-first layers are
    the planes i + j + k = d and every neighbour of a cell sits one layer
    away.  Reversed, each layer precedes the one before it, so a cell's
    lower neighbours are its neighbours one layer further out: its level is
    (nx - 1) + (ny - 1) + (nz - 1) - (i + j + k), and there are
    nx + ny + nz - 2 levels (a chain: its cells in reverse)."""
    nx, ny, nz = shape
    s = make_grid_system(nx, ny, nz, seed=2)
    nl, level, perm = oracle.rcm_levels(s.rowptr, s.colidx)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    d = (i + j + k).transpose(2, 1, 0).ravel()        # cells numbered i fastest
    assert nl == nx + ny + nz - 2
    assert np.array_equal(level, d.max() - d)
    assert np.array_equal(np.sort(perm), np.arange(s.n)) and np.all(np.diff(level[perm]) >= 0)
    if nx == ny == 1:
        assert np.array_equal(perm, np.arange(s.n)[::-1])


@pytest.mark.parametrize("case", ["c1", "grid", "chain", "nnc", "nnc_dense"])
def test_rcm_matches_scipy(case):
    """The Cuthill-McKee part equals scipy's reverse_cuthill_mckee where its
    start rows coincide with this definition's (scipy picks each component's
    start among the rows of fewest neighbours through an unstable sort; on
    these patterns it takes the lowest index): the levels computed on
    scipy's renumbering, rows sorted by (level, position), give the same
    permutation."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    s = {"c1": lambda: config_system("c1"), "grid": lambda: make_grid_system(7, 5, 3, seed=1),
         "chain": lambda: make_grid_system(1, 1, 50, seed=2),
         "nnc": lambda: make_grid_system(17, 13, 9, active_frac=0.85, nnc_frac=0.03, seed=4),
         "nnc_dense": lambda: make_grid_system(30, 20, 10, active_frac=0.9, nnc_frac=0.05, seed=9)}[case]()
    n = s.n
    a = sp.csr_matrix((np.ones(s.nnzb), s.colidx, s.rowptr), shape=(n, n))
    r = reverse_cuthill_mckee(a, symmetric_mode=True)
    pos = np.empty(n, np.int64)
    pos[r] = np.arange(n)
    q = a[r][:, r].tocsr()
    q.sort_indices()
    nl_s, lev_new, _ = oracle.level_sets(q.indptr.astype(np.int32), q.indices.astype(np.int32))
    lev = np.empty(n, np.int64)
    lev[r] = lev_new
    nl, level, perm = oracle.rcm_levels(s.rowptr, s.colidx)
    assert nl == nl_s and np.array_equal(level, lev)
    assert np.array_equal(perm, np.lexsort((pos, lev)))


def test_rcm_levels_respect_dependencies_and_shorten_nnc_schedules():
    """On a masked grid with 2% non-neighbour connections: every row's
    neighbours that precede it in the RCM numbering sit on lower levels,
    and the schedule is far shorter than plain level scheduling's."""
    s = config_system("c2", n_rhs=1)
    nl, level, perm = oracle.rcm_levels(s.rowptr, s.colidx)
    pos = np.empty(s.n, np.int64)
    pos[perm] = np.arange(s.n)
    rows = np.repeat(np.arange(s.n), np.diff(s.rowptr))
    off = rows != s.colidx
    before = pos[s.colidx[off]] < pos[rows[off]]
    assert np.all(level[s.colidx[off]][before] < level[rows[off]][before])
    assert nl < oracle.level_sets(s.rowptr, s.colidx)[0] / 20


@pytest.mark.parametrize("shape", [(20, 20, 10), (5, 6, 7)])
def test_dsatur_full_grid_is_red_black(shape):
    """DSatur colours a bipartite graph with two colours (Brelaz 1979); the
    first row coloured is the lowest-index row of highest degree, interior
    cell (1, 1, 1), so colour 0 is the odd parity class."""
    s = make_grid_system(*shape, seed=2)
    nc, col, perm = oracle.dsatur_colour(s.rowptr, s.colidx)
    assert nc == 2
    nx, ny, _ = shape
    c = np.arange(s.n)
    assert np.array_equal(col, 1 - (c % nx + (c // nx) % ny + c // (nx * ny)) % 2)
    assert np.array_equal(perm, np.argsort(col, kind="stable"))


def _ring(m, first=0):
    return [(first + k, first + (k + 1) % m) for k in range(m)]


@pytest.mark.parametrize("m", [4, 5, 6, 7, 12, 13])
def test_dsatur_cycles_and_wheels(m):
    """Closed forms DSatur reaches exactly: a cycle needs 2 colours when even
    and 3 when odd; a wheel (hub joined to every row of a cycle) one more."""
    rp, ci = pattern_from_pairs(m, _ring(m))
    assert oracle.dsatur_colour(rp, ci)[0] == (2 if m % 2 == 0 else 3)
    rp, ci = pattern_from_pairs(m + 1, _ring(m, 1) + [(0, k) for k in range(1, m + 1)])
    nc, col, _ = oracle.dsatur_colour(rp, ci)
    assert nc == (3 if m % 2 == 0 else 4) and col[0] == 0   # the hub has the highest degree


@pytest.mark.parametrize("m", [1, 2, 5, 9])
def test_dsatur_complete_graph(m):
    """K_m needs m colours; with every degree equal, rows go in index order."""
    rp, ci = dense_pattern(m)
    nc, col, perm = oracle.dsatur_colour(rp, ci)
    assert nc == m and np.array_equal(col, np.arange(m)) and np.array_equal(perm, np.arange(m))


@pytest.mark.parametrize("k", [3, 6, 10])
def test_dsatur_crown_graph_two_colours(k):
    """Crown graph (u_i ~ w_j for i != j), rows interleaved u0, w0, u1, w1 ...:
    first-fit in natural order needs k colours on it, DSatur two."""
    pairs = [(2 * i, 2 * j + 1) for i in range(k) for j in range(k) if i != j]
    rp, ci = pattern_from_pairs(2 * k, pairs)
    nc, col, _ = oracle.dsatur_colour(rp, ci)
    assert nc == 2
    assert np.all(col[0::2] == col[0]) and np.all(col[1::2] == 1 - col[0])


def test_dsatur_is_proper_on_nnc_pattern():
    s = make_grid_system(14, 12, 8, active_frac=0.85, nnc_frac=0.02, seed=5)
    nc, col, perm = oracle.dsatur_colour(s.rowptr, s.colidx)
    maxdeg = 0
    for i in range(s.n):
        nbr = [j for j in s.colidx[s.rowptr[i]:s.rowptr[i + 1]] if j != i]
        maxdeg = max(maxdeg, len(nbr))
        for j in nbr:
            assert col[i] != col[j]
        # each row took the lowest colour free when it was coloured, and its
        # neighbours keep their colours: it touches every colour below its own
        assert set(range(col[i])) <= {col[j] for j in nbr}
    assert nc <= maxdeg + 1
    assert np.array_equal(perm, np.argsort(col, kind="stable"))


def test_permute_is_similarity():
    s = make_grid_system(6, 5, 4, active_frac=0.9, nnc_frac=0.05, seed=7)
    vals = s.vals[0]
    rng = np.random.default_rng(0)
    perm = rng.permutation(s.n).astype(np.int32)
    prow, pcol, pv = oracle.permute(s.rowptr, s.colidx, vals, perm)
    assert oracle.validate(prow, pcol)[0] == oracle.OK
    P = np.zeros((3 * s.n, 3 * s.n))
    for new, old in enumerate(perm):
        P[3 * new:3 * new + 3, 3 * old:3 * old + 3] = np.eye(3)
    A = to_dense(s.rowptr, s.colidx, vals)
    assert np.array_equal(to_dense(prow, pcol, pv), P @ A @ P.T)


# --------------------------------------------------------------------- ILU0

@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_ilu0_dense_pattern_is_exact_lu(n):
    rowptr, colidx = dense_pattern(n)
    vals = random_values(rowptr, colidx, seed=n)
    st, _, lu, dinv = oracle.ilu0(rowptr, colidx, vals)
    assert st == oracle.OK
    L, U = split_lu(rowptr, colidx, lu)
    A = to_dense(rowptr, colidx, vals)
    assert np.linalg.norm(L @ U - A) / np.linalg.norm(A) < 1e-14
    for i in range(n):
        d = i * n + i
        np.testing.assert_allclose(dinv[i] @ lu[d], np.eye(3), atol=1e-13)


def test_ilu0_chain_is_exact_lu():
    rowptr, colidx = chain_pattern(30)
    vals = random_values(rowptr, colidx, seed=11, diag_boost=1.0)
    st, _, lu, _ = oracle.ilu0(rowptr, colidx, vals)
    assert st == oracle.OK
    L, U = split_lu(rowptr, colidx, lu)
    A = to_dense(rowptr, colidx, vals)
    assert np.linalg.norm(L @ U - A) / np.linalg.norm(A) < 1e-14


@pytest.mark.parametrize("case", ["c1", "nnc"])
def test_ilu0_reproduces_a_on_pattern(case):
    if case == "c1":
        s = config_system("c1")
    else:
        s = make_grid_system(10, 9, 6, active_frac=0.85, nnc_frac=0.05, seed=4)
    vals = s.vals[0]
    st, _, lu, _ = oracle.ilu0(s.rowptr, s.colidx, vals)
    assert st == oracle.OK
    L, U = split_lu(s.rowptr, s.colidx, lu)
    LU = L @ U
    A = to_dense(s.rowptr, s.colidx, vals)
    mask = np.zeros_like(A, dtype=bool)
    for (i, j) in pattern_set(s.rowptr, s.colidx):
        mask[3 * i:3 * i + 3, 3 * j:3 * j + 3] = True
    err = np.abs(LU - A)[mask].max() / np.abs(A).max()
    assert err < 1e-14
    # and the factorisation is incomplete: fill outside S is dropped
    if case == "nnc":
        assert np.abs(LU - A)[~mask].max() > 1e-6


def test_ilu0_kij_equals_ikj_bitwise():
    s = make_grid_system(9, 8, 5, active_frac=0.85, nnc_frac=0.08, seed=9)
    st1, _, lu1, d1 = oracle.ilu0(s.rowptr, s.colidx, s.vals[0])
    st2, _, lu2, d2 = oracle.ilu0(s.rowptr, s.colidx, s.vals[0], kij=True)
    assert st1 == st2 == oracle.OK
    assert np.array_equal(lu1, lu2) and np.array_equal(d1, d2)


def test_ilu0_level_order_invariance():
    s = config_system("c1")
    vals = s.vals[0]
    _, _, perm = oracle.level_sets(s.rowptr, s.colidx)
    prow, pcol, pv = oracle.permute(s.rowptr, s.colidx, vals, perm)
    _, _, lu, dinv = oracle.ilu0(s.rowptr, s.colidx, vals)
    _, _, plu, pdinv = oracle.ilu0(prow, pcol, pv)
    q_lu = oracle.permute(s.rowptr, s.colidx, lu, perm)[2]
    assert np.abs(q_lu - plu).max() <= 1e-14 * np.abs(lu).max()
    assert np.abs(dinv[perm] - pdinv).max() <= 1e-14 * np.abs(dinv).max()


def test_ilu0_zero_pivot_reports_row():
    rowptr, colidx = chain_pattern(5)
    vals = random_values(rowptr, colidx, seed=1)
    vals[rowptr[3] + 1] = 0.0           # diagonal block of row 3 (row 3 has cols 2,3,4)
    vals[rowptr[3]] = 0.0               # and no incoming update
    st, bad, _, _ = oracle.ilu0(rowptr, colidx, vals)
    assert (st, bad) == (oracle.ZERO_PIVOT, 3)


def test_inv3_matches_linalg():
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = rng.standard_normal((3, 3))
        ok, inv = oracle.inv3(a)
        assert ok
        np.testing.assert_allclose(inv, np.linalg.inv(a), rtol=1e-12, atol=1e-12)
    assert oracle.inv3(np.ones((3, 3)))[0] == 0


# -------------------------------------------------------------------- apply

def test_apply_equals_dense_triangular_solves():
    s = make_grid_system(6, 5, 4, active_frac=0.85, nnc_frac=0.05, seed=12)
    vals = s.vals[0]
    _, _, lu, dinv = oracle.ilu0(s.rowptr, s.colidx, vals)
    L, U = split_lu(s.rowptr, s.colidx, lu)
    v = np.random.default_rng(1).standard_normal((s.n, 3))
    z = oracle.apply(s.rowptr, s.colidx, lu, dinv, v)
    # L is unit lower triangular also entrywise; U is only block upper
    # triangular (full 3x3 diagonal blocks), so it takes a general solve
    y = sla.solve_triangular(L, v.ravel(), lower=True, unit_diagonal=True)
    zr = np.linalg.solve(U, y)
    assert np.linalg.norm(z.ravel() - zr) / np.linalg.norm(zr) < 1e-13


def test_apply_on_chain_is_exact_inverse():
    rowptr, colidx = chain_pattern(25)
    vals = random_values(rowptr, colidx, seed=4, diag_boost=1.0)
    _, _, lu, dinv = oracle.ilu0(rowptr, colidx, vals)
    v = np.random.default_rng(2).standard_normal((25, 3))
    z = oracle.apply(rowptr, colidx, lu, dinv, v)
    A = to_dense(rowptr, colidx, vals)
    assert np.linalg.norm(A @ z.ravel() - v.ravel()) / np.linalg.norm(v) < 1e-13


def test_apply_f32_close_to_f64():
    s = config_system("c1")
    _, _, lu, dinv = oracle.ilu0(s.rowptr, s.colidx, s.vals[0])
    v = np.random.default_rng(5).standard_normal((s.n, 3))
    z64 = oracle.apply(s.rowptr, s.colidx, lu, dinv, v)
    z32 = oracle.apply_f32(s.rowptr, s.colidx, lu, dinv, v)
    rel = np.linalg.norm(z32 - z64) / np.linalg.norm(z64)
    assert 0 < rel < 1e-5


def test_spmv_matches_dense():
    s = make_grid_system(5, 4, 3, active_frac=0.9, nnc_frac=0.1, seed=8)
    x = np.random.default_rng(0).standard_normal((s.n, 3))
    y = oracle.spmv(s.rowptr, s.colidx, s.vals[0], x)
    yr = to_dense(s.rowptr, s.colidx, s.vals[0]) @ x.ravel()
    np.testing.assert_allclose(y.ravel(), yr, rtol=1e-13, atol=1e-13)


# ----------------------------------------------------------------- BiCGStab

def _dense_with_spectrum(eigs, seed):
    """A dense 3n x 3n matrix (as a full block pattern) with the given eigenvalues."""
    n3 = len(eigs)
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((n3, n3)) + 3 * np.eye(n3)
    A = S @ np.diag(eigs) @ np.linalg.inv(S)
    n = n3 // 3
    rowptr, colidx = dense_pattern(n)
    vals = np.stack([A[3 * i:3 * i + 3, 3 * j:3 * j + 3] for i in range(n) for j in range(n)])
    return rowptr, colidx, vals, A


@pytest.mark.parametrize("k,half", [(1, 1), (2, 3), (3, 5)])
def test_bicgstab_finite_termination(k, half):
    """Unpreconditioned BiCGStab on a matrix with k distinct eigenvalues: the
    BiCG polynomial of degree k annihilates r0, so s vanishes at the half step
    of iteration k (2k-1 half steps) with the exact solution."""
    eigs = np.repeat([1.0, 2.5, -1.7][:k], [4, 3, 2][:k] if k > 1 else [9])
    eigs = np.resize(eigs, 9)
    rowptr, colidx, vals, A = _dense_with_spectrum(eigs, seed=k)
    b = np.random.default_rng(10 + k).standard_normal(9)
    x, info = oracle.bicgstab(rowptr, colidx, vals, None, None, b, precond=oracle.PREC_NONE,
                              reduction=1e-9, max_iter=20)
    assert info["status"] == oracle.OK
    assert info["half_steps"] == half
    np.testing.assert_allclose(x.ravel(), np.linalg.solve(A, b), rtol=1e-8, atol=1e-8)


def test_bicgstab_exact_preconditioner_half_step():
    rowptr, colidx = chain_pattern(40)
    vals = random_values(rowptr, colidx, seed=6, diag_boost=1.0)
    _, _, lu, dinv = oracle.ilu0(rowptr, colidx, vals)
    b = np.random.default_rng(7).standard_normal((40, 3))
    x, info = oracle.bicgstab(rowptr, colidx, vals, lu, dinv, b, reduction=1e-10)
    assert info["status"] == oracle.OK and info["half_steps"] == 1
    A = to_dense(rowptr, colidx, vals)
    np.testing.assert_allclose(x.ravel(), np.linalg.solve(A, b.ravel()), rtol=1e-12, atol=1e-12)


def test_bicgstab_omega_minimises_and_residuals_agree():
    s = make_grid_system(8, 7, 5, sigma=2.0, active_frac=0.9, nnc_frac=0.03, seed=13)
    vals = s.vals[0]
    _, _, lu, dinv = oracle.ilu0(s.rowptr, s.colidx, vals)
    b = s.b[0, 0]
    kmax = 6
    _, _, tr = oracle.bicgstab(s.rowptr, s.colidx, vals, lu, dinv, b, reduction=1e-30, max_iter=kmax,
                               trace=True)
    A = to_dense(s.rowptr, s.colidx, vals)
    for it in range(kmax):
        rho, rv, alpha, snorm, ts, tt, omega, rnorm = tr[it]
        # omega = argmin ||s - w t||: the minimum is ||s||^2 - (t,s)^2/(t,t)
        assert abs(rnorm ** 2 - (snorm ** 2 - ts ** 2 / tt)) <= 1e-9 * snorm ** 2
        assert rnorm <= snorm * (1 + 1e-12)
        # the recursively updated residual is the true residual of the iterate
        xk, info = oracle.bicgstab(s.rowptr, s.colidx, vals, lu, dinv, b, reduction=1e-30, max_iter=it + 1)
        assert info["status"] == oracle.NOT_CONVERGED and info["half_steps"] == 2 * (it + 1)
        true = np.linalg.norm(b.ravel() - A @ xk.ravel())
        assert abs(true - rnorm) <= 1e-10 * np.linalg.norm(b)


def test_bicgstab_dense_solve_tight():
    s = make_grid_system(10, 10, 5, seed=21)
    A = to_dense(s.rowptr, s.colidx, s.vals[0])
    b = s.b[0, 0]
    xr = np.linalg.solve(A, b.ravel())
    for ordering in (oracle.ORDER_NATURAL, oracle.ORDER_LEVEL, oracle.ORDER_COLOUR):
        x, info = oracle.solve(s.rowptr, s.colidx, s.vals[0], b, ordering=ordering, reduction=1e-12)
        assert info["status"] == oracle.OK
        assert info["true_rel_residual"] <= 1e-11
        assert np.linalg.norm(x.ravel() - xr) / np.linalg.norm(xr) < 1e-9


@pytest.mark.parametrize("precond", [oracle.PREC_ILU_F64, oracle.PREC_ILU_F32])
@pytest.mark.parametrize("red", [1e-2, 1e-6])
def test_solve_meets_reduction(precond, red):
    s = config_system("c1")
    x, info = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=oracle.ORDER_LEVEL,
                           precond=precond, reduction=red)
    assert info["status"] == oracle.OK
    assert info["final_norm"] <= red * info["r0_norm"]
    assert info["true_rel_residual"] <= red * (1 + 1e-6)


def test_mixed_and_fp64_iteration_counts_close():
    s = config_system("c1")
    h = []
    for precond in (oracle.PREC_ILU_F64, oracle.PREC_ILU_F32):
        _, info = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=oracle.ORDER_LEVEL,
                               precond=precond, reduction=1e-6)
        h.append(info["half_steps"])
    assert abs(h[0] - h[1]) <= 2


def test_stopping_and_fault_statuses():
    s = config_system("c1")
    vals, b = s.vals[0], s.b[0, 0]
    _, info = oracle.solve(s.rowptr, s.colidx, vals, b, reduction=1e-12, max_iter=1)
    assert info["status"] == oracle.NOT_CONVERGED and info["half_steps"] == 2
    x, info = oracle.solve(s.rowptr, s.colidx, vals, np.zeros_like(b))
    assert info["status"] == oracle.OK and info["half_steps"] == 0 and not x.any()
    bn = b.copy()
    bn[5, 1] = np.nan
    _, info = oracle.solve(s.rowptr, s.colidx, vals, bn)
    assert info["status"] == oracle.NON_FINITE
    vz = vals.copy()
    row = 17
    for p in range(s.rowptr[row], s.rowptr[row + 1]):
        if s.colidx[p] == row:
            vz[p] = 0.0
        elif s.colidx[p] < row:
            vz[p] = 0.0   # no update reaches the zeroed diagonal
    _, info = oracle.solve(s.rowptr, s.colidx, vz, b)
    assert info["status"] == oracle.ZERO_PIVOT and info["bad_row"] == row


# ------------------------------------------------------------ Block-Jacobi

def slab_partition(n, parts):
    """Contiguous row ranges of near-equal size (z-slabs of a grid numbered i, j, k)."""
    return (np.arange(n, dtype=np.int64) * parts // max(n, 1)).astype(np.int32)


def test_jacobi_matrix_keeps_exactly_the_blocks_inside_partitions():
    s = make_grid_system(6, 5, 4, nnc_frac=0.05, seed=31)
    part = np.random.default_rng(3).integers(0, 3, s.n).astype(np.int32)
    rrow, rcol, rv = oracle.jacobi_matrix(s.rowptr, s.colidx, s.vals[0], part)
    kept = []
    for i in range(s.n):                      # brute force over every stored block
        for p in range(s.rowptr[i], s.rowptr[i + 1]):
            if part[i] == part[s.colidx[p]]:
                kept.append((i, s.colidx[p], p))
    got = [(i, rcol[q]) for i in range(s.n) for q in range(rrow[i], rrow[i + 1])]
    assert got == [(i, j) for i, j, _ in kept]
    assert np.array_equal(rv, s.vals[0][[p for _, _, p in kept]])


def test_jacobi_with_one_partition_is_plain_ilu0():
    s = make_grid_system(8, 6, 5, nnc_frac=0.03, seed=32)
    for ordering in (oracle.ORDER_NATURAL, oracle.ORDER_LEVEL, oracle.ORDER_COLOUR):
        x1, i1 = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering, reduction=1e-10)
        x2, i2 = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering, reduction=1e-10,
                              part=np.zeros(s.n, np.int32))
        assert np.array_equal(x1, x2) and i1["half_steps"] == i2["half_steps"]


def test_jacobi_on_uncoupled_partitions_is_plain_ilu0():
    """A matrix with no blocks between partitions loses nothing to the Jacobi matrix."""
    a = make_grid_system(6, 5, 4, seed=33)
    b = make_grid_system(5, 4, 3, nnc_frac=0.05, seed=34)
    rowptr = np.concatenate([a.rowptr, b.rowptr[1:] + a.rowptr[-1]]).astype(np.int32)
    colidx = np.concatenate([a.colidx, b.colidx + a.n]).astype(np.int32)
    vals = np.concatenate([a.vals[0], b.vals[0]])
    rhs = np.concatenate([a.b[0, 0], b.b[0, 0]])
    part = np.concatenate([np.zeros(a.n), np.ones(b.n)]).astype(np.int32)
    for ordering in (oracle.ORDER_LEVEL, oracle.ORDER_COLOUR):
        x1, i1 = oracle.solve(rowptr, colidx, vals, rhs, ordering=ordering, reduction=1e-10)
        x2, i2 = oracle.solve(rowptr, colidx, vals, rhs, ordering=ordering, reduction=1e-10, part=part)
        assert np.array_equal(x1, x2) and i1["half_steps"] == i2["half_steps"]


def test_jacobi_factors_split_into_independent_partitions():
    """ILU0 of the Jacobi matrix restricted to one partition equals ILU0 of
    that partition's diagonal sub-matrix factored on its own."""
    s = make_grid_system(7, 6, 5, nnc_frac=0.04, seed=35)
    part = slab_partition(s.n, 3)
    rrow, rcol, rv = oracle.jacobi_matrix(s.rowptr, s.colidx, s.vals[0], part)
    st, _, lu, dinv = oracle.ilu0(rrow, rcol, rv)
    assert st == oracle.OK
    for q in range(3):
        rows = np.flatnonzero(part == q)
        local = {int(r): k for k, r in enumerate(rows)}
        sp, sc, sv, pos = [0], [], [], []
        for r in rows:                               # the sub-matrix A[P, P], built here from A
            for p in range(s.rowptr[r], s.rowptr[r + 1]):
                if int(s.colidx[p]) in local:
                    sc.append(local[int(s.colidx[p])])
                    sv.append(s.vals[0][p])
            sp.append(len(sc))
        for r in rows:                               # the same blocks' positions in the Jacobi matrix
            pos.extend(range(rrow[r], rrow[r + 1]))
        st2, _, lu2, dinv2 = oracle.ilu0(np.asarray(sp, np.int32), np.asarray(sc, np.int32), np.asarray(sv))
        assert st2 == oracle.OK
        assert np.array_equal(lu[pos], lu2) and np.array_equal(dinv[rows], dinv2)


def test_jacobi_one_row_per_partition_is_block_diagonal():
    s = make_grid_system(6, 5, 4, seed=36)
    part = np.arange(s.n, dtype=np.int32)
    rrow, rcol, rv = oracle.jacobi_matrix(s.rowptr, s.colidx, s.vals[0], part)
    assert np.array_equal(rcol, np.arange(s.n)) and np.array_equal(rrow, np.arange(s.n + 1))
    st, _, lu, dinv = oracle.ilu0(rrow, rcol, rv)
    diag = np.array([s.vals[0][p] for i in range(s.n) for p in range(s.rowptr[i], s.rowptr[i + 1])
                     if s.colidx[p] == i])
    assert np.allclose(dinv, np.linalg.inv(diag), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("parts", [2, 5, 17])
def test_jacobi_solve_converges_to_the_full_system(parts):
    """The SpMV keeps the full matrix: the solution is that of A, not of the Jacobi matrix."""
    s = make_grid_system(10, 8, 6, nnc_frac=0.03, seed=37)
    A = to_dense(s.rowptr, s.colidx, s.vals[0])
    b = s.b[0, 0]
    xr = np.linalg.solve(A, b.ravel())
    part = slab_partition(s.n, parts)
    for ordering in (oracle.ORDER_LEVEL, oracle.ORDER_COLOUR):
        x, info = oracle.solve(s.rowptr, s.colidx, s.vals[0], b, ordering=ordering, reduction=1e-12, part=part)
        assert info["status"] == oracle.OK and info["true_rel_residual"] <= 1e-11
        assert np.linalg.norm(x.ravel() - xr) / np.linalg.norm(xr) < 1e-9


def test_jacobi_levels_shrink_with_slabs():
    """Cutting a grid into z-slabs leaves the level count of the thickest slab."""
    nx, ny, nz = 7, 6, 12
    s = make_grid_system(nx, ny, nz, seed=38)
    part = (np.arange(s.n) // (nx * ny * 3)).astype(np.int32)       # 4 slabs of 3 layers
    _, info = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=oracle.ORDER_LEVEL, part=part)
    assert info["n_sets"] == nx + ny + 3 - 2


# ------------------------------------------------------------------- wells

def coupled_dense(s, w, k=0):
    """A - sum_w C_w^T D_w^-1 B_w as a dense matrix (Algorithm 4), built here from the blocks."""
    A = to_dense(s.rowptr, s.colidx, s.vals[k])
    for q in range(w.n_wells):
        Bw = np.zeros((4, 3 * s.n))
        Cw = np.zeros((4, 3 * s.n))
        for p in range(w.well_ptr[q], w.well_ptr[q + 1]):
            r = w.perf_row[p]
            Bw[:, 3 * r:3 * r + 3] += w.B[k, p]
            Cw[:, 3 * r:3 * r + 3] += w.C[k, p]
        A -= Cw.T @ w.Dinv[k, q] @ Bw
    return A


def test_separate_wells_equal_wells_in_the_matrix():
    """Algorithm 5 (wells applied after the SpMV) equals Algorithm 4 (wells folded into A)."""
    from synth import make_wells
    s = make_grid_system(7, 6, 5, active_frac=0.9, seed=41)
    w = make_wells(s, 4, seed=42)
    x = np.random.default_rng(43).standard_normal((s.n, 3))
    y = oracle.wells_apply(w.well_ptr, w.perf_row, w.B[0], w.C[0], w.Dinv[0], x,
                           oracle.spmv(s.rowptr, s.colidx, s.vals[0], x))
    ref = coupled_dense(s, w) @ x.ravel()
    assert np.abs(y.ravel() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_solve_with_wells_converges_to_the_coupled_system():
    from synth import make_wells
    s = make_grid_system(9, 7, 6, nnc_frac=0.03, seed=44)
    w = make_wells(s, 5, seed=45)
    xr = np.linalg.solve(coupled_dense(s, w), s.b[0, 0].ravel())
    for ordering in (oracle.ORDER_NATURAL, oracle.ORDER_LEVEL, oracle.ORDER_COLOUR):
        x, info = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering, reduction=1e-12,
                               wells=(w.well_ptr, w.perf_row, w.B[0], w.C[0], w.Dinv[0]))
        assert info["status"] == oracle.OK and info["true_rel_residual"] <= 1e-11
        assert np.linalg.norm(x.ravel() - xr) / np.linalg.norm(xr) < 1e-9


def test_no_wells_is_plain():
    s = make_grid_system(6, 5, 4, seed=46)
    empty = (np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros((0, 4, 3)), np.zeros((0, 4, 3)),
             np.zeros((0, 4, 4)))
    x1, i1 = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=oracle.ORDER_LEVEL, reduction=1e-10)
    x2, i2 = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=oracle.ORDER_LEVEL, reduction=1e-10,
                          wells=empty)
    assert np.array_equal(x1, x2) and i1["half_steps"] == i2["half_steps"]


# ------------------------------------------------------------------- GMRES

def test_gmres_estimate_is_the_minimal_residual_over_the_krylov_space():
    """After k steps |g_k| equals ||b - A x_k|| of the returned iterate, and
    that is the least-squares minimum over the Krylov space of A M^-1 (brute
    force with dense matrices)."""
    s = make_grid_system(5, 4, 3, seed=61)
    n3 = 3 * s.n
    st, _, lu, dinv = oracle.ilu0(s.rowptr, s.colidx, s.vals[0])
    A = to_dense(s.rowptr, s.colidx, s.vals[0])
    Minv = np.column_stack([oracle.apply(s.rowptr, s.colidx, lu, dinv, e.reshape(-1, 3)).ravel()
                            for e in np.eye(n3)])
    AM = A @ Minv
    b = s.b[0, 0].ravel()
    prev = np.inf
    for k in range(1, 6):
        x, info, tr = oracle.gmres(s.rowptr, s.colidx, s.vals[0], lu, dinv, b, restart=30, reduction=0.0,
                                   max_iter=k, trace=True)
        assert info["half_steps"] == k and len(tr) == k
        true = np.linalg.norm(b - A @ x.ravel())
        assert abs(true - tr[-1]) <= 1e-10 * np.linalg.norm(b)
        K = np.column_stack([np.linalg.matrix_power(AM, i) @ b for i in range(k)])
        c, *_ = np.linalg.lstsq(AM @ K, b, rcond=None)
        best = np.linalg.norm(b - AM @ K @ c)
        assert abs(best - tr[-1]) <= 1e-8 * np.linalg.norm(b)
        assert tr[-1] <= prev * (1 + 1e-12)          # minimal residual: never grows within a cycle
        prev = tr[-1]


def test_gmres_finite_termination_with_three_eigenvalues():
    """Unpreconditioned GMRES on a matrix with three distinct eigenvalues
    (diagonal blocks diag(1, 2, 3)) is exact after three steps."""
    n = 10
    rowptr, colidx = chain_pattern(n)
    vals = np.zeros((len(colidx), 3, 3))
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            if colidx[p] == i:
                vals[p] = np.diag([1.0, 2.0, 3.0])
    b = np.random.default_rng(62).standard_normal((n, 3))
    x, info = oracle.gmres(rowptr, colidx, vals, None, None, b, precond=oracle.PREC_NONE, restart=30,
                           reduction=1e-14, max_iter=10)
    assert info["status"] == oracle.OK and info["half_steps"] == 3
    assert np.allclose(x, b / np.array([1.0, 2.0, 3.0]), rtol=1e-13, atol=0)


def test_gmres_exact_preconditioner_one_step():
    rowptr, colidx = chain_pattern(12)
    vals = random_values(rowptr, colidx, seed=63)
    st, _, lu, dinv = oracle.ilu0(rowptr, colidx, vals)
    b = np.random.default_rng(64).standard_normal((12, 3))
    x, info = oracle.gmres(rowptr, colidx, vals, lu, dinv, b, restart=30, reduction=1e-12, max_iter=10)
    assert info["status"] == oracle.OK and info["half_steps"] == 1
    A = to_dense(rowptr, colidx, vals)
    assert np.linalg.norm(A @ x.ravel() - b.ravel()) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("restart", [2, 30])
def test_gmres_dense_solve(restart):
    s = make_grid_system(10, 8, 6, nnc_frac=0.03, seed=65)
    A = to_dense(s.rowptr, s.colidx, s.vals[0])
    xr = np.linalg.solve(A, s.b[0, 0].ravel())
    for ordering in (oracle.ORDER_NATURAL, oracle.ORDER_LEVEL, oracle.ORDER_COLOUR):
        x, info = oracle.solve_gmres(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering, restart=restart,
                                     reduction=1e-12, max_iter=500)
        assert info["status"] == oracle.OK and info["true_rel_residual"] <= 1e-11
        assert np.linalg.norm(x.ravel() - xr) / np.linalg.norm(xr) < 1e-9


def test_gmres_restart_one_is_the_minimal_residual_iteration():
    """GMRES(1) restarts after every step from the explicit residual, so it is
    the preconditioned minimal residual iteration x += a M^-1 r with
    a = (A M^-1 r, r) / ||A M^-1 r||^2 (written out with dense matrices)."""
    s = make_grid_system(5, 4, 3, seed=66)
    n3 = 3 * s.n
    st, _, lu, dinv = oracle.ilu0(s.rowptr, s.colidx, s.vals[0])
    A = to_dense(s.rowptr, s.colidx, s.vals[0])
    Minv = np.column_stack([oracle.apply(s.rowptr, s.colidx, lu, dinv, e.reshape(-1, 3)).ravel()
                            for e in np.eye(n3)])
    b = s.b[0, 0].ravel()
    xr = np.zeros(n3)
    for k in range(1, 7):
        r = b - A @ xr
        q = A @ (Minv @ r)
        xr = xr + (q @ r) / (q @ q) * (Minv @ r)
        x, info = oracle.gmres(s.rowptr, s.colidx, s.vals[0], lu, dinv, b, restart=1, reduction=0.0, max_iter=k)
        assert info["half_steps"] == k
        assert np.linalg.norm(x.ravel() - xr) <= 1e-11 * np.linalg.norm(xr)
        assert abs(info["final_norm"] - np.linalg.norm(b - A @ xr)) <= 1e-10 * np.linalg.norm(b)


def test_gmres_no_steps():
    s = make_grid_system(4, 3, 2, seed=67)
    st, _, lu, dinv = oracle.ilu0(s.rowptr, s.colidx, s.vals[0])
    x, info = oracle.gmres(s.rowptr, s.colidx, s.vals[0], lu, dinv, s.b[0, 0], restart=5, max_iter=0)
    assert info["status"] == oracle.NOT_CONVERGED and info["half_steps"] == 0 and not x.any()
    x, info = oracle.gmres(s.rowptr, s.colidx, s.vals[0], lu, dinv, np.zeros((s.n, 3)), restart=5, max_iter=10)
    assert info["status"] == oracle.OK and info["half_steps"] == 0 and not x.any()


@pytest.mark.parametrize("restart", [3, 30])
def test_gmres_with_wells_converges_to_the_coupled_system(restart):
    """GMRES with standard wells kept separate solves the coupled system
    A - sum_w C_w^T D_w^-1 B_w (dense, Algorithm 4) for every ordering, and
    its first step's estimate is the minimal residual over span{b} of that
    operator times M^-1 (so the wells enter the Arnoldi products)."""
    from synth import make_wells
    s = make_grid_system(9, 7, 6, nnc_frac=0.03, seed=68)
    w = make_wells(s, 5, seed=69)
    wells = (w.well_ptr, w.perf_row, w.B[0], w.C[0], w.Dinv[0])
    Ac = coupled_dense(s, w)
    b = s.b[0, 0].ravel()
    xr = np.linalg.solve(Ac, b)
    for ordering in (oracle.ORDER_NATURAL, oracle.ORDER_LEVEL, oracle.ORDER_COLOUR):
        x, info = oracle.solve_gmres(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering, restart=restart,
                                     reduction=1e-12, max_iter=2000, wells=wells)
        assert info["status"] == oracle.OK and info["true_rel_residual"] <= 1e-11
        assert np.linalg.norm(x.ravel() - xr) / np.linalg.norm(xr) < 1e-9
    st, _, lu, dinv = oracle.ilu0(s.rowptr, s.colidx, s.vals[0])
    Minv = np.column_stack([oracle.apply(s.rowptr, s.colidx, lu, dinv, e.reshape(-1, 3)).ravel()
                            for e in np.eye(3 * s.n)])
    q = Ac @ (Minv @ b)
    best = np.linalg.norm(b - (q @ b) / (q @ q) * q)
    _, info = oracle.gmres(s.rowptr, s.colidx, s.vals[0], lu, dinv, b, restart=restart, reduction=0.0, max_iter=1,
                           wells=wells)
    assert abs(info["final_norm"] - best) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("case", ["c1", "nnc"])
@pytest.mark.parametrize("ordering", [oracle.ORDER_NATURAL, oracle.ORDER_LEVEL, oracle.ORDER_COLOUR])
def test_fp32_apply_within_its_error_bound(case, ordering):
    """The FP32 apply stays within the first-order FP32 error bound of the
    exact apply of the same rounded factors and input (computed here in
    FP64): the bound the GPU's FP32 apply is held to as well."""
    from tests.helpers import fp32_apply_bound
    s = config_system("c1") if case == "c1" else make_grid_system(17, 13, 9, active_frac=0.85, nnc_frac=0.03,
                                                                  seed=4, sigma=2.0)
    perm = oracle.ordering_perm(s.rowptr, s.colidx, ordering)
    prow, pcol, pv = oracle.permute(s.rowptr, s.colidx, s.vals[0], perm)
    _, _, lu, dinv = oracle.ilu0(prow, pcol, pv)
    v = np.random.default_rng(3).standard_normal((s.n, 3))
    r32 = [a.astype(np.float32).astype(np.float64) for a in (lu, dinv, v)]
    z32 = oracle.apply_f32(prow, pcol, lu, dinv, v)
    exact = oracle.apply(prow, pcol, *r32)
    assert np.all(np.abs(z32 - exact) <= fp32_apply_bound(prow, pcol, *r32) / 2)
    assert not np.array_equal(z32, exact)
