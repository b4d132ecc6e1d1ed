"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances: ILU0 factors within 1e-12 relative (per block row, max-norm of
the difference over the max-norm of the factor) under the same ordering;
solutions within 1e-8 relative 2-norm at a reduction of 1e-10 with equal
half-step counts.  SpMV and the preconditioner apply have no stated bound:
both sides sum the same terms in the same order, the GPU contracting
multiply-adds into FMAs, so each entry may differ by a few units of
eps * (|A| |x|)_i; the tests allow 1e-13 of that.
"""

import numpy as np
import pytest

import oracle
import paper_2309_11488_amd as rs
from synth import config_system, make_ensemble, make_grid_system
from tests.helpers import (BREAKDOWN_CASES, breakdown_as_well, chain_pattern, dense_pattern,
                           fp32_apply_bound, outcome, random_values, trajectory_check)

pytestmark = pytest.mark.gpu

ORDERINGS = [rs.ORDER_NATURAL, rs.ORDER_LEVEL_SET, rs.ORDER_GRAPH_COLOUR, rs.ORDER_RCM_LEVEL_SET]


def cases():
    out = {
        "c1": config_system("c1"),
        "nnc": make_grid_system(17, 13, 9, active_frac=0.85, nnc_frac=0.03, seed=4, sigma=2.0),
        "thin": make_grid_system(1, 1, 200, seed=5),
        "ragged": make_grid_system(5, 17, 1, seed=6),     # 85 rows: one full tile + 1
        "one": make_grid_system(1, 1, 1, seed=7),
        # bipartite, in many components with single-row islands (the
        # analysis colours such patterns without its queue)
        "islands": make_grid_system(15, 11, 7, active_frac=0.45, seed=8),
    }
    return out


CASES = cases()


def oracle_factors(s, ordering, vals=None):
    vals = s.vals[0] if vals is None else vals
    perm = oracle.ordering_perm(s.rowptr, s.colidx, ordering)
    prow, pcol, pv = oracle.permute(s.rowptr, s.colidx, vals, perm)
    st, bad, lu, dinv = oracle.ilu0(prow, pcol, pv)
    return perm, prow, pcol, pv, st, bad, lu, dinv


def rel_block_err(a, b):
    """max over block rows of ||a - b||_inf, over max ||b||_inf."""
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture
def solver_of():
    made = []

    def make(s, ordering, precision=rs.PREC_FP64, vals=None):
        v = s.vals if vals is None else vals
        A = rs.bcsr_create(s.rowptr, s.colidx, v)
        M = rs.ilu0_analyse(A, ordering)
        made.append((A, M))
        st, bad = rs.ilu0_factor(M, A, precision)
        return A, M, st, bad

    yield make
    for A, M in made:
        rs.ilu0_destroy(M)
        rs.bcsr_destroy(A)


@pytest.mark.parametrize("name", list(CASES))
def test_spmv_parity(name):
    s = CASES[name]
    A = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
    try:
        x = np.random.default_rng(1).standard_normal((1, s.n, 3))
        y = rs.bcsr_spmv(A, x)
        yo = oracle.spmv(s.rowptr, s.colidx, s.vals[0], x[0])
        ax = oracle.spmv(s.rowptr, s.colidx, np.abs(s.vals[0]), np.abs(x[0]))
        assert np.all(np.abs(y[0] - yo) <= 1e-13 * ax + 1e-300)
    finally:
        rs.bcsr_destroy(A)


def test_spmv_batch_and_sizes():
    s = make_ensemble(9, 10, 3, seeds=[1, 2, 3])
    A = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
    try:
        x = np.random.default_rng(2).standard_normal((3, s.n, 3))
        y = rs.bcsr_spmv(A, x)
        for k in range(3):
            yo = oracle.spmv(s.rowptr, s.colidx, s.vals[k], x[k])
            assert np.abs(y[k] - yo).max() <= 1e-13 * np.abs(yo).max()
        y2 = rs.bcsr_spmv(A, x[1:2], first_sys=1, n_sys=1)
        assert np.array_equal(y2[0], y[1])
    finally:
        rs.bcsr_destroy(A)


@pytest.mark.parametrize("ordering", ORDERINGS)
@pytest.mark.parametrize("name", list(CASES))
def test_schedule_matches_oracle(solver_of, name, ordering):
    s = CASES[name]
    A, M, st, _ = solver_of(s, ordering)
    perm, ns, sp = rs.ilu0_get_schedule(M, s.n)
    assert np.array_equal(perm, oracle.ordering_perm(s.rowptr, s.colidx, ordering))


@pytest.mark.parametrize("ordering", ORDERINGS)
@pytest.mark.parametrize("name", list(CASES))
def test_factor_parity(solver_of, name, ordering):
    s = CASES[name]
    A, M, st, bad = solver_of(s, ordering)
    assert st == rs.OK and bad[0] == -1
    perm, prow, pcol, pv, ost, obad, lu, dinv = oracle_factors(s, ordering)
    assert ost == oracle.OK
    glu, gdinv = rs.ilu0_get_factors(M, 0, s.n, s.nnzb)
    offd = np.array([pcol[p] != i for i in range(s.n) for p in range(prow[i], prow[i + 1])], bool)
    if offd.any():
        assert rel_block_err(glu[offd], lu[offd]) <= 1e-12
    assert rel_block_err(gdinv, dinv) <= 1e-12


@pytest.mark.parametrize("n", [2, 6])
def test_factor_parity_dense_pattern(solver_of, n):
    rowptr, colidx = dense_pattern(n)
    vals = random_values(rowptr, colidx, seed=n)

    class S:
        pass
    s = S()
    s.rowptr, s.colidx, s.vals, s.n, s.nnzb = rowptr, colidx, vals[None], n, len(colidx)
    A, M, st, _ = solver_of(s, rs.ORDER_NATURAL)
    assert st == rs.OK
    _, _, lu, dinv = oracle.ilu0(rowptr, colidx, vals)
    glu, gdinv = rs.ilu0_get_factors(M, 0, n, len(colidx))
    offd = colidx != np.repeat(np.arange(n), n)
    assert rel_block_err(glu[offd], lu[offd]) <= 1e-12
    assert rel_block_err(gdinv, dinv) <= 1e-12


@pytest.mark.parametrize("ordering", ORDERINGS)
@pytest.mark.parametrize("name", ["c1", "nnc", "ragged", "islands"])
@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
def test_apply_parity(solver_of, name, ordering, precision):
    s = CASES[name]
    A, M, st, _ = solver_of(s, ordering, precision)
    v = np.random.default_rng(3).standard_normal((1, s.n, 3))
    z = rs.ilu0_apply(M, v)
    perm, prow, pcol, pv, _, _, lu, dinv = oracle_factors(s, ordering)
    if precision == rs.PREC_FP64:
        zp = oracle.apply(prow, pcol, lu, dinv, v[0][perm])
        zo = np.empty_like(zp)
        zo[perm] = zp
        assert np.linalg.norm(z[0] - zo) <= 1e-12 * np.linalg.norm(zo)
    else:
        # FP32 factors, input and arithmetic on both sides, in different
        # orders of rounding (the GPU fuses multiply-adds): element by
        # element within the first-order FP32 error bound of two such
        # evaluations of the same rounded data
        zp = oracle.apply_f32(prow, pcol, lu, dinv, v[0][perm])
        r32 = [a.astype(np.float32).astype(np.float64) for a in (lu, dinv, v[0][perm])]
        bound = fp32_apply_bound(prow, pcol, *r32)
        assert np.all(np.abs(z[0][perm] - zp) <= bound)


@pytest.mark.parametrize("case", ["nnc_level_sets", "grid_batch_colour"])
def test_fp32_factors_are_rounded_fp64_factors(solver_of, case):
    """FP32 factors within an ulp of the oracle's FP64 factors rounded to
    FP32: non-neighbour connections under level sets (levels whose rows
    keep their slices in 8 and in 6 registers), and a batch of two grid
    systems under colouring (the second colour's L blocks leave through the
    workgroup's LDS as one range, at a per-system offset)."""
    if case == "nnc_level_sets":
        s, ordering = CASES["nnc"], rs.ORDER_LEVEL_SET
    else:
        s, ordering = make_ensemble(17, 13, 7, seeds=[41, 42]), rs.ORDER_GRAPH_COLOUR
    A, M, st, _ = solver_of(s, ordering, rs.PREC_FP32_FACTORS)
    assert st == rs.OK
    for k in range(s.vals.shape[0]):
        _, prow, pcol, _, _, _, lu, dinv = oracle_factors(s, ordering, s.vals[k])
        glu, gdinv = rs.ilu0_get_factors(M, k, s.n, s.nnzb)
        offd = np.array([pcol[p] != i for i in range(s.n) for p in range(prow[i], prow[i + 1])], bool)
        for g, o in ((glu[offd], lu[offd]), (gdinv, dinv)):
            o32 = o.astype(np.float32)
            ulp = np.spacing(np.abs(o32)).astype(np.float64)
            assert np.all(np.abs(g - o32.astype(np.float64)) <= ulp)


@pytest.mark.parametrize("ordering", ORDERINGS)
@pytest.mark.parametrize("name", ["c1", "nnc", "thin", "ragged", "one", "islands"])
def test_solve_parity_tight(solver_of, name, ordering):
    s = CASES[name]
    A, M, st, _ = solver_of(s, ordering)
    b = s.b[0, 0]
    x, st, info = rs.bicgstab_solve(M, A, b[None], reduction=1e-10)
    xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[0], b, ordering=ordering, reduction=1e-10)
    assert st == rs.OK and info[0]["status"] == rs.OK
    assert np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)
    hs, ohs = info[0]["half_steps"], oinfo["half_steps"]
    near = abs(oinfo["final_norm"] - 1e-10 * oinfo["r0_norm"]) <= 1e-3 * 1e-10 * oinfo["r0_norm"]
    assert hs == ohs or (abs(hs - ohs) == 1 and near)
    assert info[0]["true_rel_residual"] <= 1e-9
    assert abs(info[0]["r0_norm"] - oinfo["r0_norm"]) <= 1e-13 * oinfo["r0_norm"]


@pytest.mark.parametrize("tiles", [0, 1])
@pytest.mark.parametrize("ordering", ORDERINGS)
@pytest.mark.parametrize("name", ["c1", "nnc"])
def test_sweep_modes_agree(solver_of, name, ordering, tiles):
    """One launch per level and single-launch tiled sweeps give the same bits
    (same arithmetic per row, only the launch structure differs).  The
    upper launch fused with the SpMV runs with per-level sweeps only, so it
    is off here (its own tests compare it with the unfused solve)."""
    s = CASES[name]
    A, M, _, _ = solver_of(s, ordering)
    rs.ilu0_set_option(M, rs.OPT_FUSE_SPMV, 0)
    rs.ilu0_set_option(M, rs.OPT_SWEEP_TILES, tiles)
    assert rs.ilu0_get_option(M, rs.OPT_SWEEP_TILES) == tiles
    v = np.random.default_rng(9).standard_normal((1, s.n, 3))
    z = rs.ilu0_apply(M, v)
    x, st, info = rs.bicgstab_solve(M, A, s.b[0], reduction=1e-8)
    rs.ilu0_set_option(M, rs.OPT_SWEEP_TILES, 1 - tiles)
    z2 = rs.ilu0_apply(M, v)
    x2, st2, info2 = rs.bicgstab_solve(M, A, s.b[0], reduction=1e-8)
    assert np.array_equal(z, z2) and np.array_equal(x, x2) and outcome(info) == outcome(info2)


@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
@pytest.mark.parametrize("ordering", [rs.ORDER_LEVEL_SET, rs.ORDER_GRAPH_COLOUR])
def test_graph_replays_equal_eager(solver_of, ordering, precision):
    """An iteration replayed from a captured graph gives the eager result,
    replay after replay, with eager work and synchronisations in between.
    The fused upper launch is off: it follows the sweep mode, which the
    test switches before a recapture."""
    s = make_ensemble(11, 9, 7, seeds=[3, 4])
    A, M, _, _ = solver_of(s, ordering, precision)
    rs.ilu0_set_option(M, rs.OPT_FUSE_SPMV, 0)
    rs.ilu0_set_option(M, rs.OPT_USE_GRAPH, 0)
    ref = [rs.bicgstab_solve(M, A, s.b[:, 0] * (k + 1), reduction=1e-9) for k in range(3)]
    rs.ilu0_set_option(M, rs.OPT_USE_GRAPH, 1)
    for rep in range(2):
        for k in range(3):
            x, st, info = rs.bicgstab_solve(M, A, s.b[:, 0] * (k + 1), reduction=1e-9)
            rs.ilu0_apply(M, s.b[0, 0][None])           # eager work between replays
            assert np.array_equal(x, ref[k][0]) and outcome(info) == outcome(ref[k][2])
    rs.ilu0_set_option(M, rs.OPT_SWEEP_TILES, 1 - rs.ilu0_get_option(M, rs.OPT_SWEEP_TILES))
    x, st, info = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-9)   # recaptured
    assert np.array_equal(x, ref[0][0])
    # timing v = A phat: two graph segments with a direct launch between them
    rs.rsolve_profile_enable(1 << rs.PROF_SPMV_V)
    try:
        for k in range(3):
            x, st, info = rs.bicgstab_solve(M, A, s.b[:, 0] * (k + 1), reduction=1e-9)
            assert np.array_equal(x, ref[k][0]) and outcome(info) == outcome(ref[k][2])
        ms, units, byts = rs.rsolve_profile_get(rs.PROF_SPMV_V)
        assert units > 0 and ms > 0 and byts > 0
    finally:
        rs.rsolve_profile_enable(0)


@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
def test_row_variants(solver_of, precision):
    """Every launch shape (waves per workgroup; LDS staging, direct loads, or
    LDS staging with non-temporal loads) of the SpMV and of the per-level
    sweeps does the same arithmetic: plain SpMV and sweeps are bit-identical
    across shapes, with FP64 and with FP32 factors.  The SpMV shape also
    sets the number of partial sums of the fused dot products, so solves
    under different SpMV shapes agree to rounding (each one deterministic)."""
    s = CASES["nnc"]
    A, M, _, _ = solver_of(s, rs.ORDER_GRAPH_COLOUR, precision)
    x = np.random.default_rng(4).standard_normal((1, s.n, 3))
    ref_y = None
    for v in range(rs.N_ROW_VARIANTS):
        rs.bcsr_set_option(A, rs.OPT_SPMV_VARIANT, v)
        y = rs.bcsr_spmv(A, x)
        ref_y = y if ref_y is None else ref_y
        assert np.array_equal(y, ref_y), v
    ref = None
    for v in range(rs.N_ROW_VARIANTS):
        rs.ilu0_set_option(M, rs.OPT_SWEEP_VARIANT, v)
        z = rs.ilu0_apply(M, x)
        xs, st, info = rs.bicgstab_solve(M, A, s.b[0], reduction=1e-9)
        ref = (z, xs, info) if ref is None else ref
        assert np.array_equal(z, ref[0]) and np.array_equal(xs, ref[1]) and outcome(info) == outcome(ref[2]), v
    for v in range(rs.N_ROW_VARIANTS):
        rs.ilu0_set_option(M, rs.OPT_SPMV_VARIANT, v)
        xs, st, info = rs.bicgstab_solve(M, A, s.b[0], reduction=1e-9)
        xs2, _, info2 = rs.bicgstab_solve(M, A, s.b[0], reduction=1e-9)
        assert np.array_equal(xs, xs2) and outcome(info) == outcome(info2), v
        # FP32 sweeps round the rounding differences of alpha and omega once more
        tol = 1e-10 if precision == rs.PREC_FP64 else 1e-7
        assert np.linalg.norm(xs - ref[1]) <= tol * np.linalg.norm(ref[1]), v
        assert abs(info[0]["half_steps"] - ref[2][0]["half_steps"]) <= 1, v
    with pytest.raises(rs.RsolveError):
        rs.ilu0_set_option(M, rs.OPT_SPMV_VARIANT, rs.N_ROW_VARIANTS)


def test_autotune_picks_valid_config_and_caches(solver_of, tmp_path, monkeypatch):
    s = make_ensemble(13, 11, 9, seeds=[5, 6, 7])
    A, M, _, _ = solver_of(s, rs.ORDER_GRAPH_COLOUR, rs.PREC_FP32_FACTORS)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("RSOLVE_TUNE_CACHE", str(cache))
    r = rs.ilu0_autotune(M, A, s.b[:, 0], reduction=1e-2, reps=1)
    assert r["from_cache"] == 0 and r["candidates"] >= 10 and r["us_per_solve"] > 0
    assert rs.ilu0_get_option(M, rs.OPT_SPMV_VARIANT) == r["spmv_variant"]
    assert rs.ilu0_get_option(M, rs.OPT_SWEEP_TILES) == r["sweep_tiles"]
    assert rs.ilu0_get_option(M, rs.OPT_REDUCE_SPLIT) == r["reduce_split"]
    x, st, info = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-8)
    for k in range(3):
        xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[k], s.b[k, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                             precond=oracle.PREC_ILU_F32, reduction=1e-8)
        assert np.linalg.norm(x[k] - xo) <= 1e-6 * np.linalg.norm(xo)
    assert cache.exists() and cache.read_text().count("\n") == 1
    rs.ilu0_set_option(M, rs.OPT_SPMV_VARIANT, (r["spmv_variant"] + 1) % rs.N_ROW_VARIANTS)
    r2 = rs.ilu0_autotune(M, A, s.b[:, 0], reduction=1e-2, reps=1)
    assert r2["from_cache"] == 1 and r2["spmv_variant"] == r["spmv_variant"]
    assert r2["reduce_split"] == r["reduce_split"]
    assert rs.ilu0_get_option(M, rs.OPT_SPMV_VARIANT) == r["spmv_variant"]


@pytest.mark.parametrize("grid", [1, 3, 64])
def test_tiled_sweep_small_grids(solver_of, grid):
    """Fewer workgroups than tiles: each workgroup walks many tiles in ticket order."""
    s = CASES["nnc"]
    A, M, _, _ = solver_of(s, rs.ORDER_LEVEL_SET)
    rs.ilu0_set_option(M, rs.OPT_SWEEP_GRID, grid)
    x, st, info = rs.bicgstab_solve(M, A, s.b[0], reduction=1e-10)
    xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_LEVEL_SET, reduction=1e-10)
    assert st == rs.OK and np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)


@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
@pytest.mark.parametrize("red", [1e-2, 1e-6])
def test_solve_reduction_and_true_residual(solver_of, precision, red):
    s = CASES["nnc"]
    A, M, st, _ = solver_of(s, rs.ORDER_LEVEL_SET, precision)
    x, st, info = rs.bicgstab_solve(M, A, s.b[0], reduction=red)
    oprec = oracle.PREC_ILU_F64 if precision == rs.PREC_FP64 else oracle.PREC_ILU_F32
    xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_LEVEL_SET,
                             precond=oprec, reduction=red)
    assert st == rs.OK
    assert info[0]["final_norm"] <= red * info[0]["r0_norm"]
    assert info[0]["true_rel_residual"] <= red * (1 + 1e-6)
    assert abs(info[0]["half_steps"] - oinfo["half_steps"]) <= 1
    xt = oracle.spmv(s.rowptr, s.colidx, s.vals[0], x[0])
    assert np.linalg.norm(s.b[0, 0] - xt) / np.linalg.norm(s.b[0, 0]) <= red * (1 + 1e-6)


def test_batch_members_equal_alone(solver_of):
    s = make_ensemble(12, 10, 6, seeds=[11, 12, 13, 14])
    A, M, st, _ = solver_of(s, rs.ORDER_LEVEL_SET, rs.PREC_FP32_FACTORS)
    assert st == rs.OK
    xb, stb, infob = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-6)
    for k in range(4):
        class S1:
            pass
        one = S1()
        one.rowptr, one.colidx, one.vals, one.n, one.nnzb = s.rowptr, s.colidx, s.vals[k:k + 1], s.n, s.nnzb
        A1, M1, _, _ = solver_of(one, rs.ORDER_LEVEL_SET, rs.PREC_FP32_FACTORS)
        x1, st1, info1 = rs.bicgstab_solve(M1, A1, s.b[k:k + 1, 0], reduction=1e-6)
        assert np.array_equal(x1[0], xb[k])
        assert info1[0]["half_steps"] == infob[k]["half_steps"]


def test_repeat_solve_bitwise(solver_of):
    s = CASES["nnc"]
    A, M, _, _ = solver_of(s, rs.ORDER_GRAPH_COLOUR)
    x1, _, i1 = rs.bicgstab_solve(M, A, s.b[0], reduction=1e-8)
    x2, _, i2 = rs.bicgstab_solve(M, A, s.b[0], reduction=1e-8)
    assert np.array_equal(x1, x2) and outcome(i1) == outcome(i2)


def test_status_paths(solver_of):
    s = CASES["c1"]
    A, M, st, _ = solver_of(s, rs.ORDER_LEVEL_SET)
    b = s.b[0]
    x, st, info = rs.bicgstab_solve(M, A, np.zeros_like(b))
    assert st == rs.OK and info[0]["half_steps"] == 0 and not x.any()
    bn = b.copy()
    bn[0, 7, 2] = np.nan
    x, st, info = rs.bicgstab_solve(M, A, bn)
    assert st == rs.NON_FINITE
    x, st, info = rs.bicgstab_solve(M, A, b, reduction=1e-12, max_iter=1)
    assert st == rs.NOT_CONVERGED and info[0]["half_steps"] == 2
    xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[0], b[0], ordering=rs.ORDER_LEVEL_SET, reduction=1e-12,
                             max_iter=1)
    assert np.linalg.norm(x[0] - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("row", [1234, 1235])
def test_zero_pivot_reports_oracle_row(solver_of, row):
    """A zero block row (L_ik = 0 and U_ii = 0 whatever the ordering); two
    neighbouring rows, so that under graph colouring one of them is in the
    first colour (the factorisation's first level, rows without lower
    blocks) and the other in the second."""
    s = CASES["c1"]
    vz = s.vals.copy()
    vz[0, s.rowptr[row]:s.rowptr[row + 1]] = 0.0
    for ordering in ORDERINGS:
        A, M, st, bad = solver_of(s, ordering, vals=vz)
        _, oinfo = oracle.solve(s.rowptr, s.colidx, vz[0], s.b[0, 0], ordering=ordering)
        assert st == rs.ZERO_PIVOT and oinfo["status"] == oracle.ZERO_PIVOT
        assert bad[0] == oinfo["bad_row"]
        x, sst, info = rs.bicgstab_solve(M, A, s.b[0])
        assert sst == rs.ZERO_PIVOT


def test_handle_errors(solver_of):
    s = CASES["c1"]
    A = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
    M = rs.ilu0_analyse(A, rs.ORDER_LEVEL_SET)
    try:
        with pytest.raises(rs.RsolveError) as e:
            rs.bicgstab_solve(M, A, s.b[0])
        assert e.value.status == rs.NOT_FACTORED
        other = CASES["nnc"]
        B = rs.bcsr_create(other.rowptr, other.colidx, other.vals)
        with pytest.raises(rs.RsolveError) as e:
            rs.ilu0_factor(M, B)
        assert e.value.status == rs.PATTERN_MISMATCH
        rs.bcsr_destroy(B)
        bad_cols = s.colidx.copy()
        bad_cols[[0, 1]] = bad_cols[[1, 0]]
        with pytest.raises(rs.RsolveError) as e:
            rs.bcsr_create(s.rowptr, bad_cols, s.vals)
        assert e.value.status == rs.BAD_PATTERN and e.value.bad_row == 0
    finally:
        rs.ilu0_destroy(M)
        rs.bcsr_destroy(A)


def test_shared_analysis_gives_identical_factors_and_solutions():
    s = CASES["nnc"]
    for ordering in ORDERINGS:
        A = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
        M = rs.ilu0_analyse(A, ordering)
        A2 = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
        M2 = rs.ilu0_analyse_shared(A2, M)
        try:
            rs.ilu0_factor(M, A)
            x1, st1, i1 = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-10)
            lu1, d1 = rs.ilu0_get_factors(M, 0, s.n, s.nnzb)
            rs.ilu0_destroy(M)                    # the shared analysis outlives the handle it came from
            M = None
            rs.ilu0_factor(M2, A2)
            x2, st2, i2 = rs.bicgstab_solve(M2, A2, s.b[:, 0], reduction=1e-10)
            lu2, d2 = rs.ilu0_get_factors(M2, 0, s.n, s.nnzb)
            assert st1 == st2 == rs.OK and i1[0]["half_steps"] == i2[0]["half_steps"]
            assert np.array_equal(lu1, lu2) and np.array_equal(d1, d2) and np.array_equal(x1, x2)
            assert rs.ilu0_get_schedule(M2, s.n)[0].tolist() == oracle.ordering_perm(
                s.rowptr, s.colidx, ordering).tolist()
            other = CASES["c1"]
            B = rs.bcsr_create(other.rowptr, other.colidx, other.vals)
            with pytest.raises(rs.RsolveError) as e:
                rs.ilu0_analyse_shared(B, M2)
            assert e.value.status == rs.PATTERN_MISMATCH
            rs.bcsr_destroy(B)
        finally:
            rs.ilu0_destroy(M)
            rs.ilu0_destroy(M2)
            rs.bcsr_destroy(A)
            rs.bcsr_destroy(A2)


def test_fresh_handles_on_a_non_blocking_stream():
    """Every device initialisation (pattern and schedule uploads, workspace
    clearing) must be ordered before work that the caller queues on its own
    stream, which need not synchronise with the null stream."""
    torch = pytest.importorskip("torch")
    s = CASES["nnc"]
    ref = {}
    for ordering in ORDERINGS:
        with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=ordering) as sol:
            sol.factor()
            ref[ordering] = sol.solve(s.b[:, 0], reduction=1e-10)
    side = torch.cuda.Stream()
    dev = torch.device("cuda:0")
    vals = torch.from_numpy(s.vals).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(s.b[:, 0])).to(dev)
    torch.cuda.synchronize()
    for rep in range(3):
        for ordering in ORDERINGS:
            x = torch.empty_like(b)
            A = rs.bcsr_create(s.rowptr, s.colidx, stream=side.cuda_stream)
            M = rs.ilu0_analyse(A, ordering)
            try:
                rs.bcsr_set_values(A, vals, stream=side.cuda_stream)
                rs.ilu0_factor(M, A, stream=side.cuda_stream)
                _, st, info = rs.bicgstab_solve(M, A, b, x, reduction=1e-10, stream=side.cuda_stream)
                side.synchronize()
                xr, str_, ir = ref[ordering]
                assert st == str_ == rs.OK and info[0]["half_steps"] == ir[0]["half_steps"]
                assert np.array_equal(x.cpu().numpy(), xr)
            finally:
                rs.ilu0_destroy(M)
                rs.bcsr_destroy(A)


def jacobi_case(parts):
    s = CASES["nnc"]
    return s, rs.bcsr_partition(s.rowptr, s.colidx, parts, weights=s.trans)


def jacobi_handles(s, ordering, part, precision=rs.PREC_FP64):
    A = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
    M = rs.ilu0_analyse_jacobi(A, ordering, part)
    st, bad = rs.ilu0_factor(M, A, precision)
    return A, M, st


@pytest.mark.parametrize("ordering", ORDERINGS)
@pytest.mark.parametrize("parts", [3, 40])
def test_jacobi_factor_and_solve_parity(ordering, parts):
    s, part = jacobi_case(parts)
    A, M, st = jacobi_handles(s, ordering, part)
    try:
        assert st == rs.OK
        # oracle: ILU0 of the Jacobi matrix in its own ordering
        rrow, rcol, rv = oracle.jacobi_matrix(s.rowptr, s.colidx, s.vals[0], part)
        perm = oracle.ordering_perm(rrow, rcol, ordering)
        gperm, nsets, _ = rs.ilu0_get_schedule(M, s.n)
        assert np.array_equal(gperm, perm)
        mrow, mcol, mv = oracle.permute(rrow, rcol, rv, perm)
        ost, _, lu, dinv = oracle.ilu0(mrow, mcol, mv)
        assert ost == oracle.OK
        prow, pcol, _ = oracle.permute(s.rowptr, s.colidx, s.vals[0], perm)
        glu, gdinv = rs.ilu0_get_factors(M, 0, s.n, s.nnzb)
        keep = np.array([part[perm[i]] == part[perm[pcol[p]]] for i in range(s.n)
                         for p in range(prow[i], prow[i + 1])], bool)
        offd = np.array([mcol[p] != i for i in range(s.n) for p in range(mrow[i], mrow[i + 1])], bool)
        assert not glu[~keep].any()                               # dropped blocks stay empty
        assert rel_block_err(glu[keep][offd], lu[offd]) <= 1e-12
        assert rel_block_err(gdinv, dinv) <= 1e-12
        x, sst, info = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-10)
        xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering, reduction=1e-10,
                                 part=part)
        assert sst == oinfo["status"] == rs.OK
        assert np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)
        assert info[0]["half_steps"] == oinfo["half_steps"]
        assert info[0]["true_rel_residual"] <= 1e-9
    finally:
        rs.ilu0_destroy(M)
        rs.bcsr_destroy(A)


def test_jacobi_single_partition_is_plain_ilu0(solver_of):
    s = CASES["nnc"]
    for ordering in ORDERINGS:
        A, M, st = jacobi_handles(s, ordering, np.zeros(s.n, np.int32))
        try:
            A2, M2, st2, _ = solver_of(s, ordering)
            x1, st1, i1 = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-10)
            x2, st2, i2 = rs.bicgstab_solve(M2, A2, s.b[:, 0], reduction=1e-10)
            assert np.array_equal(x1, x2) and i1[0]["half_steps"] == i2[0]["half_steps"]
        finally:
            rs.ilu0_destroy(M)
            rs.bcsr_destroy(A)


def test_jacobi_mixed_precision_and_fewer_levels():
    s = make_grid_system(20, 18, 24, seed=9)
    part = (np.arange(s.n) // (20 * 18 * 6)).astype(np.int32)          # 4 z-slabs of 6 layers
    A, M, st = jacobi_handles(s, rs.ORDER_LEVEL_SET, part, rs.PREC_FP32_FACTORS)
    try:
        assert st == rs.OK
        assert rs.ilu0_get_sweep_levels(M) == (20 + 18 + 6 - 2, 20 + 18 + 6 - 2)
        x, sst, info = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-6)
        xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_LEVEL_SET,
                                 precond=oracle.PREC_ILU_F32, reduction=1e-6, part=part)
        assert sst == rs.OK and info[0]["true_rel_residual"] <= 1e-6 * (1 + 1e-6)
        assert abs(info[0]["half_steps"] - oinfo["half_steps"]) <= 2
    finally:
        rs.ilu0_destroy(M)
        rs.bcsr_destroy(A)


@pytest.mark.parametrize("variant", [0, 2, 5])
def test_reduce_split_modes_match_the_oracle(solver_of, variant):
    """Both ways of adding the SpMVs' dot products give oracle-matching,
    reproducible solutions."""
    s = CASES["nnc"]
    A, M, st, _ = solver_of(s, rs.ORDER_GRAPH_COLOUR)
    xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                             reduction=1e-10)
    rs.ilu0_set_option(M, rs.OPT_SPMV_VARIANT, variant)
    for split in (0, 1, 2):
        rs.ilu0_set_option(M, rs.OPT_REDUCE_SPLIT, split)
        assert rs.ilu0_get_option(M, rs.OPT_REDUCE_SPLIT) == split
        x1, st1, i1 = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-10)
        x2, st2, i2 = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-10)
        assert st1 == st2 == rs.OK and np.array_equal(x1, x2)
        assert np.linalg.norm(x1[0] - xo) <= 1e-8 * np.linalg.norm(xo)
        assert i1[0]["half_steps"] == oinfo["half_steps"]
        assert abs(i1[0]["true_rel_residual"] - oinfo["true_rel_residual"]) <= 1e-12 + 1e-3 * oinfo["true_rel_residual"]


def test_graph_recaptured_for_every_setting(solver_of):
    """A captured iteration is replayed only under the settings it was
    captured with: after each change of sweep shape and dot-product split
    (pairs whose settings once shared a cache key among them) the replayed
    solve equals the eager solve under the same settings."""
    s = CASES["nnc"]
    A, M, _, _ = solver_of(s, rs.ORDER_GRAPH_COLOUR)
    rs.ilu0_set_option(M, rs.OPT_SPMV_VARIANT, 0)
    for sweep, split in ((4, 0), (0, 1), (4, 0), (2, 2), (0, 0)):
        rs.ilu0_set_option(M, rs.OPT_SWEEP_VARIANT, sweep)
        rs.ilu0_set_option(M, rs.OPT_REDUCE_SPLIT, split)
        rs.ilu0_set_option(M, rs.OPT_USE_GRAPH, 0)
        xe, ste, ie = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-10)
        rs.ilu0_set_option(M, rs.OPT_USE_GRAPH, 1)
        xg, stg, ig = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-10)
        assert ste == stg == rs.OK and np.array_equal(xe, xg) and outcome(ie) == outcome(ig), (sweep, split)


def test_device_memory_path():
    torch = pytest.importorskip("torch")
    s = CASES["nnc"]
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(s.rowptr).to(dev)
    ci = torch.from_numpy(s.colidx).to(dev)
    vals = torch.from_numpy(s.vals).to(dev)
    b = torch.from_numpy(s.b[:, 0].copy()).to(dev)
    x = torch.zeros_like(b)
    A = rs.bcsr_create(rp, ci, vals)
    M = rs.ilu0_analyse(A, rs.ORDER_GRAPH_COLOUR)
    try:
        rs.ilu0_factor(M, A)
        rs.bicgstab_solve(M, A, b, x, reduction=1e-10)
        torch.cuda.synchronize()
        xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                             reduction=1e-10)
        xg = x.cpu().numpy()[0]
        assert np.linalg.norm(xg - xo) <= 1e-8 * np.linalg.norm(xo)
    finally:
        rs.ilu0_destroy(M)
        rs.bcsr_destroy(A)


@pytest.mark.parametrize("ordering", [rs.ORDER_GRAPH_COLOUR, rs.ORDER_LEVEL_SET, rs.ORDER_RCM_LEVEL_SET])
def test_c2_full_size_parity(solver_of, ordering):
    """The 46x112x22 masked grid with 2% NNCs at full size: factors on sampled
    rows, and the solution at 1e-10 for the first right-hand side."""
    s = config_system("c2", n_rhs=2)
    A, M, st, _ = solver_of(s, ordering)
    assert st == rs.OK
    perm, prow, pcol, pv, ost, _, lu, dinv = oracle_factors(s, ordering)
    glu, gdinv = rs.ilu0_get_factors(M, 0, s.n, s.nnzb)
    assert rel_block_err(gdinv, dinv) <= 1e-12
    offd = np.repeat(np.arange(s.n), np.diff(prow)) != pcol
    assert rel_block_err(glu[offd], lu[offd]) <= 1e-12
    x, st, info = rs.bicgstab_solve(M, A, s.b[0, :1], reduction=1e-10)
    xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering, reduction=1e-10)
    assert st == rs.OK
    assert np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)
    assert abs(info[0]["half_steps"] - oinfo["half_steps"]) <= 1
    x, st, info = rs.bicgstab_solve(M, A, s.b[0, 1:2], reduction=1e-2)
    assert st == rs.OK and info[0]["true_rel_residual"] <= 1e-2


def test_c3_full_size_parity():
    """The 100^3 grid (1M cells, sigma 2) at full size in the configuration the
    benchmark times (graph colouring, autotuned launch shapes): FP64 factors
    against the oracle's, the FP64 solution at 1e-10, FP32 factors as
    roundings of the oracle's, and the mixed solve at 1e-2."""
    s = config_system("c3")
    A = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
    M = rs.ilu0_analyse(A, rs.ORDER_GRAPH_COLOUR)
    try:
        st, _ = rs.ilu0_factor(M, A, rs.PREC_FP64)
        assert st == rs.OK
        perm, prow, pcol, pv, ost, _, lu, dinv = oracle_factors(s, rs.ORDER_GRAPH_COLOUR)
        assert ost == oracle.OK
        glu, gdinv = rs.ilu0_get_factors(M, 0, s.n, s.nnzb)
        assert rel_block_err(gdinv, dinv) <= 1e-12
        offd = np.repeat(np.arange(s.n), np.diff(prow)) != pcol
        assert rel_block_err(glu[offd], lu[offd]) <= 1e-12
        del glu
        rs.ilu0_autotune(M, A, s.b[:, 0], reduction=1e-2, reps=1)
        x, st, info = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-10)
        xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                                 reduction=1e-10)
        assert st == oinfo["status"] == rs.OK
        assert np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)
        # 1M rows summed in different orders: at 1e-10 the erratic BiCGStab
        # residual of this sigma = 2 system crosses the threshold a few half
        # steps apart on the two sides (x agrees to 1e-8 all the same)
        assert abs(info[0]["half_steps"] - oinfo["half_steps"]) <= max(1, oinfo["half_steps"] // 5)
        st, _ = rs.ilu0_factor(M, A, rs.PREC_FP32_FACTORS)
        glu, gdinv = rs.ilu0_get_factors(M, 0, s.n, s.nnzb)
        for g, o in ((glu[offd], lu[offd]), (gdinv, dinv)):
            o32 = o.astype(np.float32)
            assert np.all(np.abs(g - o32.astype(np.float64)) <= np.spacing(np.abs(o32)).astype(np.float64))
        del glu
        x, st, info = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-2)
        _, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                                precond=oracle.PREC_ILU_F32, reduction=1e-2)
        assert st == rs.OK and info[0]["true_rel_residual"] <= 1e-2
        assert abs(info[0]["half_steps"] - oinfo["half_steps"]) <= 1
    finally:
        rs.ilu0_destroy(M)
        rs.bcsr_destroy(A)


def test_c4_full_size_batch_parity():
    """The 64-member 40x40x30 ensemble at full size, FP32 factors, one batched
    factorisation and solve in the autotuned configuration; every eighth
    member checked against the oracle at 1e-8."""
    s = config_system("c4")
    A = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
    M = rs.ilu0_analyse(A, rs.ORDER_GRAPH_COLOUR)
    try:
        st, bad = rs.ilu0_factor(M, A, rs.PREC_FP32_FACTORS)
        assert st == rs.OK and (bad == -1).all()
        rs.ilu0_autotune(M, A, s.b[:, 0], reduction=1e-2, reps=1)
        x, st, info = rs.bicgstab_solve(M, A, s.b[:, 0], reduction=1e-8)
        assert st == rs.OK and all(i["status"] == rs.OK for i in info)
        for k in range(0, 64, 8):
            xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[k], s.b[k, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                                     precond=oracle.PREC_ILU_F32, reduction=1e-8)
            assert np.linalg.norm(x[k] - xo) <= 1e-6 * np.linalg.norm(xo)
            assert info[k]["true_rel_residual"] <= 1e-8 * (1 + 1e-6)
    finally:
        rs.ilu0_destroy(M)
        rs.bcsr_destroy(A)
