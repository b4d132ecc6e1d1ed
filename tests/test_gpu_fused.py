"""GPU checks of the upper launch fused with the SpMV rows it can form
(RS_OPT_FUSE_SPMV): where the rows without lower blocks lead the analysed
order and share one upper level, BiCGStab forms their rows of v = A phat and
t = A shat inside the upper sweep.  z keeps its bits; v and t of those rows
add the same terms in another order, and the dot products' summation order
changes, so solves with and without the fusion agree to rounding, and the
fused solve meets the oracle's parity bar (x within 1e-8 at a reduction of
1e-10, equal half steps where decisive)."""

import numpy as np
import pytest

import oracle
import paper_2309_11488_amd as rs
from synth import config_system, make_ensemble, make_grid_system
from tests.helpers import outcome, trajectory_check

pytestmark = pytest.mark.gpu


def _solve(A, M, b, fuse, red, max_iter=200):
    rs.ilu0_set_option(M, rs.OPT_FUSE_SPMV, fuse)
    return rs.bicgstab_solve(M, A, b, reduction=red, max_iter=max_iter)


@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
@pytest.mark.parametrize("grid", [(20, 20, 10), (7, 5, 3), (9, 1, 1), (33, 17, 5)])
def test_fused_equals_unfused_to_rounding(grid, precision):
    """Bipartite grids under graph colouring (the first colour holds every
    row without lower blocks): the fusion engages; fused and unfused solves
    agree to rounding and take the same number of half steps; each is
    deterministic."""
    s = make_grid_system(*grid, sigma=2.0, seed=sum(grid))
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR, precision=precision) as sol:
        assert sol.factor()[0] == rs.OK
        n0 = rs.ilu0_get_option(sol.M, rs.OPT_FUSED_ROWS)
        assert n0 in (s.n // 2, (s.n + 1) // 2)       # one colour of the checkerboard
        b = s.b[:, 0]
        xu, stu, iu = _solve(sol.A, sol.M, b, 0, 1e-10)
        xf, stf, inf = _solve(sol.A, sol.M, b, 1, 1e-10)
        xf2, _, inf2 = _solve(sol.A, sol.M, b, 1, 1e-10)
    assert stu == stf == rs.OK
    assert np.array_equal(xf, xf2) and outcome(inf) == outcome(inf2)
    tol = 1e-10 if precision == rs.PREC_FP64 else 1e-7
    assert np.linalg.norm(xf - xu) <= tol * np.linalg.norm(xu)
    assert abs(inf[0]["half_steps"] - iu[0]["half_steps"]) <= 1
    assert inf[0]["true_rel_residual"] <= 1e-9


def test_fused_solve_matches_oracle_on_its_trajectory():
    """The 40x40x30 grid (the ensemble's member size), FP64 factors, fusion
    on: the fixed-iteration comparison with the oracle, then the solve at
    1e-10."""
    s = make_grid_system(40, 40, 30, seed=11)
    b = s.b[0, 0]
    perm = oracle.ordering_perm(s.rowptr, s.colidx, rs.ORDER_GRAPH_COLOUR)
    prow, pcol, pv = oracle.permute(s.rowptr, s.colidx, s.vals[0], perm)
    st, _, lu, dinv = oracle.ilu0(prow, pcol, pv)
    assert st == oracle.OK
    bp = np.ascontiguousarray(b.reshape(-1, 3)[perm])

    def run(reduction, max_iter):
        xp, info, tr = oracle.bicgstab(prow, pcol, pv, lu, dinv, bp, precond=oracle.PREC_ILU_F64,
                                       reduction=reduction, max_iter=max_iter, trace=True)
        x = np.empty_like(xp)
        x[perm] = xp
        return x, info, tr

    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR) as sol:
        sol.factor()
        assert rs.ilu0_get_option(sol.M, rs.OPT_FUSED_ROWS) in (s.n // 2, (s.n + 1) // 2)

        def gpu(red, max_iter):
            x, st, info = _solve(sol.A, sol.M, b[None], 1, red, max_iter)
            return x[0], st, info[0]
        trajectory_check(gpu, run, 1e-10, 1e-8, rs.NOT_CONVERGED)


def test_fused_batch_members_equal_alone_and_graphs_equal_eager():
    """A same-pattern batch: each member's fused solve equals its solve
    alone bit for bit, and graph replays equal eager launches."""
    s = make_ensemble(14, 12, 10, seeds=[21, 22, 23, 24])
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR,
                   precision=rs.PREC_FP32_FACTORS) as sol:
        sol.factor()
        assert rs.ilu0_get_option(sol.M, rs.OPT_FUSED_ROWS) > 0
        rs.ilu0_set_option(sol.M, rs.OPT_USE_GRAPH, 0)
        xe, ste, ie = sol.solve(s.b[:, 0], reduction=1e-8)
        rs.ilu0_set_option(sol.M, rs.OPT_USE_GRAPH, 1)
        xg, stg, ig = sol.solve(s.b[:, 0], reduction=1e-8)
        assert ste == stg == rs.OK and np.array_equal(xe, xg) and outcome(ie) == outcome(ig)
    for k in range(s.batch):
        with rs.Solver(s.rowptr, s.colidx, s.vals[k:k + 1], ordering=rs.ORDER_GRAPH_COLOUR,
                       precision=rs.PREC_FP32_FACTORS) as one:
            one.factor()
            x1, _, i1 = one.solve(s.b[k:k + 1, 0], reduction=1e-8)
        assert np.array_equal(x1[0], xg[k]) and outcome(i1) == outcome([ig[k]])


def test_fusion_stays_off_where_the_pattern_does_not_allow_it():
    """Level sets on a full grid (a single row without lower blocks), a
    masked grid with single-row islands, and Block-Jacobi partitions: no
    fusion, and every solve matches the oracle."""
    grid = make_grid_system(12, 9, 7, seed=3)
    islands = make_grid_system(15, 11, 7, active_frac=0.45, seed=8)
    for s, ordering in ((grid, rs.ORDER_LEVEL_SET), (islands, rs.ORDER_GRAPH_COLOUR)):
        with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=ordering) as sol:
            sol.factor()
            # level sets: one row without lower blocks; islands: isolated rows hold no upper block
            assert rs.ilu0_get_option(sol.M, rs.OPT_FUSED_ROWS) == 0
            x, st, info = sol.solve(s.b[:, 0], reduction=1e-10)
        xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering, reduction=1e-10)
        assert st == rs.OK and np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)
    part = rs.bcsr_partition(grid.rowptr, grid.colidx, 4, weights=grid.trans)
    with rs.Solver(grid.rowptr, grid.colidx, grid.vals, ordering=rs.ORDER_GRAPH_COLOUR, part=part) as sol:
        assert rs.ilu0_get_option(sol.M, rs.OPT_FUSED_ROWS) == 0
    with pytest.raises(rs.RsolveError):
        with rs.Solver(grid.rowptr, grid.colidx, grid.vals) as sol:
            rs.ilu0_set_option(sol.M, rs.OPT_FUSED_ROWS, 1)


def test_c3_fused_and_unfused_at_full_size():
    """The 100^3 grid (sigma 2) in FP64: the fused solve (the benchmark's
    configuration) and the unfused one agree to rounding at 1e-10 (x within
    1e-10; about 95 half steps on a sigma-2 field, over which the last bits
    of the two recurrences drift apart: the counts agree within 5 %), and
    the fused x matches the oracle within 1e-8 (the same-trajectory
    comparison at this size is in the contract tests)."""
    s = config_system("c3")
    b = s.b[0, 0]
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR) as sol:
        sol.factor()
        assert rs.ilu0_get_option(sol.M, rs.OPT_FUSED_ROWS) in (s.n // 2, (s.n + 1) // 2)
        xu, stu, iu = _solve(sol.A, sol.M, b[None], 0, 1e-10)
        xf, stf, inf = _solve(sol.A, sol.M, b[None], 1, 1e-10)
    assert stu == stf == rs.OK
    assert np.linalg.norm(xf - xu) <= 1e-10 * np.linalg.norm(xu)
    assert abs(inf[0]["half_steps"] - iu[0]["half_steps"]) <= max(2, 0.05 * iu[0]["half_steps"])
    xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[0], b, ordering=rs.ORDER_GRAPH_COLOUR, reduction=1e-10)
    assert np.linalg.norm(xf[0] - xo) <= 1e-8 * np.linalg.norm(xo)


@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
def test_apply_outside_a_solve_ignores_the_solvers_state(precision):
    """With FP64 factors the upper launch of the rows without lower blocks
    reads their rows of A' (the factorisation stores no U for them) in every
    application.  A preconditioner application after a finished solve (whose
    systems are all done) and GMRES's end-of-cycle application compute every
    system: ilu0_apply gives the same bits before and after a solve, with
    one launch per level and with single-launch sweeps (which read U, filled
    from A' on first use)."""
    s = make_ensemble(12, 10, 7, seeds=[41, 42, 43])
    v = np.random.default_rng(3).standard_normal((s.batch, s.n, 3))
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR, precision=precision) as sol:
        sol.factor()
        assert rs.ilu0_get_option(sol.M, rs.OPT_FUSED_ROWS) > 0
        z0 = rs.ilu0_apply(sol.M, v, None, 0, s.batch)
        sol.solve(s.b[:, 0], reduction=1e-8)
        z1 = rs.ilu0_apply(sol.M, v, None, 0, s.batch)
        rs.ilu0_set_option(sol.M, rs.OPT_SWEEP_TILES, 1)
        z2 = rs.ilu0_apply(sol.M, v, None, 0, s.batch)
        sol.factor()                                   # U of the fused rows dropped again
        z3 = rs.ilu0_apply(sol.M, v, None, 0, s.batch)
        lu, dinv = rs.ilu0_get_factors(sol.M, 1, s.n, s.nnzb)
    assert np.array_equal(z0, z1) and np.array_equal(z0, z2) and np.array_equal(z0, z3)
    perm = oracle.ordering_perm(s.rowptr, s.colidx, rs.ORDER_GRAPH_COLOUR)
    prow, pcol, pv = oracle.permute(s.rowptr, s.colidx, s.vals[1], perm)
    st, _, olu, odinv = oracle.ilu0(prow, pcol, pv)
    assert st == oracle.OK
    if precision == rs.PREC_FP64:       # U of the fused rows, filled from A', is the oracle's U
        offd = np.array([pcol[p] != i for i in range(s.n) for p in range(prow[i], prow[i + 1])], bool)
        assert np.abs(lu[offd] - olu[offd]).max() <= 1e-12 * np.abs(olu[offd]).max()
        assert np.abs(dinv - odinv).max() <= 1e-12 * np.abs(odinv).max()


def _solves(sol, b, red):
    """BiCGStab with the fused iteration, BiCGStab without it, GMRES(5) and
    one application per system, on the current options."""
    out = []
    for fuse in (1, 0):
        rs.ilu0_set_option(sol.M, rs.OPT_FUSE_SPMV, fuse)
        out.append(rs.bicgstab_solve(sol.M, sol.A, b, reduction=red))
    rs.ilu0_set_option(sol.M, rs.OPT_FUSE_SPMV, 1)
    out.append(rs.gmres_solve(sol.M, sol.A, b, restart=5, reduction=red))
    v = np.ascontiguousarray(b.reshape(b.shape[0], -1, 3))
    out.append(rs.ilu0_apply(sol.M, v, None, 0, b.shape[0]))
    return out


@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
@pytest.mark.parametrize("grid", [(20, 20, 10), (7, 5, 3), (9, 1, 1), (33, 17, 5)])
def test_y_from_the_input_gives_the_same_bits(grid, precision):
    """Bipartite grids under graph colouring: the applications read the y
    of the first colour from their input and store no y (RS_OPT_Y_INPUT).
    Every result -- BiCGStab with and without the fused iteration, GMRES
    and a lone application, on a batch of two systems, graphs replayed --
    has the same bits as with y stored, and the solve meets the oracle."""
    s = make_ensemble(*grid, seeds=[sum(grid), sum(grid) + 1])
    b = s.b[:, 0]
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR, precision=precision) as sol:
        assert sol.factor()[0] == rs.OK
        # the lower parts need y from the input; they round differently
        rs.ilu0_set_option(sol.M, rs.OPT_LOWER_PARTS, 0)
        assert rs.ilu0_get_option(sol.M, rs.OPT_Y_INPUT_PATTERN) == 1
        assert rs.ilu0_get_option(sol.M, rs.OPT_Y_INPUT) == 1
        on = _solves(sol, b, 1e-10)
        rs.ilu0_set_option(sol.M, rs.OPT_Y_INPUT, 0)
        off = _solves(sol, b, 1e-10)
        rs.ilu0_set_option(sol.M, rs.OPT_Y_INPUT, 1)
        again = _solves(sol, b, 1e-10)
    for a, c, d in zip(on[:3], off[:3], again[:3]):
        assert a[1] == c[1] == d[1] == rs.OK
        assert np.array_equal(a[0], c[0]) and np.array_equal(a[0], d[0])
        assert outcome(a[2]) == outcome(c[2]) == outcome(d[2])
    assert np.array_equal(on[3], off[3]) and np.array_equal(on[3], again[3])
    for k in range(s.batch):
        xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[k], s.b[k, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                             reduction=1e-10)
        assert np.linalg.norm(on[0][0][k] - xo) <= 1e-8 * np.linalg.norm(xo)


def test_y_from_the_input_stays_off_where_the_pattern_does_not_allow_it():
    """Level sets on a grid (many lower levels), a grid with non-neighbour
    connections under colouring (more than two colours), single-row islands
    (no fused rows), and single-launch sweeps: y is stored, and the solves
    match the oracle."""
    grid = make_grid_system(12, 9, 7, seed=3)
    nnc = make_grid_system(12, 9, 7, nnc_frac=0.02, seed=6)
    islands = make_grid_system(15, 11, 7, active_frac=0.45, seed=8)
    for s, ordering in ((grid, rs.ORDER_LEVEL_SET), (nnc, rs.ORDER_GRAPH_COLOUR), (islands, rs.ORDER_GRAPH_COLOUR)):
        with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=ordering) as sol:
            sol.factor()
            assert rs.ilu0_get_option(sol.M, rs.OPT_Y_INPUT_PATTERN) == 0
            x, st, info = sol.solve(s.b[:, 0], reduction=1e-10)
        xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering, reduction=1e-10)
        assert st == rs.OK and np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)
    with rs.Solver(grid.rowptr, grid.colidx, grid.vals, ordering=rs.ORDER_GRAPH_COLOUR) as sol:
        sol.factor()
        assert rs.ilu0_get_option(sol.M, rs.OPT_Y_INPUT_PATTERN) == 1
        xl, _, il = sol.solve(grid.b[:, 0], reduction=1e-10)
        rs.ilu0_set_option(sol.M, rs.OPT_SWEEP_TILES, 1)
        xt, _, it = sol.solve(grid.b[:, 0], reduction=1e-10)
    xo, _ = oracle.solve(grid.rowptr, grid.colidx, grid.vals[0], grid.b[0, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                         reduction=1e-10)
    for x in (xl, xt):
        assert np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)
    with pytest.raises(rs.RsolveError):
        with rs.Solver(grid.rowptr, grid.colidx, grid.vals) as sol:
            rs.ilu0_set_option(sol.M, rs.OPT_Y_INPUT_PATTERN, 1)


@pytest.mark.parametrize("grid", [(20, 20, 10), (7, 5, 3), (33, 17, 5)])
def test_lower_parts_agree_with_the_lower_launch(grid):
    """FP64 factors, bipartite grids under graph colouring: BiCGStab's second
    application with its lower parts formed in v = A phat
    (RS_OPT_LOWER_PARTS) agrees with the lower launch that reads L to
    rounding (x within 1e-10 at a reduction of 1e-10, half steps within 2),
    on a batch of two with graphs replayed and eager; each configuration is
    deterministic and the batch members equal their solves alone."""
    s = make_ensemble(*grid, seeds=[sum(grid) + 7, sum(grid) + 8])
    b = s.b[:, 0]
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR) as sol:
        sol.factor()
        assert rs.ilu0_get_option(sol.M, rs.OPT_LOWER_PARTS) == 1
        x1, st1, i1 = sol.solve(b, reduction=1e-10)
        x1b, _, i1b = sol.solve(b, reduction=1e-10)
        rs.ilu0_set_option(sol.M, rs.OPT_USE_GRAPH, 0)
        x1e, _, i1e = sol.solve(b, reduction=1e-10)
        rs.ilu0_set_option(sol.M, rs.OPT_USE_GRAPH, 1)
        rs.ilu0_set_option(sol.M, rs.OPT_LOWER_PARTS, 0)
        x0, st0, i0 = sol.solve(b, reduction=1e-10)
    assert st1 == st0 == rs.OK
    assert np.array_equal(x1, x1b) and np.array_equal(x1, x1e) and outcome(i1) == outcome(i1b) == outcome(i1e)
    for k in range(s.batch):
        assert np.linalg.norm(x1[k] - x0[k]) <= 1e-10 * np.linalg.norm(x0[k])
        assert abs(i1[k]["half_steps"] - i0[k]["half_steps"]) <= 2
        assert i1[k]["true_rel_residual"] <= 1e-9
        with rs.Solver(s.rowptr, s.colidx, s.vals[k:k + 1], ordering=rs.ORDER_GRAPH_COLOUR) as one:
            one.factor()
            xa, _, ia = one.solve(s.b[k:k + 1, 0], reduction=1e-10)
        assert np.array_equal(xa[0], x1[k]) and outcome(ia) == outcome([i1[k]])
