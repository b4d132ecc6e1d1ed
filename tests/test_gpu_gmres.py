"""GPU parity of restarted GMRES (the simulator's alternative Krylov solver,
Section "OPM Flow") on the same factors, sweeps and SpMV as BiCGStab,
against the oracle's GMRES(m)."""

import numpy as np
import pytest

import oracle
import paper_2309_11488_amd as rs
from synth import config_system, make_ensemble, make_grid_system, make_wells
from tests.helpers import chain_pattern, random_values

pytestmark = pytest.mark.gpu

ORDERINGS = [rs.ORDER_NATURAL, rs.ORDER_LEVEL_SET, rs.ORDER_GRAPH_COLOUR]


def system():
    # 1266 active cells: 3798 unknowns, four 1024-entry tiles of the vector
    # kernels with a ragged tail
    return make_grid_system(14, 11, 9, active_frac=0.9, nnc_frac=0.02, seed=71)


def oprec(precision):
    return oracle.PREC_ILU_F64 if precision == rs.PREC_FP64 else oracle.PREC_ILU_F32


@pytest.mark.parametrize("ordering", ORDERINGS)
@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
@pytest.mark.parametrize("restart", [5, 30])
def test_gmres_matches_oracle(ordering, precision, restart):
    s = system()
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=ordering, precision=precision) as sol:
        sol.factor()
        x, st, info = sol.solve_gmres(s.b[:, 0], restart=restart, reduction=1e-10, max_iter=1000)
    xo, oinfo = oracle.solve_gmres(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering,
                                   precond=oprec(precision), restart=restart, reduction=1e-10, max_iter=1000)
    assert st == oinfo["status"] == rs.OK, (info, oinfo)
    tol = 1e-8 if precision == rs.PREC_FP64 else 1e-7      # FP32 sweeps: summation order not pinned
    assert np.linalg.norm(x[0] - xo) <= tol * np.linalg.norm(xo)
    # within a cycle the estimate never grows, so rounding moves the step
    # at which it crosses the threshold by at most one
    assert abs(info[0]["half_steps"] - oinfo["half_steps"]) <= 1, (info, oinfo)
    assert info[0]["r0_norm"] == pytest.approx(oinfo["r0_norm"], rel=1e-14)
    if precision == rs.PREC_FP64:
        assert info[0]["true_rel_residual"] <= 1e-9
    else:
        # x += M^-1 (V y) applies the FP32 sweeps to a combination of the
        # basis, which is not exactly the combination of the sweeps applied to
        # each basis vector: the true residual stalls near FP32 rounding while
        # the estimate goes on falling, the oracle's alike
        assert info[0]["true_rel_residual"] <= 1e-5
        assert info[0]["true_rel_residual"] == pytest.approx(oinfo["true_rel_residual"], rel=0.5)


def test_gmres_step_limit_matches_oracle():
    """Stopping on the step limit mid-cycle: the same steps, the same x."""
    s = system()
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_LEVEL_SET) as sol:
        sol.factor()
        for restart, max_iter in ((3, 7), (4, 8), (30, 1)):
            x, st, info = sol.solve_gmres(s.b[:, 0], restart=restart, reduction=1e-14, max_iter=max_iter)
            xo, oinfo = oracle.solve_gmres(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_LEVEL_SET,
                                           restart=restart, reduction=1e-14, max_iter=max_iter)
            assert st == oinfo["status"] == rs.NOT_CONVERGED
            assert info[0]["half_steps"] == oinfo["half_steps"] == max_iter
            assert np.linalg.norm(x[0] - xo) <= 1e-12 * np.linalg.norm(xo)
            assert info[0]["final_norm"] == pytest.approx(oinfo["final_norm"], rel=1e-9)


def test_gmres_trace_matches_oracle():
    """With no reduction target the solve stops on the step limit, and its
    residual estimate equals the oracle's after the same number of steps,
    for every count (restarts included)."""
    s = make_grid_system(9, 8, 5, nnc_frac=0.02, seed=72)
    perm = oracle.ordering_perm(s.rowptr, s.colidx, oracle.ORDER_COLOUR)
    prow, pcol, pv = oracle.permute(s.rowptr, s.colidx, s.vals[0], perm)
    _, _, lu, dinv = oracle.ilu0(prow, pcol, pv)
    _, _, tr = oracle.gmres(prow, pcol, pv, lu, dinv, s.b[0, 0][perm], restart=6, reduction=0.0, max_iter=20,
                            trace=True)
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR) as sol:
        sol.factor()
        for k in range(1, 21):
            _, st, info = sol.solve_gmres(s.b[:, 0], restart=6, reduction=0.0, max_iter=k)
            assert st == rs.NOT_CONVERGED and info[0]["half_steps"] == k
            assert info[0]["final_norm"] == pytest.approx(tr[k - 1], rel=1e-9), k


def test_gmres_batch_equals_alone():
    e = make_ensemble(10, 9, 6, range(73, 77), sigma=1.0, n_rhs=1)
    with rs.Solver(e.rowptr, e.colidx, e.vals, ordering=rs.ORDER_GRAPH_COLOUR) as sol:
        sol.factor()
        xb, st, infob = sol.solve_gmres(e.b[:, 0], restart=8, reduction=1e-9, max_iter=400)
    assert st == rs.OK
    for k in range(e.vals.shape[0]):
        with rs.Solver(e.rowptr, e.colidx, e.vals[k:k + 1], ordering=rs.ORDER_GRAPH_COLOUR) as sol:
            sol.factor()
            xa, _, infoa = sol.solve_gmres(e.b[k:k + 1, 0], restart=8, reduction=1e-9, max_iter=400)
        assert np.array_equal(xa[0], xb[k])
        assert infoa[0]["half_steps"] == infob[k]["half_steps"]
        xo, oinfo = oracle.solve_gmres(e.rowptr, e.colidx, e.vals[k], e.b[k, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                                       restart=8, reduction=1e-9, max_iter=400)
        assert np.linalg.norm(xb[k] - xo) <= 1e-7 * np.linalg.norm(xo)
        assert abs(infob[k]["half_steps"] - oinfo["half_steps"]) <= 1


def test_gmres_exact_preconditioner_one_step():
    """A block-tridiagonal chain has no fill-in: ILU0 is exact and GMRES
    stops after one step, as the oracle does."""
    rowptr, colidx = chain_pattern(40)
    vals = random_values(rowptr, colidx, seed=74)
    b = np.random.default_rng(75).standard_normal((1, 40, 3))
    with rs.Solver(rowptr, colidx, vals[None], ordering=rs.ORDER_NATURAL) as sol:
        sol.factor()
        x, st, info = sol.solve_gmres(b, restart=10, reduction=1e-12, max_iter=10)
    xo, oinfo = oracle.solve_gmres(rowptr, colidx, vals, b[0], restart=10, reduction=1e-12, max_iter=10)
    assert st == oinfo["status"] == rs.OK
    assert info[0]["half_steps"] == oinfo["half_steps"] == 1
    assert np.linalg.norm(x[0] - xo) <= 1e-12 * np.linalg.norm(xo)


def test_gmres_degenerate_inputs():
    s = make_grid_system(6, 5, 4, seed=76)
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_LEVEL_SET) as sol:
        sol.factor()
        x, st, info = sol.solve_gmres(np.zeros((1, s.n, 3)), restart=5, max_iter=10)
        assert st == rs.OK and info[0]["half_steps"] == 0 and not x.any()
        x, st, info = sol.solve_gmres(s.b[:, 0], restart=5, max_iter=0)
        assert st == rs.NOT_CONVERGED and info[0]["half_steps"] == 0 and not x.any()
        for restart in (0, rs.GMRES_MAX_RESTART + 1):
            with pytest.raises(rs.RsolveError):
                sol.solve_gmres(s.b[:, 0], restart=restart)
        x, st, info = sol.solve_gmres(s.b[:, 0], restart=rs.GMRES_MAX_RESTART, reduction=1e-8, max_iter=300)
        assert st == rs.OK and info[0]["true_rel_residual"] <= 1e-7


def test_gmres_then_bicgstab_on_one_handle():
    """GMRES and BiCGStab share the handle's workspace and states."""
    s = system()
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR) as sol:
        sol.factor()
        x1, _, i1 = sol.solve(s.b[:, 0], reduction=1e-8)
        sol.solve_gmres(s.b[:, 0], restart=10, reduction=1e-8, max_iter=500)
        x2, _, i2 = sol.solve(s.b[:, 0], reduction=1e-8)
    assert np.array_equal(x1, x2) and i1[0]["half_steps"] == i2[0]["half_steps"]


@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
def test_gmres_full_size_96k(precision):
    """The 96k-cell grid with non-neighbour connections at the solver's
    working reduction 1e-2, graph colouring, GMRES(30)."""
    s = config_system("c2")
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR, precision=precision) as sol:
        sol.factor()
        x, st, info = sol.solve_gmres(s.b[:, 0], restart=30, reduction=1e-2, max_iter=300)
    xo, oinfo = oracle.solve_gmres(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                                   precond=oprec(precision), restart=30, reduction=1e-2, max_iter=300)
    assert st == oinfo["status"] == rs.OK
    assert abs(info[0]["half_steps"] - oinfo["half_steps"]) <= 1
    if info[0]["half_steps"] == oinfo["half_steps"]:
        tol = 1e-9 if precision == rs.PREC_FP64 else 1e-6
        assert np.linalg.norm(x[0] - xo) <= tol * np.linalg.norm(xo)
    assert info[0]["true_rel_residual"] <= 1e-2


@pytest.mark.parametrize("ordering", ORDERINGS)
@pytest.mark.parametrize("restart", [4, 30])
def test_gmres_with_wells_matches_oracle(ordering, restart):
    """Standard wells kept separate (Algorithm 5) in every product with A."""
    s = make_grid_system(14, 11, 9, active_frac=0.9, nnc_frac=0.02, seed=51)
    w = make_wells(s, 6, seed=52)
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=ordering) as sol:
        rs.bcsr_set_wells(sol.A, w.well_ptr, w.perf_row, w.B, w.C, w.Dinv)
        sol.factor()
        x, st, info = sol.solve_gmres(s.b[:, 0], restart=restart, reduction=1e-10, max_iter=2000)
    xo, oinfo = oracle.solve_gmres(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering, restart=restart,
                                   reduction=1e-10, max_iter=2000,
                                   wells=(w.well_ptr, w.perf_row, w.B[0], w.C[0], w.Dinv[0]))
    assert st == oinfo["status"] == rs.OK
    assert np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)
    assert abs(info[0]["half_steps"] - oinfo["half_steps"]) <= 1, (info, oinfo)
    assert info[0]["true_rel_residual"] <= 1e-9
    assert info[0]["true_rel_residual"] == pytest.approx(oinfo["true_rel_residual"], rel=0.5, abs=1e-12)


def test_fused_gmres_steps_with_wells():
    """A full grid under graph colouring with wells: GMRES's fused steps
    (the upper launch forms the first colour's rows of w) take those rows'
    well terms after the SpMV; the solve matches the oracle, and the
    unfused steps to rounding."""
    s = make_grid_system(16, 13, 9, seed=71)
    w = make_wells(s, 7, seed=72)
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR) as sol:
        rs.bcsr_set_wells(sol.A, w.well_ptr, w.perf_row, w.B, w.C, w.Dinv)
        sol.factor()
        assert rs.ilu0_get_option(sol.M, rs.OPT_FUSED_ROWS) > 0
        xf, stf, inf = sol.solve_gmres(s.b[:, 0], restart=30, reduction=1e-10, max_iter=2000)
        rs.ilu0_set_option(sol.M, rs.OPT_FUSE_SPMV, 0)
        xu, stu, inu = sol.solve_gmres(s.b[:, 0], restart=30, reduction=1e-10, max_iter=2000)
    xo, oinfo = oracle.solve_gmres(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                                   restart=30, reduction=1e-10, max_iter=2000,
                                   wells=(w.well_ptr, w.perf_row, w.B[0], w.C[0], w.Dinv[0]))
    assert stf == stu == oinfo["status"] == rs.OK
    assert np.linalg.norm(xf[0] - xo) <= 1e-8 * np.linalg.norm(xo)
    assert np.linalg.norm(xf[0] - xu[0]) <= 1e-8 * np.linalg.norm(xu[0])
    assert abs(inf[0]["half_steps"] - oinfo["half_steps"]) <= 1, (inf, oinfo)
    assert inf[0]["true_rel_residual"] <= 1e-9
