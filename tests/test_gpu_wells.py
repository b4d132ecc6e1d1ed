"""GPU parity of standard wells kept separate (Section "Well Contributions",
Algorithm 5): products with A subtract C^T D^-1 B x for every well."""

import numpy as np
import pytest

import oracle
import paper_2309_11488_amd as rs
from synth import make_ensemble, make_grid_system, make_wells

pytestmark = pytest.mark.gpu

ORDERINGS = [rs.ORDER_NATURAL, rs.ORDER_LEVEL_SET, rs.ORDER_GRAPH_COLOUR, rs.ORDER_RCM_LEVEL_SET]


def system():
    s = make_grid_system(14, 11, 9, active_frac=0.9, nnc_frac=0.02, seed=51)
    return s, make_wells(s, 6, seed=52)


def wells_args(w, k=0):
    return w.well_ptr, w.perf_row, w.B[k], w.C[k], w.Dinv[k]


def test_spmv_with_wells_matches_oracle():
    s, w = system()
    A = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
    try:
        rs.bcsr_set_wells(A, w.well_ptr, w.perf_row, w.B, w.C, w.Dinv)
        x = np.random.default_rng(1).standard_normal((1, s.n, 3))
        y = rs.bcsr_spmv(A, x)
        yo = oracle.wells_apply(w.well_ptr, w.perf_row, w.B[0], w.C[0], w.Dinv[0], x[0],
                                oracle.spmv(s.rowptr, s.colidx, s.vals[0], x[0]))
        assert np.abs(y[0] - yo).max() <= 1e-13 * np.abs(yo).max()
        rs.bcsr_set_wells(A)                                  # removed: plain SpMV again
        y2 = rs.bcsr_spmv(A, x)
        assert np.abs(y2[0] - oracle.spmv(s.rowptr, s.colidx, s.vals[0], x[0])).max() <= 1e-13 * np.abs(yo).max()
    finally:
        rs.bcsr_destroy(A)


@pytest.mark.parametrize("ordering", ORDERINGS)
@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
def test_solve_with_wells_matches_oracle(ordering, precision):
    s, w = system()
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=ordering, precision=precision) as sol:
        rs.bcsr_set_wells(sol.A, w.well_ptr, w.perf_row, w.B, w.C, w.Dinv)
        sol.factor()
        x, st, info = sol.solve(s.b[:, 0], reduction=1e-10)
    prec = oracle.PREC_ILU_F64 if precision == rs.PREC_FP64 else oracle.PREC_ILU_F32
    xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=ordering, precond=prec,
                             reduction=1e-10, wells=wells_args(w))
    assert st == oinfo["status"] == rs.OK
    tol = 1e-8 if precision == rs.PREC_FP64 else 1e-7      # FP32 sweeps: summation order not pinned
    assert np.linalg.norm(x[0] - xo) <= tol * np.linalg.norm(xo)
    # the well terms are summed in another order than the oracle's; over the
    # 20+ erratic BiCGStab iterations a well-coupled system needs at 1e-10,
    # the two runs stop a few half steps apart (x and the true residual agree)
    assert abs(info[0]["half_steps"] - oinfo["half_steps"]) <= max(2, oinfo["half_steps"] // 5)
    assert info[0]["true_rel_residual"] <= 1e-9


def test_wells_in_a_batch_equal_each_system_alone():
    s = make_ensemble(10, 9, 7, seeds=[3, 4, 5])
    w = make_wells(s, 4, seed=6, batch=3)
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR) as sol:
        rs.bcsr_set_wells(sol.A, w.well_ptr, w.perf_row, w.B, w.C, w.Dinv)
        sol.factor()
        xb, st, infos = sol.solve(s.b[:, 0], reduction=1e-10)
    assert st == rs.OK
    for k in range(3):
        with rs.Solver(s.rowptr, s.colidx, s.vals[k:k + 1], ordering=rs.ORDER_GRAPH_COLOUR) as one:
            rs.bcsr_set_wells(one.A, w.well_ptr, w.perf_row, w.B[k:k + 1], w.C[k:k + 1], w.Dinv[k:k + 1])
            one.factor()
            x1, st1, i1 = one.solve(s.b[k:k + 1, 0], reduction=1e-10)
        assert np.array_equal(xb[k], x1[0]) and infos[k]["half_steps"] == i1[0]["half_steps"]
        xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[k], s.b[k, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                             reduction=1e-10, wells=wells_args(w, k))
        assert np.linalg.norm(xb[k] - xo) <= 1e-8 * np.linalg.norm(xo)


def test_changing_wells_between_solves_rebuilds_their_mapping():
    s, w = system()
    w2 = make_wells(s, 3, seed=77)
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_LEVEL_SET) as sol:
        sol.factor()
        results = []
        for wells in (w, w2, None):
            if wells is None:
                rs.bcsr_set_wells(sol.A)
            else:
                rs.bcsr_set_wells(sol.A, wells.well_ptr, wells.perf_row, wells.B, wells.C, wells.Dinv)
            results.append(sol.solve(s.b[:, 0], reduction=1e-10))
    for (x, st, info), wells in zip(results, (w, w2, None)):
        xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_LEVEL_SET,
                             reduction=1e-10, wells=None if wells is None else wells_args(wells))
        assert st == rs.OK and np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)


def test_bad_wells_are_rejected():
    s, w = system()
    A = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
    try:
        bad_rows = w.perf_row.copy()
        bad_rows[0] = s.n
        with pytest.raises(rs.RsolveError) as e:
            rs.bcsr_set_wells(A, w.well_ptr, bad_rows, w.B, w.C, w.Dinv)
        assert e.value.status == rs.INVALID_ARG
        bad_ptr = w.well_ptr.copy()
        bad_ptr[0] = 1
        with pytest.raises(rs.RsolveError):
            rs.bcsr_set_wells(A, bad_ptr, w.perf_row, w.B, w.C, w.Dinv)
    finally:
        rs.bcsr_destroy(A)


@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
def test_fused_iteration_with_wells(precision):
    """A full grid under graph colouring with wells, a batch of two: the
    fused iteration (RS_OPT_FUSE_SPMV) forms the first colour's rows of v
    and t without their well terms and subtracts them once the whole x of
    the product is known, correcting both dot products; it agrees with the
    unfused iteration to rounding, and both match the oracle."""
    s = make_ensemble(16, 13, 9, seeds=[63, 64])
    w = make_wells(s, 7, seed=65, batch=2)
    b = s.b[:, 0]
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR, precision=precision) as sol:
        rs.bcsr_set_wells(sol.A, w.well_ptr, w.perf_row, w.B, w.C, w.Dinv)
        sol.factor()
        n0 = rs.ilu0_get_option(sol.M, rs.OPT_FUSED_ROWS)
        assert n0 > 0
        xf, stf, inf = sol.solve(b, reduction=1e-10)
        xf2, _, inf2 = sol.solve(b, reduction=1e-10)
        rs.ilu0_set_option(sol.M, rs.OPT_FUSE_SPMV, 0)
        xu, stu, inu = sol.solve(b, reduction=1e-10)
    assert stf == stu == rs.OK
    assert np.array_equal(xf, xf2) and [i["half_steps"] for i in inf] == [i["half_steps"] for i in inf2]
    prec = oracle.PREC_ILU_F64 if precision == rs.PREC_FP64 else oracle.PREC_ILU_F32
    tol = 1e-8 if precision == rs.PREC_FP64 else 1e-7
    for k in range(2):
        assert np.linalg.norm(xf[k] - xu[k]) <= tol * np.linalg.norm(xu[k])
        xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[k], s.b[k, 0], ordering=rs.ORDER_GRAPH_COLOUR,
                                 precond=prec, reduction=1e-10, wells=wells_args(w, k))
        assert oinfo["status"] == rs.OK
        assert np.linalg.norm(xf[k] - xo) <= tol * np.linalg.norm(xo)
        assert inf[k]["true_rel_residual"] <= 1e-9
