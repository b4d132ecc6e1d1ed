"""GPU checks of the solver's contract beyond plain parity: breakdown
statuses, same-trajectory comparison with the oracle at full size and with
wells, recovery after a sweep wait gives up, the bounded poll prediction,
and the device phase times every solve reports."""

import time

import numpy as np
import pytest

import oracle
import paper_2309_11488_amd as rs
from synth import config_system, make_grid_system, make_wells
from tests.helpers import BREAKDOWN_CASES, breakdown_as_well, outcome, trajectory_check

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ordering", [rs.ORDER_NATURAL, rs.ORDER_LEVEL_SET])
@pytest.mark.parametrize("case", sorted(BREAKDOWN_CASES))
def test_breakdown_statuses_on_the_gpu(case, ordering):
    """Each breakdown branch of BiCGStab, reached on the GPU: the identity
    matrix with one standard well kept separate makes the operator the 3x3
    block K while ILU0 of A is the identity, so the device runs plain
    BiCGStab on K.  Every quantity is exact in FP64, so the status, the half
    steps and x (after omega = 0, x keeps its half-step update) equal the
    hand-derived values and the oracle's bit for bit."""
    c = BREAKDOWN_CASES[case]
    K = np.asarray(c["K"], np.float64)
    b = np.asarray(c["b"], np.float64).reshape(1, 1, 3)
    rp, ci, vals, wp, pr, B, C, Dinv = breakdown_as_well(K)
    with rs.Solver(rp, ci, vals, ordering=ordering) as sol:
        rs.bcsr_set_wells(sol.A, wp, pr, B, C, Dinv)
        st, _ = sol.factor()
        assert st == rs.OK
        x, st, info = sol.solve(b, reduction=0.1)
    assert st == info[0]["status"] == rs.BREAKDOWN
    assert info[0]["half_steps"] == c["half"]
    assert np.array_equal(x[0].ravel(), np.asarray(c["x"], np.float64))
    xo, oinfo = oracle.solve(rp, ci, vals[0], b[0, 0], ordering=ordering, reduction=0.1,
                             wells=(wp, pr, B[0], C[0], Dinv[0]))
    assert oinfo["status"] == oracle.BREAKDOWN and oinfo["half_steps"] == info[0]["half_steps"]
    assert np.array_equal(xo, x[0])


def oracle_runner(s, ordering, prec, b, wells=None):
    """The oracle's path with its per-iteration trace: (reduction, max_iter)
    -> (x in caller order, info, trace)."""
    perm = oracle.ordering_perm(s.rowptr, s.colidx, ordering)
    prow, pcol, pv = oracle.permute(s.rowptr, s.colidx, s.vals[0], perm)
    st, _, lu, dinv = oracle.ilu0(prow, pcol, pv)
    assert st == oracle.OK
    pw = None
    if wells is not None:
        iperm = np.empty_like(perm)
        iperm[perm] = np.arange(len(perm), dtype=perm.dtype)
        pw = (wells[0], iperm[np.asarray(wells[1], np.int32)], wells[2], wells[3], wells[4])
    bp = np.ascontiguousarray(b.reshape(-1, 3)[perm])

    def run(reduction, max_iter):
        xp, info, tr = oracle.bicgstab(prow, pcol, pv, lu, dinv, bp, precond=prec, reduction=reduction,
                                       max_iter=max_iter, trace=True, wells=pw)
        x = np.empty_like(xp)
        x[perm] = xp
        return x, info, tr
    return run


def test_c3_full_size_same_trajectory():
    """The 100^3 grid (sigma 2) at full size in the benchmark's configuration
    (graph colouring, autotuned launch shapes, FP64 factors): GPU and oracle
    run the same number of full iterations with no stopping test (reduction
    0): equal statuses and half steps, x within 1e-8; then at 1e-10, x
    within 1e-8 and equal half-step counts wherever the oracle's residual
    crosses the threshold by more than the two sides' observed deviation."""
    s = config_system("c3")
    b = s.b[0, 0]
    A = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
    M = rs.ilu0_analyse(A, rs.ORDER_GRAPH_COLOUR)
    try:
        st, _ = rs.ilu0_factor(M, A, rs.PREC_FP64)
        assert st == rs.OK
        rs.ilu0_autotune(M, A, s.b[:, 0], reduction=1e-2, reps=1)

        def gpu(red, max_iter):
            x, st, info = rs.bicgstab_solve(M, A, b[None], reduction=red, max_iter=max_iter)
            return x[0], st, info[0]
        run = oracle_runner(s, rs.ORDER_GRAPH_COLOUR, oracle.PREC_ILU_F64, b)
        dev, decisive = trajectory_check(gpu, run, 1e-10, 1e-8, rs.NOT_CONVERGED)
        print(f"c3 trajectory: final-norm deviation {dev:.2e}, decisive {decisive}")
    finally:
        rs.ilu0_destroy(M)
        rs.bcsr_destroy(A)


@pytest.mark.parametrize("ordering", [rs.ORDER_LEVEL_SET, rs.ORDER_GRAPH_COLOUR, rs.ORDER_RCM_LEVEL_SET])
def test_wells_same_trajectory(ordering):
    """Standard wells kept separate (Algorithm 5 in every product with A):
    the same fixed-iteration comparison, then the solve at 1e-10."""
    s = make_grid_system(14, 11, 9, active_frac=0.9, nnc_frac=0.02, seed=51)
    w = make_wells(s, 6, seed=52)
    b = s.b[0, 0]
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=ordering) as sol:
        rs.bcsr_set_wells(sol.A, w.well_ptr, w.perf_row, w.B, w.C, w.Dinv)
        sol.factor()

        def gpu(red, max_iter):
            x, st, info = sol.solve(b[None], reduction=red, max_iter=max_iter)
            return x[0], st, info[0]
        run = oracle_runner(s, ordering, oracle.PREC_ILU_F64, b,
                            wells=(w.well_ptr, w.perf_row, w.B[0], w.C[0], w.Dinv[0]))
        trajectory_check(gpu, run, 1e-10, 1e-8, rs.NOT_CONVERGED)


def test_recovery_after_a_sweep_wait_gives_up():
    """With a spin limit of zero the single-launch sweeps' dependency waits
    give up (every launch still ends); the solve reports RS_HIP_ERROR and the
    handle resets its sweep counters and tile flags.  With the default limit
    restored, the next solves on the same handle equal those of a fresh
    handle bit for bit and match the oracle."""
    s = make_grid_system(17, 13, 9, active_frac=0.85, nnc_frac=0.03, seed=4, sigma=2.0)
    b = s.b[:, 0]
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_LEVEL_SET) as ref:
        ref.factor()
        xr, str_, ir = ref.solve(b, reduction=1e-10)
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_LEVEL_SET) as sol:
        assert rs.ilu0_get_option(sol.M, rs.OPT_SWEEP_TILES) == 1
        default = rs.ilu0_get_option(sol.M, rs.OPT_SPIN_LIMIT)
        sol.factor()
        sol.solve(b, reduction=1e-10)                     # epochs advanced before the failure
        rs.ilu0_set_option(sol.M, rs.OPT_SPIN_LIMIT, 0)
        failed = 0
        for _ in range(5):
            try:
                sol.solve(b, reduction=1e-10)
            except rs.RsolveError as e:
                assert e.status == rs.HIP_ERROR
                failed += 1
                break
        assert failed, "no dependency wait gave up with a zero spin limit"
        rs.ilu0_set_option(sol.M, rs.OPT_SPIN_LIMIT, default)
        for _ in range(3):
            x, st, info = sol.solve(b, reduction=1e-10)
            assert st == str_ == rs.OK
            assert np.array_equal(x, xr) and outcome(info) == outcome(ir)
    xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[0], b[0], ordering=rs.ORDER_LEVEL_SET, reduction=1e-10)
    assert np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)


def test_prediction_learns_only_from_converged_solves():
    """The first poll comes after as many iterations as the last converged
    solve needed: a tight solve followed by a loose one, and a solve that
    ends at max_iter followed by a normal one, give the results of a fresh
    handle, and the iterations queued past convergence after the failed
    solve do not cost another max_iter of launches."""
    s = make_grid_system(16, 12, 8, seed=31)
    b = s.b[:, 0]
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR) as fresh:
        fresh.factor()
        x2, _, i2 = fresh.solve(b, reduction=1e-2)
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR) as sol:
        sol.factor()
        _, st, tight = sol.solve(b, reduction=1e-12)
        assert st == rs.OK and tight[0]["half_steps"] > 4 * i2[0]["half_steps"]
        x, st, info = sol.solve(b, reduction=1e-2)
        assert np.array_equal(x, x2) and outcome(info) == outcome(i2)
        _, st, failed = sol.solve(b, reduction=0.0, max_iter=150)
        assert st in (rs.NOT_CONVERGED, rs.BREAKDOWN) and failed[0]["half_steps"] > 100
        t = time.perf_counter()
        x, st, info = sol.solve(b, reduction=1e-2)
        wall = time.perf_counter() - t
        assert np.array_equal(x, x2) and outcome(info) == outcome(i2)
        # the prediction still comes from the converged solve at 1e-12 (at most
        # 50 iterations), not from the 150 iterations of the failed one
        assert info[0]["solve_ms"] < 0.5 * failed[0]["solve_ms"], (info[0]["solve_ms"], failed[0]["solve_ms"])
        assert info[0]["solve_ms"] <= wall * 1e3 * 1.01 + 0.05


def test_phase_times_are_reported():
    """solve_info carries the device time of the factorisation the solve
    used and of the solve itself (HIP events on the caller's stream)."""
    s = make_grid_system(20, 20, 10, seed=2)
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR,
                   precision=rs.PREC_FP32_FACTORS) as sol:
        t = time.perf_counter()
        sol.factor()
        fwall = (time.perf_counter() - t) * 1e3
        t = time.perf_counter()
        x, st, info = sol.solve(s.b[:, 0], reduction=1e-6)
        swall = (time.perf_counter() - t) * 1e3
        assert st == rs.OK
        assert 0 < info[0]["factor_ms"] <= fwall * 1.01 + 0.05
        assert 0 < info[0]["solve_ms"] <= swall * 1.01 + 0.05
        x, st, ig = sol.solve_gmres(s.b[:, 0], reduction=1e-6)
        assert ig[0]["factor_ms"] == info[0]["factor_ms"] and ig[0]["solve_ms"] > 0


def test_rcm_ordering_shortens_the_nnc_schedule():
    """On the 46x112x22 grid with 2% non-neighbour connections, level sets
    after the reverse Cuthill-McKee renumbering need a small fraction of the
    plain level schedule's levels; the schedule is the oracle's."""
    s = config_system("c2", n_rhs=1)
    A = rs.bcsr_create(s.rowptr, s.colidx, s.vals)
    M1 = rs.ilu0_analyse(A, rs.ORDER_LEVEL_SET)
    M3 = rs.ilu0_analyse(A, rs.ORDER_RCM_LEVEL_SET)
    try:
        _, n1, _ = rs.ilu0_get_schedule(M1, s.n)
        perm, n3, sp = rs.ilu0_get_schedule(M3, s.n)
        nl, level, operm = oracle.rcm_levels(s.rowptr, s.colidx)
        assert np.array_equal(perm, operm) and n3 == nl
        assert n3 * 20 < n1
        assert rs.ilu0_get_option(M3, rs.OPT_SWEEP_TILES) == 0       # few wide levels: a launch per level
    finally:
        rs.ilu0_destroy(M1)
        rs.ilu0_destroy(M3)
        rs.bcsr_destroy(A)


def test_queued_factorisation_gives_the_same_results():
    """RS_OPT_FACTOR_ASYNC: ilu0_factor only queues the factorisation.  The
    solves that follow on the same stream give the bits of the waiting
    call's solves, report the factorisation's device time, and
    ilu0_factor_status gives the waiting call's status.  A singular pivot in
    one system of a batch surfaces as RS_ZERO_PIVOT in that system's solve
    status and in ilu0_factor_status with the waiting call's bad rows."""
    s = make_grid_system(20, 20, 10, seed=4)
    batch = 3
    vals = np.repeat(s.vals, batch, axis=0)
    vals[1] *= 1.5
    b = np.repeat(s.b[:, 0], batch, axis=0)
    bad_vals = vals.copy()
    bad_vals[2, s.rowptr[777]:s.rowptr[778]] = 0.0
    for prec in (rs.PREC_FP64, rs.PREC_FP32_FACTORS):
        with rs.Solver(s.rowptr, s.colidx, vals, ordering=rs.ORDER_GRAPH_COLOUR, precision=prec) as sol:
            with pytest.raises(rs.RsolveError) as e:
                rs.ilu0_factor_status(sol.M, batch)
            assert e.value.status == rs.NOT_FACTORED
            assert rs.ilu0_get_option(sol.M, rs.OPT_FACTOR_ASYNC) == 0
            assert sol.factor()[0] == rs.OK
            x0, st0, i0 = sol.solve(b, reduction=1e-8)
            rs.ilu0_set_option(sol.M, rs.OPT_FACTOR_ASYNC, 1)
            st, bad = sol.factor()
            assert st == rs.OK and list(bad) == [-1] * batch
            x1, st1, i1 = sol.solve(b, reduction=1e-8)
            assert st0 == st1 == rs.OK and np.array_equal(x0, x1) and outcome(i0) == outcome(i1)
            assert all(i["factor_ms"] > 0 for i in i1)
            st, bad = rs.ilu0_factor_status(sol.M, batch)
            assert st == rs.OK and list(bad) == [-1] * batch
            # a singular pivot in system 2
            rs.ilu0_set_option(sol.M, rs.OPT_FACTOR_ASYNC, 0)
            sst, sbad = sol.factor(bad_vals)
            assert sst == rs.ZERO_PIVOT and sbad[2] >= 0 and sbad[0] == sbad[1] == -1
            rs.ilu0_set_option(sol.M, rs.OPT_FACTOR_ASYNC, 1)
            st, _ = sol.factor(bad_vals)
            assert st == rs.OK
            x2, st2, i2 = sol.solve(b, reduction=1e-8)
            assert st2 == rs.ZERO_PIVOT
            assert [i["status"] for i in i2] == [rs.OK, rs.OK, rs.ZERO_PIVOT]
            assert np.array_equal(x2[:2], x0[:2])
            qst, qbad = rs.ilu0_factor_status(sol.M, batch)
            assert qst == rs.ZERO_PIVOT and np.array_equal(qbad, sbad)
            # the answer stays until the next factorisation
            assert rs.ilu0_factor_status(sol.M, batch)[0] == rs.ZERO_PIVOT
