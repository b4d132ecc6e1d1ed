"""GPU tests of the request server: admission under a memory budget,
overlap of concurrent requests, and results that do not depend on the mix."""

import numpy as np
import pytest

import oracle
import paper_2309_11488_amd as rs
from synth import config_system, make_grid_system
from tests.helpers import outcome

pytestmark = pytest.mark.gpu


def systems():
    out = [make_grid_system(12, 10, 8, seed=1), make_grid_system(12, 10, 8, seed=2),
           make_grid_system(20, 15, 6, seed=3), make_grid_system(9, 9, 9, nnc_frac=0.02, seed=4),
           make_grid_system(30, 20, 10, sigma=2.0, seed=5)]
    return out


SYS = systems()


def requests(n):
    rng = np.random.default_rng(0)
    return [SYS[int(k)] for k in rng.integers(0, len(SYS), n)]


def register(srv, systems):
    return {id(s): srv.add_pattern(s.rowptr, s.colidx) for s in systems}


def test_results_same_alone_and_in_the_mix():
    reqs = requests(24)
    with rs.Server(max_slots=1, ordering=rs.ORDER_GRAPH_COLOUR) as alone:
        pid = register(alone, SYS)
        ref = []
        for s in reqs:
            t = alone.submit(pid[id(s)], s.vals[0], s.b[0, 0], reduction=1e-8)
            ref.append(alone.wait(t))
    with rs.Server(max_slots=4, ordering=rs.ORDER_GRAPH_COLOUR) as mix:
        pid = register(mix, SYS)
        tickets = [mix.submit(pid[id(s)], s.vals[0], s.b[0, 0], reduction=1e-8) for s in reqs]
        got = [mix.wait(t) for t in tickets]
        slots = {g[3]["slot"] for g in got}
        stats = mix.stats()
    assert len(slots) > 1
    # one analysis per pattern (SYS[0] and SYS[1] share theirs), shared by every instance of it
    assert stats["analyses"] == 4 and stats["evicted"] == 0
    for (x1, st1, i1, _), (x2, st2, i2, _) in zip(ref, got):
        assert st1 == st2 == rs.OK
        assert np.array_equal(x1, x2) and outcome(i1) == outcome(i2)


def test_results_match_oracle():
    with rs.Server(max_slots=3, ordering=rs.ORDER_LEVEL_SET, precision=rs.PREC_FP64) as srv:
        pid = register(srv, SYS)
        tickets = [(s, srv.submit(pid[id(s)], s.vals[0], s.b[0, 0], reduction=1e-10)) for s in SYS]
        for s, t in tickets:
            x, st, info, tm = srv.wait(t)
            xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_LEVEL_SET,
                                 reduction=1e-10)
            assert st == rs.OK and np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
            assert info["true_rel_residual"] <= 1e-9
            assert tm["total_ms"] >= tm["solve_ms"] > 0


def test_budget_is_never_exceeded_and_oversize_is_refused():
    big = SYS[4]
    need = rs.Server.request_bytes(big.n, big.nnzb) + rs.Server.analysis_bytes(big.n, big.nnzb)
    budget = int(need * 1.5)          # room for one resident instance of this size
    reqs = requests(12)
    with rs.Server(hbm_budget_bytes=budget, max_slots=4) as srv:
        pid = register(srv, SYS)
        tickets = [(s, srv.submit(pid[id(s)], s.vals[0], s.b[0, 0], reduction=1e-6)) for s in reqs]
        for s, t in tickets:
            x, st, info, _ = srv.wait(t)
            assert st == rs.OK and info["true_rel_residual"] <= 1e-6 * (1 + 1e-6)
        stats = srv.stats()
        assert stats["completed"] == len(reqs) and stats["peak_reserved_bytes"] <= budget
        assert stats["evicted"] > 0 and stats["reserved_bytes"] <= budget
    with rs.Server(hbm_budget_bytes=need - 1, max_slots=2) as srv:
        with pytest.raises(rs.RsolveError) as e:
            srv.add_pattern(big.rowptr, big.colidx)
        assert e.value.status == rs.OUT_OF_MEMORY


def test_poll_then_wait_and_ticket_release():
    s = SYS[4]
    with rs.Server(max_slots=1) as srv:
        p = srv.add_pattern(s.rowptr, s.colidx)
        ts = [srv.submit(p, s.vals[0], s.b[0, 0], reduction=1e-10) for _ in range(4)]
        early = srv.poll(ts[-1])                # one slot, four requests: usually still queued
        results = [early] if early is not None else []
        for t in (ts[:-1] if early is not None else ts):
            results.append(srv.wait(t))
        assert all(r[1] == rs.OK for r in results)
        with pytest.raises(rs.RsolveError):     # a collected ticket is released
            srv.wait(ts[0])


def test_instances_share_one_analysis_and_match_a_standalone_solver():
    s = SYS[2]
    with rs.Solver(s.rowptr, s.colidx, s.vals, ordering=rs.ORDER_GRAPH_COLOUR, precision=rs.PREC_FP32_FACTORS) as ref:
        ref.factor()
        xr, str_, ir = ref.solve(s.b[:, 0], reduction=1e-8)
    with rs.Server(max_slots=4, ordering=rs.ORDER_GRAPH_COLOUR) as srv:
        p = srv.add_pattern(s.rowptr, s.colidx)
        assert srv.add_pattern(s.rowptr.copy(), s.colidx.copy()) == p      # same pattern, same id
        ts = [srv.submit(p, s.vals[0], s.b[0, 0], reduction=1e-8) for _ in range(16)]
        got = [srv.wait(t) for t in ts]
        stats = srv.stats()
    assert stats["analyses"] == 1 and 1 <= stats["created"] <= 4 and stats["evicted"] == 0
    assert any(g[3]["resident"] for g in got)
    for x, st, info, _ in got:
        assert st == str_ == rs.OK
        assert np.array_equal(x, xr[0]) and info["half_steps"] == ir[0]["half_steps"]


def test_autotuned_server_matches_oracle():
    with rs.Server(max_slots=2, ordering=rs.ORDER_LEVEL_SET, precision=rs.PREC_FP64, autotune=True) as srv:
        pid = register(srv, SYS)
        tickets = [(s, srv.submit(pid[id(s)], s.vals[0], s.b[0, 0], reduction=1e-10)) for s in SYS + SYS]
        for s, t in tickets:
            x, st, info, tm = srv.wait(t)
            xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_LEVEL_SET,
                                 reduction=1e-10)
            assert st == rs.OK and np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)


def test_autotuned_results_same_alone_and_in_the_mix():
    """With the launch-shape autotuner on (the benchmark's serving setup),
    requests of a pattern wait until its tuner has ended, so every request of
    the pattern runs one launch configuration: each request's result is the
    same bit for bit whether it ran alone (submitted and collected one at a
    time) or in a mix of concurrent requests on the same server."""
    reqs = requests(20)
    with rs.Server(max_slots=4, ordering=rs.ORDER_GRAPH_COLOUR, autotune=True) as srv:
        pid = register(srv, SYS)
        alone = []
        for s in reqs:
            t = srv.submit(pid[id(s)], s.vals[0], s.b[0, 0], reduction=1e-8)
            alone.append(srv.wait(t))
        tickets = [srv.submit(pid[id(s)], s.vals[0], s.b[0, 0], reduction=1e-8) for s in reqs]
        mixed = [srv.wait(t) for t in tickets]
    assert len({g[3]["slot"] for g in mixed}) > 1
    for (x1, st1, i1, _), (x2, st2, i2, _) in zip(alone, mixed):
        assert st1 == st2 == rs.OK
        assert np.array_equal(x1, x2) and outcome(i1) == outcome(i2)


def test_one_million_cell_request_matches_oracle():
    """A request of the largest size class (the 100^3 grid, sigma 2)
    through the server, FP64 factors, reduction 1e-10: x within 1e-8 of the
    oracle's solution under the same ordering."""
    s = config_system("c3")
    b = s.b[0, 0]
    with rs.Server(max_slots=2, ordering=rs.ORDER_GRAPH_COLOUR, precision=rs.PREC_FP64) as srv:
        p = srv.add_pattern(s.rowptr, s.colidx)
        x, st, info, tm = srv.wait(srv.submit(p, s.vals[0], b, reduction=1e-10))
    assert st == rs.OK and info["true_rel_residual"] <= 1e-9
    xo, oinfo = oracle.solve(s.rowptr, s.colidx, s.vals[0], b, ordering=rs.ORDER_GRAPH_COLOUR, reduction=1e-10)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"1M-cell request: rel err vs oracle {err:.2e}, half steps {info['half_steps']} "
          f"(oracle {oinfo['half_steps']}), total {tm['total_ms']:.1f} ms")
    assert err <= 1e-8


def test_bad_pattern_and_unknown_pattern_are_rejected():
    s = SYS[0]
    with rs.Server(max_slots=1) as srv:
        c = s.colidx.copy()
        r0, r1 = s.rowptr[0], s.rowptr[1]
        c[r0:r1] = c[r0:r1][::-1]                       # unsorted first row
        with pytest.raises(rs.RsolveError) as e:
            srv.add_pattern(s.rowptr, c)
        assert e.value.status == rs.BAD_PATTERN and e.value.bad_row == 0
        with pytest.raises(rs.RsolveError) as e:
            srv.submit(7, s.vals[0], s.b[0, 0])
        assert e.value.status == rs.INVALID_ARG
