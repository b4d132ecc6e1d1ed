"""GPU tests of the request server: admission under a memory budget,
overlap of concurrent requests, and results that do not depend on the mix."""

import numpy as np
import pytest

import oracle
import paper_2309_11488_amd as rs
from synth import make_grid_system

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


def test_results_same_alone_and_in_the_mix():
    reqs = requests(24)
    with rs.Server(max_slots=1, ordering=rs.ORDER_GRAPH_COLOUR) as alone:
        ref = []
        for s in reqs:
            t = alone.submit(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], reduction=1e-8)
            ref.append(alone.wait(t))
    with rs.Server(max_slots=4, ordering=rs.ORDER_GRAPH_COLOUR) as mix:
        tickets = [mix.submit(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], reduction=1e-8) for s in reqs]
        got = [mix.wait(t) for t in tickets]
        slots = {g[3]["slot"] for g in got}
    assert len(slots) > 1
    for (x1, st1, i1, _), (x2, st2, i2, _) in zip(ref, got):
        assert st1 == st2 == rs.OK
        assert np.array_equal(x1, x2) and i1 == i2


def test_results_match_oracle():
    with rs.Server(max_slots=3, ordering=rs.ORDER_LEVEL_SET, precision=rs.PREC_FP64) as srv:
        tickets = [(s, srv.submit(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], reduction=1e-10)) for s in SYS]
        for s, t in tickets:
            x, st, info, tm = srv.wait(t)
            xo, _ = oracle.solve(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], ordering=rs.ORDER_LEVEL_SET,
                                 reduction=1e-10)
            assert st == rs.OK and np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
            assert info["true_rel_residual"] <= 1e-9
            assert tm["total_ms"] >= tm["solve_ms"] > 0


def test_budget_is_never_exceeded_and_oversize_is_refused():
    big = SYS[4]
    need = rs.Server.request_bytes(big.n, big.nnzb)
    budget = int(need * 1.5)          # room for one resident request of this size
    reqs = requests(12)
    with rs.Server(hbm_budget_bytes=budget, max_slots=4) as srv:
        tickets = [(s, srv.submit(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], reduction=1e-6)) for s in reqs]
        for s, t in tickets:
            x, st, info, _ = srv.wait(t)
            assert st == rs.OK and info["true_rel_residual"] <= 1e-6 * (1 + 1e-6)
        stats = srv.stats()
        assert stats["completed"] == len(reqs) and stats["peak_reserved_bytes"] <= budget
    with rs.Server(hbm_budget_bytes=need - 1, max_slots=2) as srv:
        with pytest.raises(rs.RsolveError) as e:
            srv.submit(big.rowptr, big.colidx, big.vals[0], big.b[0, 0])
        assert e.value.status == rs.OUT_OF_MEMORY


def test_poll_then_wait_and_ticket_release():
    s = SYS[4]
    with rs.Server(max_slots=1) as srv:
        ts = [srv.submit(s.rowptr, s.colidx, s.vals[0], s.b[0, 0], reduction=1e-10) for _ in range(4)]
        early = srv.poll(ts[-1])                # one slot, four requests: usually still queued
        results = [early] if early is not None else []
        for t in (ts[:-1] if early is not None else ts):
            results.append(srv.wait(t))
        assert all(r[1] == rs.OK for r in results)
        with pytest.raises(rs.RsolveError):     # a collected ticket is released
            srv.wait(ts[0])
