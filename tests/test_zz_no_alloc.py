"""ilu0_apply_noalloc, the preconditioner application for callers that
cannot allocate device memory: through the C ABI it gives ilu0_apply's
result bit for bit (same kernels, intermediates in the library's fixed
per-GPU workspace), on consecutive calls whose second input is smaller, in
every sweep mode and precision, and it refuses inputs beyond the
workspace."""

import numpy as np
import pytest

import paper_2309_11488_amd as rs
from synth import make_ensemble, make_grid_system

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _factored(s, ordering, precision, tiles):
    sol = rs.Solver(s.rowptr, s.colidx, s.vals, ordering=ordering, precision=precision)
    rs.ilu0_set_option(sol.M, rs.OPT_SWEEP_TILES, tiles)
    st, _ = sol.factor()
    assert st == rs.OK
    return sol


def _check_pair(sol, first_sys, n_sys, seed):
    """ilu0_apply vs ilu0_apply_noalloc on the same device input."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.randn(n_sys * sol.n * 3, generator=g, dtype=torch.float64).cuda()
    z_ref = torch.zeros_like(v)
    rs.ilu0_apply(sol.M, v, z_ref, first_sys, n_sys)
    z = torch.full_like(v, float("nan"))
    rs.ilu0_apply_noalloc(sol.M, v, z, first_sys, n_sys)
    torch.cuda.synchronize()
    assert torch.equal(z, z_ref), (z - z_ref).abs().max().item()
    assert torch.isfinite(z).all()


@pytest.mark.parametrize("precision", [rs.PREC_FP64, rs.PREC_FP32_FACTORS])
@pytest.mark.parametrize("tiles", [0, 1])
@pytest.mark.parametrize("ordering", [rs.ORDER_GRAPH_COLOUR, rs.ORDER_LEVEL_SET])
def test_noalloc_apply_equals_apply(ordering, tiles, precision):
    """Two calls in a row, the second on a smaller system of another handle
    (whose tile counts differ, so the workspace still holds the first
    call's flags and epochs), then the first handle again with fewer
    systems: every result equals ilu0_apply's bit for bit."""
    big = make_ensemble(23, 17, 11, seeds=[3, 4, 5])
    small = make_grid_system(9, 7, 5, active_frac=0.9, nnc_frac=0.03, seed=8)
    with _factored(big, ordering, precision, tiles) as a, _factored(small, ordering, precision, tiles) as b:
        _check_pair(a, 0, 3, seed=1)
        _check_pair(b, 0, 1, seed=2)
        _check_pair(a, 1, 2, seed=3)
        _check_pair(a, 2, 1, seed=4)


def test_noalloc_apply_after_a_full_solve():
    """The handle's own workspace and the library's fixed one do not
    interfere: solve, apply without allocating, solve again."""
    s = make_grid_system(21, 13, 8, active_frac=0.85, nnc_frac=0.02, seed=12, sigma=2.0)
    with _factored(s, rs.ORDER_LEVEL_SET, rs.PREC_FP64, 1) as sol:
        x1, st1, i1 = sol.solve(s.b[:, 0], reduction=1e-8)
        _check_pair(sol, 0, 1, seed=5)
        x2, st2, i2 = sol.solve(s.b[:, 0], reduction=1e-8)
        assert st1 == st2 == rs.OK and np.array_equal(x1, x2)
        assert i1[0]["half_steps"] == i2[0]["half_steps"]


def test_noalloc_apply_rejects_inputs_beyond_its_workspace():
    """25 systems of 48 000 block rows need three vectors of 3.6M doubles
    each, above the fixed workspace: a clear RS_OUT_OF_MEMORY; 20 fit."""
    s = make_grid_system(40, 40, 30, seed=0)
    vals = np.repeat(s.vals, 25, axis=0)
    with rs.Solver(s.rowptr, s.colidx, vals, ordering=rs.ORDER_GRAPH_COLOUR) as sol:
        assert sol.factor()[0] == rs.OK
        v = torch.zeros(25 * sol.n * 3, dtype=torch.float64, device="cuda")
        z = torch.zeros_like(v)
        with pytest.raises(rs.RsolveError) as e:
            rs.ilu0_apply_noalloc(sol.M, v, z, 0, 25)
        assert e.value.status == rs.OUT_OF_MEMORY and "workspace" in str(e.value)
        _check_pair(sol, 5, 20, seed=6)


def test_noalloc_apply_argument_errors():
    s = make_grid_system(6, 5, 4, seed=1)
    with rs.Solver(s.rowptr, s.colidx, s.vals) as sol:
        v = torch.zeros(sol.n * 3, dtype=torch.float64, device="cuda")
        with pytest.raises(rs.RsolveError) as e:
            rs.ilu0_apply_noalloc(sol.M, v, v.clone(), 0, 1)
        assert e.value.status == rs.NOT_FACTORED
        sol.factor()
        with pytest.raises(rs.RsolveError) as e:
            rs.ilu0_apply_noalloc(sol.M, v, v.clone(), 0, 2)
        assert e.value.status == rs.INVALID_ARG
        with pytest.raises(TypeError):
            rs.ilu0_apply_noalloc(sol.M, np.zeros(sol.n * 3), np.zeros(sol.n * 3), 0, 1)
