"""Host-side checks of the C-ABI library (no GPU): it loads, exports every
declared symbol, and its host analysis (validation, orderings) matches the
oracle's independent implementation of the same definitions."""

import os
import re

import numpy as np
import pytest

import oracle
import paper_2309_11488_amd as rs
from synth import config_system, make_grid_system
from tests.helpers import chain_pattern, pattern_from_pairs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "rsolve.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert "bicgstab_solve" in names and "ilu0_factor" in names and len(names) >= 15
    L = rs.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(rs.EXPORTS)


def test_status_strings():
    assert rs.status_string(rs.OK) == "ok"
    assert rs.status_string(rs.ZERO_PIVOT) == "zero pivot"
    assert rs.status_string(12345) == "unknown status"


@pytest.mark.parametrize("ordering", [rs.ORDER_NATURAL, rs.ORDER_LEVEL_SET, rs.ORDER_GRAPH_COLOUR,
                                      rs.ORDER_RCM_LEVEL_SET])
@pytest.mark.parametrize("case", ["c1", "mask_nnc", "c2", "random", "hub", "mask_only"])
def test_host_ordering_matches_oracle(ordering, case):
    if case == "c1":
        s = config_system("c1")
    elif case == "c2":
        s = config_system("c2", n_rhs=1)
    elif case == "random":
        # irregular degrees and many ties of saturation and degree
        rng = np.random.default_rng(8)
        pairs = {(int(a), int(b)) for a, b in rng.integers(0, 300, (900, 2)) if a != b}
        rp, ci = pattern_from_pairs(300, sorted(pairs))
        s = type("P", (), {"rowptr": rp, "colidx": ci, "n": 300})
    elif case == "hub":
        # a row with 400 neighbours (past the bucketed queue's degree bound)
        # on a graph that is not bipartite
        rng = np.random.default_rng(9)
        pairs = {(0, k) for k in range(1, 401)}
        pairs |= {(int(a), int(b)) for a, b in rng.integers(1, 500, (800, 2)) if a != b}
        rp, ci = pattern_from_pairs(500, sorted(pairs))
        s = type("P", (), {"rowptr": rp, "colidx": ci, "n": 500})
    elif case == "mask_only":
        # bipartite, in many components, some of them single rows
        s = make_grid_system(15, 11, 7, active_frac=0.45, nnc_frac=0.0, seed=4)
    else:
        s = make_grid_system(15, 11, 7, active_frac=0.8, nnc_frac=0.04, seed=3)
    st, perm, ns, bad = rs.ilu0_analyse_host(s.rowptr, s.colidx, ordering)
    assert st == rs.OK and bad == -1
    if ordering == rs.ORDER_LEVEL_SET:
        nl, _, operm = oracle.level_sets(s.rowptr, s.colidx)
        assert ns == nl
    elif ordering == rs.ORDER_GRAPH_COLOUR:
        nc, _, operm = oracle.dsatur_colour(s.rowptr, s.colidx)
        assert ns == nc
    elif ordering == rs.ORDER_RCM_LEVEL_SET:
        nl, _, operm = oracle.rcm_levels(s.rowptr, s.colidx)
        assert ns == nl
    else:
        operm = np.arange(s.n, dtype=np.int32)
        assert ns == s.n
    assert np.array_equal(perm, operm)


def test_host_analysis_rejects_bad_patterns():
    rowptr, colidx = chain_pattern(5)
    assert rs.ilu0_analyse_host(rowptr, colidx)[0] == rs.OK
    c = colidx.copy()
    c[3], c[4] = c[4], c[3]
    st, _, _, bad = rs.ilu0_analyse_host(rowptr, c)
    assert (st, bad) == (rs.BAD_PATTERN, 1)
    c = colidx.copy()
    c[-1] = 9
    assert rs.ilu0_analyse_host(rowptr, c)[0] == rs.BAD_PATTERN
    rp, ci = pattern_from_pairs(4, [(0, 1), (2, 3)])
    drop = [p for p in range(len(ci)) if not (ci[p] == 1 and rp[1] <= p < rp[2])]
    rows = np.repeat(np.arange(4), np.diff(rp))[drop]
    rp2 = np.zeros(5, np.int32)
    np.cumsum(np.bincount(rows, minlength=4), out=rp2[1:])
    st, _, _, bad = rs.ilu0_analyse_host(rp2, ci[drop])
    assert (st, bad) == (rs.MISSING_DIAGONAL, 1)


def test_host_analysis_nonsymmetric_pattern():
    # (0,2) present without (2,0): orderings still valid permutations
    rowptr = np.array([0, 2, 4, 5], np.int32)
    colidx = np.array([0, 2, 0, 1, 2], np.int32)
    for ordering in (0, 1, 2, 3):
        st, perm, ns, _ = rs.ilu0_analyse_host(rowptr, colidx, ordering)
        assert st == rs.OK
        assert sorted(perm.tolist()) == [0, 1, 2]
        operm = oracle.ordering_perm(rowptr, colidx, ordering)
        assert np.array_equal(perm, operm)


@pytest.mark.parametrize("parts", [1, 3, 8, 50])
def test_partition_is_balanced_and_deterministic(parts):
    s = make_grid_system(9, 7, 6, active_frac=0.9, nnc_frac=0.03, seed=12)
    part = rs.bcsr_partition(s.rowptr, s.colidx, parts, weights=s.trans)
    assert part.shape == (s.n,) and part.min() == 0 and part.max() == parts - 1
    sizes = np.bincount(part, minlength=parts)
    assert sizes.max() - sizes.min() <= 1
    assert np.array_equal(part, rs.bcsr_partition(s.rowptr, s.colidx, parts, weights=s.trans))


def test_partition_keeps_strong_couplings_inside():
    """Two tightly coupled chains joined by weak links split along the weak links."""
    n = 40
    pairs = [(i, i + 1) for i in range(19)] + [(i, i + 1) for i in range(20, 39)] + [(i, i + 20) for i in range(20)]
    rowptr, colidx = pattern_from_pairs(n, pairs)
    w = np.zeros(len(colidx))
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            j = colidx[p]
            w[p] = 100.0 if abs(i - j) == 1 and (i < 20) == (j < 20) else 1e-3
    part = rs.bcsr_partition(rowptr, colidx, 2, weights=w)
    assert (part[:20] == part[0]).all() and (part[20:] == part[20]).all() and part[0] != part[20]
    cut_weak = rs.bcsr_partition(rowptr, colidx, 2)                 # unweighted: grown breadth-first
    assert np.bincount(cut_weak).tolist() == [20, 20]


def test_partition_rejects_bad_input():
    s = make_grid_system(4, 3, 2, seed=1)
    with pytest.raises(rs.RsolveError):
        rs.bcsr_partition(s.rowptr, s.colidx, 0)
    bad = s.colidx.copy()
    bad[[0, 1]] = bad[[1, 0]]
    with pytest.raises(rs.RsolveError) as e:
        rs.bcsr_partition(s.rowptr, bad, 2)
    assert e.value.status == rs.BAD_PATTERN
