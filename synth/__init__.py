"""Seeded synthetic block-sparse systems that stand in for reservoir Jacobians.

This module only draws random inputs: it builds a BCSR pattern from a
Cartesian grid (7-point stencil, optional active-cell mask, optional
non-neighbour connections) and fills 3x3 FP64 blocks.  It contains none of
the solver's arithmetic (no factorisation, no sweep, no Krylov step), so both
the CPU oracle and the HIP path may read what it returns.

The paper's workloads (NORNE, NORNE refined, a 1M-cell proprietary model;
Section "Benchmarks", table of benchmark characteristics) are not available;
these grids reproduce their shape class: 3 unknowns per cell, about 7 blocks
per block row, structurally symmetric, numerically non-symmetric matrices
(Section "OPM Flow" states the assembled systems are non-symmetric and
ill-conditioned).
"""

from .grids import (  # noqa: F401
    GridSystem,
    make_grid_system,
    make_ensemble,
    config_system,
    serving_classes,
    CONFIGS,
)
from .wells import Wells, make_wells  # noqa: F401
