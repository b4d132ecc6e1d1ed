"""Seeded standard wells for the grid systems (inputs only, no solver arithmetic).

A standard well couples the cells it perforates through one extra block
equation: B (one block row, a 4x3 block per perforated cell), C (the same
shape) and the inverse of its 4x4 diagonal block D.  The paper's separate
well application subtracts C^T D^-1 B x from A x for every well (Section
"Well Contributions"); its matrices come from the simulator, so here they are
drawn:

* wells are vertical: ``n_wells`` distinct (i, j) columns of the grid, drawn
  uniformly; each perforates the active cells of its column from a random
  top layer down to a random bottom layer (at least one cell);
* a perforation's well index WI = the geometric mean permeability scale
  ``exp(N(0, sigma^2))``;
* B_p = WI_p (E + 0.1 U(-1,1)^{4x3}) and C_p = WI_p (E + 0.1 U(-1,1)^{4x3})
  with E = [I_3; (1 1 1)/3] (the fourth equation is the well's control);
* D^-1 = (I + 0.1 U(-1,1)^{4x4}) / (2 sum_p WI_p), drawn directly as the
  inverse (the simulator stores D^-1).

Draws come from ``numpy.random.Generator(PCG64(seed))`` in this order:
columns, then per well (top, bottom), then per perforation WI, B noise,
C noise, then per well the D^-1 noise.  ``batch`` members draw their values
(not the placement) from seed + 1, seed + 2, ...
"""

from __future__ import annotations

import dataclasses

import numpy as np

_E = np.vstack([np.eye(3), np.full((1, 3), 1.0 / 3.0)])


@dataclasses.dataclass
class Wells:
    """Standard wells of one pattern: ``well_ptr[w]..well_ptr[w+1]`` index the
    perforations of well w, ``perf_row`` their block rows.  Values per batch
    member: ``B``/``C`` (batch, n_perf, 4, 3), ``Dinv`` (batch, n_wells, 4, 4)."""

    well_ptr: np.ndarray
    perf_row: np.ndarray
    B: np.ndarray
    C: np.ndarray
    Dinv: np.ndarray

    @property
    def n_wells(self) -> int:
        return int(len(self.well_ptr) - 1)

    @property
    def n_perf(self) -> int:
        return int(len(self.perf_row))


def _values(rng, well_ptr, sigma):
    n_perf = int(well_ptr[-1])
    wi = np.exp(sigma * rng.standard_normal(n_perf))
    B = wi[:, None, None] * (_E[None] + 0.1 * rng.uniform(-1.0, 1.0, size=(n_perf, 4, 3)))
    C = wi[:, None, None] * (_E[None] + 0.1 * rng.uniform(-1.0, 1.0, size=(n_perf, 4, 3)))
    nw = len(well_ptr) - 1
    tot = np.add.reduceat(wi, well_ptr[:-1]) if nw else np.zeros(0)
    Dinv = (np.eye(4)[None] + 0.1 * rng.uniform(-1.0, 1.0, size=(nw, 4, 4))) / (2.0 * tot)[:, None, None]
    return B, C, Dinv


def make_wells(system, n_wells: int, *, seed: int = 0, sigma: float = 1.0, batch: int = 1) -> Wells:
    """Vertical standard wells on ``system``'s grid (see the module recipe)."""
    nx, ny, nz = system.shape
    cell_row = system.cell_row
    if cell_row is None:
        raise ValueError("system carries no cell -> row map")
    rng = np.random.Generator(np.random.PCG64(seed))
    n_wells = min(n_wells, nx * ny)
    cols = rng.choice(nx * ny, size=n_wells, replace=False)
    ptr, rows = [0], []
    for c in cols:
        top, bottom = sorted(rng.integers(0, nz, 2))
        i, j = int(c) % nx, int(c) // nx
        perf = [cell_row[i + nx * (j + ny * k)] for k in range(top, bottom + 1)]
        perf = [r for r in perf if r >= 0]
        if not perf:                          # every cell of the range inactive: take any active cell
            act = np.flatnonzero(cell_row >= 0)
            perf = [int(cell_row[act[int(c) % len(act)]])]
        rows.extend(perf)
        ptr.append(len(rows))
    well_ptr = np.asarray(ptr, np.int32)
    perf_row = np.asarray(rows, np.int32)
    Bs, Cs, Ds = [], [], []
    for m in range(batch):
        r = rng if m == 0 else np.random.Generator(np.random.PCG64(seed + m))
        B, C, D = _values(r, well_ptr, sigma)
        Bs.append(B)
        Cs.append(C)
        Ds.append(D)
    return Wells(well_ptr=well_ptr, perf_row=perf_row, B=np.stack(Bs), C=np.stack(Cs), Dinv=np.stack(Ds))
