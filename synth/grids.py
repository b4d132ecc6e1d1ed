"""Cartesian-grid BCSR generator with 3x3 FP64 blocks.

Recipe (all draws from one ``numpy.random.Generator(PCG64(seed))`` in this
order, so a seed fixes the system bit for bit):

1. active-cell mask: Bernoulli(active_frac) per cell (skipped when
   ``active_frac`` is None, i.e. all cells active);
2. log-permeability: ``log k_i ~ N(0, sigma^2)`` per active cell;
3. accumulation scale ``a_i ~ U(0.5, 1.5)`` per active cell;
4. non-neighbour connections (NNCs): ``round(nnc_frac * n_conn)`` unordered
   pairs of distinct active cells drawn uniformly, rejecting self pairs and
   pairs that already exist (stencil or earlier NNC);
5. coupling ``C_ij = I + 0.2 U(-1,1)^{3x3}`` per *directed* connection;
6. diagonal perturbation ``0.1 U(-1,1)^{3x3}`` per active cell;
7. right-hand sides ``N(0,1)`` per scalar entry, ``n_rhs`` vectors.

Cells are numbered i fastest, then j, then k; active cells keep that order
when compressed to block rows.  Transmissibility is the harmonic mean
``T_ij = 2 k_i k_j / (k_i + k_j)``.  The off-diagonal block at (i, j) is
``-T_ij C_ij``; the diagonal block is ``a_i (I + 0.1 U) + sum_j T_ij C_ij``
using row i's own couplings, so every block row sums to ``a_i (I + 0.1 U)``.
Blocks are stored row-major, block rows with ascending, unique column
indices.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class GridSystem:
    """A BCSR system (or a same-pattern batch of systems) and its right-hand sides.

    ``vals`` has shape ``(batch, nnzb, 3, 3)`` and ``b`` shape
    ``(batch, n_rhs, n, 3)``; ``rowptr``/``colidx`` are int32.
    ``trans`` holds ``T_ij`` for every stored off-diagonal block (0 on the
    diagonal), so a transmissibility-weighted partitioner can read it.
    """

    n: int
    rowptr: np.ndarray
    colidx: np.ndarray
    vals: np.ndarray
    b: np.ndarray
    trans: np.ndarray
    shape: tuple
    name: str = ""
    cell_row: np.ndarray | None = None   # grid cell (i fastest) -> block row, -1 if inactive

    @property
    def nnzb(self) -> int:
        return int(self.colidx.shape[0])

    @property
    def batch(self) -> int:
        return int(self.vals.shape[0])


def _stencil_pairs(nx: int, ny: int, nz: int) -> tuple[np.ndarray, np.ndarray]:
    """Undirected 7-point neighbour pairs (cell ids), x then y then z."""
    c3 = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    us = [c3[:, :, :-1].ravel(), c3[:, :-1, :].ravel(), c3[:-1, :, :].ravel()]
    vs = [c3[:, :, 1:].ravel(), c3[:, 1:, :].ravel(), c3[1:, :, :].ravel()]
    return np.concatenate(us), np.concatenate(vs)


def _draw_nncs(rng: np.random.Generator, n: int, m: int, existing: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Draw ``m`` new unordered pairs (u < v) of distinct rows, none in ``existing``.

    ``existing`` holds keys ``u * n + v`` (u < v) of connections already present.
    """
    taken = set(existing.tolist()) if m > 0 else set()
    out_u: list[int] = []
    out_v: list[int] = []
    while len(out_u) < m:
        need = m - len(out_u)
        cand = rng.integers(0, n, size=(need, 2))
        for p, q in cand:
            if p == q:
                continue
            u, v = (int(p), int(q)) if p < q else (int(q), int(p))
            key = u * n + v
            if key in taken:
                continue
            taken.add(key)
            out_u.append(u)
            out_v.append(v)
            if len(out_u) == m:
                break
    return np.asarray(out_u, dtype=np.int64), np.asarray(out_v, dtype=np.int64)


def _pattern(nx, ny, nz, rng, active_frac, nnc_frac):
    ncell = nx * ny * nz
    if active_frac is None:
        active = np.ones(ncell, dtype=bool)
    else:
        active = rng.random(ncell) < active_frac
    cell2row = np.full(ncell, -1, dtype=np.int64)
    n = int(active.sum())
    cell2row[active] = np.arange(n, dtype=np.int64)
    cu, cv = _stencil_pairs(nx, ny, nz)
    keep = active[cu] & active[cv]
    u = cell2row[cu[keep]]
    v = cell2row[cv[keep]]
    return n, u, v, cell2row


def _assemble(n, u, v, k, a, cmat, dpert):
    """Blocks from the drawn fields; returns rowptr, colidx, vals, trans.

    Every block is written straight to its sorted position (row, then
    column), so no unsorted copy of the values is ever materialised.
    """
    trans_u = 2.0 * k[u] * k[v] / (k[u] + k[v])
    du = np.concatenate([u, v])
    dv = np.concatenate([v, u])
    dt = np.concatenate([trans_u, trans_u])
    m = du.shape[0]
    rows = np.concatenate([du, np.arange(n, dtype=np.int64)])
    cols = np.concatenate([dv, np.arange(n, dtype=np.int64)])
    order = np.argsort(rows * max(n, 1) + cols, kind="stable")
    pos = np.empty_like(order)
    pos[order] = np.arange(order.shape[0], dtype=order.dtype)
    vals = np.empty((m + n, 3, 3))
    diag = a[:, None, None] * (np.eye(3)[None, :, :] + dpert)
    for r in range(3):
        for c in range(3):
            diag[:, r, c] += np.bincount(du, weights=dt * cmat[:, r, c], minlength=n)
    cmat *= -dt[:, None, None]          # the couplings become the off-diagonal blocks
    vals[pos[:m]] = cmat
    vals[pos[m:]] = diag
    trans = np.concatenate([dt, np.zeros(n)])[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return rowptr.astype(np.int32), cols[order].astype(np.int32), vals, trans


def _one(nx, ny, nz, sigma, active_frac, nnc_frac, seed, n_rhs):
    rng = np.random.Generator(np.random.PCG64(seed))
    n, u, v, cell2row = _pattern(nx, ny, nz, rng, active_frac, nnc_frac)
    k = np.exp(sigma * rng.standard_normal(n))
    a = rng.uniform(0.5, 1.5, n)
    if nnc_frac > 0.0:
        m = int(round(nnc_frac * u.shape[0]))
        lo = np.minimum(u, v)
        hi = np.maximum(u, v)
        nu, nv = _draw_nncs(rng, n, m, lo * n + hi)
        u = np.concatenate([u, nu])
        v = np.concatenate([v, nv])
    cmat = np.eye(3)[None, :, :] + 0.2 * rng.uniform(-1.0, 1.0, size=(2 * u.shape[0], 3, 3))
    dpert = 0.1 * rng.uniform(-1.0, 1.0, size=(n, 3, 3))
    rowptr, colidx, vals, trans = _assemble(n, u, v, k, a, cmat, dpert)
    b = rng.standard_normal((n_rhs, n, 3))
    return n, rowptr, colidx, vals, b, trans, cell2row


def make_grid_system(nx: int, ny: int, nz: int, *, sigma: float = 1.0,
                     active_frac: float | None = None, nnc_frac: float = 0.0,
                     seed: int = 0, n_rhs: int = 1, name: str = "") -> GridSystem:
    """One system on an ``nx x ny x nz`` grid (see the module recipe)."""
    n, rowptr, colidx, vals, b, trans, cell2row = _one(nx, ny, nz, sigma, active_frac, nnc_frac, seed, n_rhs)
    return GridSystem(n=n, rowptr=rowptr, colidx=colidx, vals=vals[None], b=b[None],
                      trans=trans, shape=(nx, ny, nz), name=name, cell_row=cell2row)


def make_ensemble(nx: int, ny: int, nz: int, seeds, *, sigma: float = 1.0,
                  n_rhs: int = 1, name: str = "") -> GridSystem:
    """Same-pattern realisations (no mask, no NNCs): one seed per member.

    Every member draws its own permeability field, couplings, accumulation
    terms and right-hand sides; the pattern depends only on the grid.
    """
    seeds = list(seeds)
    vals, bs = [], []
    first = None
    for s in seeds:
        n, rowptr, colidx, v, b, trans, cell2row = _one(nx, ny, nz, sigma, None, 0.0, s, n_rhs)
        if first is None:
            first = (n, rowptr, colidx, trans, cell2row)
        vals.append(v)
        bs.append(b)
    n, rowptr, colidx, trans, cell2row = first
    return GridSystem(n=n, rowptr=rowptr, colidx=colidx, vals=np.stack(vals), b=np.stack(bs),
                      trans=trans, shape=(nx, ny, nz), name=name, cell_row=cell2row)


# The five workload recipes: grid, permeability spread, mask, NNC fraction,
# right-hand-side count and reduction.  "c4" is a 64-member same-pattern
# ensemble; "c5" is a request mix (see ``serving_classes``).
CONFIGS = {
    "c1": dict(shape=(20, 20, 10), sigma=1.0, active_frac=None, nnc_frac=0.0, n_rhs=1, reduction=1e-2),
    "c2": dict(shape=(46, 112, 22), sigma=1.0, active_frac=0.85, nnc_frac=0.02, n_rhs=10, reduction=1e-2),
    "c3": dict(shape=(100, 100, 100), sigma=2.0, active_frac=None, nnc_frac=0.0, n_rhs=1, reduction=1e-2),
    "c4": dict(shape=(40, 40, 30), sigma=1.0, active_frac=None, nnc_frac=0.0, n_rhs=1, reduction=1e-2, batch=64),
}


def config_system(name: str, seed: int = 0, **over) -> GridSystem:
    """Build the named workload (``c1`` .. ``c4``) with an optional override of its fields."""
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    nx, ny, nz = cfg["shape"]
    if cfg.get("batch", 1) > 1:
        return make_ensemble(nx, ny, nz, range(seed, seed + cfg["batch"]), sigma=cfg["sigma"],
                             n_rhs=cfg["n_rhs"], name=name)
    return make_grid_system(nx, ny, nz, sigma=cfg["sigma"], active_frac=cfg["active_frac"],
                            nnc_frac=cfg["nnc_frac"], seed=seed, n_rhs=cfg["n_rhs"], name=name)


def serving_classes() -> dict:
    """Request size classes of the serving stream: cells -> grid shape."""
    return {10_000: (25, 20, 20), 50_000: (50, 50, 20), 200_000: (100, 100, 20), 1_000_000: (100, 100, 100)}
