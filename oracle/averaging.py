"""Block-edge averaging of co-located points (reference implementation).

Sec. III-B lists block-edge averaging among the BC kinds: where points of
different blocks share one physical location, their relation is a sparse
sub-matrix ``Sync`` over those points, with 2 or 3 entries per row, and its
rows are *data* rows (the BC overwrites interior values).  Every row of one
application is computed from the input field, before any row is written.

The co-located points modelled here are those of a vertex-centred
equiangular cubed sphere with ``Np`` points per face side: point (f, j, i),
0 <= i, j < Np, lies at angles ``alpha_i = -pi/4 + i * pi / (2 (Np - 1))``
(``beta_j`` likewise) in face f's frame, so the boundary points of a face
coincide with boundary points of its neighbours (2 copies along a cube edge,
3 at a cube corner).  The sets are found by comparing 3-D positions, with no
connectivity table.  Each member of a set of k points becomes a row that
averages the k copies with weight 1/k, entries in ascending cell order
(reading: equal weights; the paper states the sparsity, not the values).
Scalar fields only: a vector field would also need the component rotation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

from .cubed_sphere import FRAMES
from .grid import Grid
from .operator import Operator, apply


@dataclass
class DataRowsSub:
    """Rows on data cells: ``entries[k]`` = [(column coord, weight)] of ``rows[k]``."""
    rows: List[tuple]
    entries: List[List[Tuple[tuple, float]]]


@dataclass
class DataOperator:
    grid: Grid
    S: sp.csr_matrix     # (ndata, ndata): row r gives the new value of data cell r
    rows: np.ndarray     # bool over data cells: rows written


def vertex_point(f: int, j: int, i: int, Np: int) -> np.ndarray:
    """Unit vector of vertex (f, j, i) of the vertex-centred cubed sphere."""
    c, e1, e2 = FRAMES[f]
    d = math.pi / (2 * (Np - 1))
    p = c + math.tan(-math.pi / 4 + i * d) * e1 + math.tan(-math.pi / 4 + j * d) * e2
    return p / np.linalg.norm(p)


def colocated_sets(Np: int, which: str = "boundary") -> List[List[tuple]]:
    """Sets of points (f, j, i) with one 3-D position, found by position.

    ``which='boundary'`` scans the face-boundary points (where copies live);
    ``'all'`` scans every point (used to count distinct positions).
    """
    key_of: Dict[tuple, List[tuple]] = {}
    for f in range(6):
        for j in range(Np):
            for i in range(Np):
                if which == "boundary" and 0 < i < Np - 1 and 0 < j < Np - 1:
                    continue
                p = vertex_point(f, j, i, Np)
                key = tuple(int(round(v * 1e9)) for v in p)
                key_of.setdefault(key, []).append((f, j, i))
    return list(key_of.values())


def edge_average_subs(Np: int) -> List[DataRowsSub]:
    """One DataRowsSub holding every row of the edge-averaging Sync matrix."""
    rows, ents = [], []
    for s in colocated_sets(Np):
        if len(s) < 2:
            continue
        members = sorted(s)
        w = 1.0 / len(members)
        cols = [(f, j, i) for (f, j, i) in members]
        for m in members:
            rows.append(m)
            ents.append([(c, w) for c in cols])
    return [DataRowsSub(rows, ents)]


def _cell(grid: Grid, fji) -> int:
    f, j, i = fji
    return grid.cell((f, j, i))


def assemble_data(grid: Grid, subs: Sequence[DataRowsSub]) -> DataOperator:
    """Evaluate the data-row sub-matrices into S over the data cells."""
    nD = grid.ndata
    I, J, V = [], [], []
    written = np.zeros(nD, dtype=bool)
    for sub in subs:
        for r, row_ents in zip(sub.rows, sub.entries):
            rc = grid.cell(tuple(r))
            if not grid.is_data_coord(tuple(r)):
                raise ValueError(f"row {r} is not a data cell")
            ri = int(grid.cell2col[rc])
            if written[ri]:
                raise ValueError(f"data row {r} given twice")
            written[ri] = True
            for col, w in row_ents:
                if not grid.is_data_coord(tuple(col)):
                    raise ValueError(f"column {col} is not a data cell")
                I.append(ri)
                J.append(int(grid.cell2col[grid.cell(tuple(col))]))
                V.append(float(w))
    S = sp.coo_matrix((V, (I, J)), shape=(nD, nD)).tocsr()
    return DataOperator(grid, S, written)


def apply_with_data_rows(op: Operator, dop: DataOperator, u: np.ndarray, vec=None) -> np.ndarray:
    """Ghost rows (A x + b) and data rows (S x), all from the input field."""
    g = op.grid
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 1:
        u = u[:, None]
    out = apply(op, u, vec)
    X = u[g.data_cells]
    Z = dop.S @ X
    cells = g.data_cells[dop.rows]
    out[cells] = Z[dop.rows]
    return out
