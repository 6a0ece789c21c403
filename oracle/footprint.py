"""Consumer footprint: ghost rows no later read depends on (reference).

Sec. IV-C unions, for every boundary write, the reads of the following
(inner) computation that depend on it, and drops the writes outside that
union.  With the consuming operator given by its read offsets around each
data cell, a ghost cell is live exactly when some data cell of its block plus
some offset lands on it.  Evaluated here by brute force over the data cells.
"""
from __future__ import annotations

from dataclasses import replace
from typing import Sequence

import numpy as np

from .grid import Grid, box_coords, box_contains
from .operator import Operator


def live_ghost_mask(grid: Grid, offsets: Sequence[Sequence[int]]) -> np.ndarray:
    """Bool over ghost rows (grid.ghost_cells order): reached by a consumer read."""
    live = np.zeros(grid.nghost, dtype=bool)
    ghost_row = -np.ones(grid.ncells, dtype=np.int64)
    ghost_row[grid.ghost_cells] = np.arange(grid.nghost)
    for blk in grid.blocks:
        for d in box_coords(blk.data):
            for o in offsets:
                c = tuple(int(a) + int(b) for a, b in zip(d, o))
                if not box_contains(blk.full, c) or box_contains(blk.data, c):
                    continue
                live[ghost_row[grid.cell(c)]] = True
    return live


def restrict(op: Operator, live: np.ndarray) -> Operator:
    """The operator with every row outside ``live`` dropped (left unwritten)."""
    part_rows = {k: m & live for k, m in op.part_rows.items()}
    return replace(op, part_rows=part_rows, has_b=op.has_b & live, covered=op.covered & live)
