"""The operator that reads the BC's ghosts, evaluated after the BC (reference).

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. IV-C: the boundary writes exist to feed the inner computation that
follows them, and the two are expressed together so that they can be
optimised together.  The following computation here is a stencil of offsets
and weights over each block's data cells, applied to the field the BC has
just written:

    y[c, l] = sum_o w_o u'[c + o, l],   u' = apply(op, u)

for every data cell c of every block (blocks in order, each block's data box
in row-major order), each read inside the cell's block's full region.  It is
computed literally: the BC first, then the weighted sum of shifted views.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .grid import box_contains
from .operator import Operator, apply


def stencil_after_bc(op: Operator, u: np.ndarray, offsets: Sequence[Sequence[int]], weights: Sequence[float],
                     vec=None) -> np.ndarray:
    """(data cells, I) array of the stencil applied to apply(op, u, vec)."""
    g = op.grid
    up = apply(op, u, vec)
    out = []
    for b, blk in enumerate(g.blocks):
        dcells = g.cells_of_box(b, blk.data)
        acc = np.zeros((len(dcells), up.shape[1]))
        for o, w in zip(offsets, weights):
            box = [(a + s, c + s) for (a, c), s in zip(blk.data, o)]
            if not (box_contains(blk.full, [a for a, _ in box]) and box_contains(blk.full, [c - 1 for _, c in box])):
                raise ValueError(f"offset {tuple(o)} reads outside block {b}'s full region")
            acc = acc + w * up[g.cells_of_box(b, box)]
        out.append(acc)
    return np.concatenate(out)
