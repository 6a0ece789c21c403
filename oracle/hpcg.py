"""HPCG-shaped Cartesian case: halo-1 BC on 2x2x2 blocks + 27-point operator (reference).

Sec. III-B: halo copying (a ghost that is another block's data copies it) and
padding with zeros (a ghost outside the domain is 0).  Sec. IV-C: the BC
writes exist only to feed the inner operator that follows.  The inner operator
here is the 27-point stencil with diagonal 26 and off-diagonals -1.

Two independent paths are provided:

* ``ghosted_blocks`` + ``stencil27``: split the domain into blocks with a
  halo of one cell, fill the halos from the global positions, apply the
  stencil per block;
* ``stencil27_padded``: ``numpy.pad`` of the unsplit domain with zeros
  followed by the same 27 shifted views.

``grid`` / ``subs`` express the same BC as basic sub-matrices (block id as
the leading coordinate, one sub-matrix per block and neighbour direction).
"""
from __future__ import annotations

import itertools
from typing import List

import numpy as np

from .grid import Grid
from .operator import MapSub, ZeroSub

OFFSETS = [d for d in itertools.product((-1, 0, 1), repeat=3) if d != (0, 0, 0)]


def block_index(nb: int, bz: int, by: int, bx: int) -> int:
    return (bz * nb + by) * nb + bx


def ghosted_blocks(x: np.ndarray, nb: int = 2) -> List[np.ndarray]:
    """Blocks of ``x`` (n^3 each) with a one-cell halo filled from the global array."""
    Nd = x.shape[0]
    n = Nd // nb
    xp = np.pad(x, 1)  # zero outside the domain
    out = []
    for bz, by, bx in itertools.product(range(nb), repeat=3):
        out.append(xp[bz * n: bz * n + n + 2, by * n: by * n + n + 2, bx * n: bx * n + n + 2].copy())
    return out


def stencil27(xg: np.ndarray) -> np.ndarray:
    """y = 26 x_c - sum of the 26 neighbours, on the interior of a ghosted array."""
    n0, n1, n2 = (s - 2 for s in xg.shape)
    y = 26.0 * xg[1:1 + n0, 1:1 + n1, 1:1 + n2]
    for dz, dy, dx in OFFSETS:
        y = y - xg[1 + dz:1 + dz + n0, 1 + dy:1 + dy + n1, 1 + dx:1 + dx + n2]
    return y


def stencil27_padded(x: np.ndarray) -> np.ndarray:
    return stencil27(np.pad(x, 1))


def abs_row_sum(xg: np.ndarray) -> np.ndarray:
    """Per output point, sum over the stencil of |a_ij x_j| (for rounding bounds)."""
    a = np.abs(xg)
    n0, n1, n2 = (s - 2 for s in xg.shape)
    acc = 26.0 * a[1:1 + n0, 1:1 + n1, 1:1 + n2]
    for dz, dy, dx in OFFSETS:
        acc = acc + a[1 + dz:1 + dz + n0, 1 + dy:1 + dy + n1, 1 + dx:1 + dx + n2]
    return acc


def grid(nb: int, n: int) -> Grid:
    """nb^3 blocks of n^3 data cells, halo 1, along a leading block coordinate."""
    nblk = nb ** 3
    g = Grid([0, -1, -1, -1], [nblk, n + 1, n + 1, n + 1])
    for b in range(nblk):
        g.add_block([(b, b + 1)] + [(-1, n + 1)] * 3, [(b, b + 1)] + [(0, n)] * 3)
    return g


def subs(nb: int, n: int) -> List:
    """One sub-matrix per block and neighbour direction: copy or zero."""
    out = []
    for bz, by, bx in itertools.product(range(nb), repeat=3):
        b = block_index(nb, bz, by, bx)
        for d in OFFSETS:
            box = [(b, b + 1)]
            for dd in d:
                box.append({-1: (-1, 0), 0: (0, n), 1: (n, n + 1)}[dd])
            nbr = (bz + d[0], by + d[1], bx + d[2])
            if all(0 <= v < nb for v in nbr):
                src = block_index(nb, *nbr)

                def fmap(c, src=src, d=d):
                    # ghost at local position p of block b = data at p - d*n of the neighbour
                    return (src, c[1] - d[0] * n, c[2] - d[1] * n, c[3] - d[2] * n)

                out.append(MapSub(box, fmap))
            else:
                out.append(ZeroSub(box))
    return out
