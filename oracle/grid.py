"""Region model of a block-structured grid (reference implementation).

Follows Sec. III-A (full region = data region + ghost region) and Sec. IV-A-1
(each block's full and data regions are slices of one global box; the ghost
region is full minus data).  As in Alg. 1, the block id is the leading
coordinate of the global box, so blocks never overlap in global coordinates.
A slice (start, stop, step) selects the points start + k * step < stop of its
dimension (Sec. IV-A-1: step 2 for staggered variables, 2^k for multigrid
levels); a block's cells are the points of its full slices, its data cells
those that are also points of its data slices, its ghost cells the rest.

Storage convention shared with the tests: cells are numbered block by block
(in the order blocks were added), each block's full-slice points in row-major
order (last coordinate fastest).  Inner values (levels x fields x components) form a
separate trailing axis, so the reference is layout-agnostic.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

Box = List[Tuple[int, int]]  # [(start, stop)] per dimension, half-open


def box_shape(box: Sequence[Tuple[int, int]]) -> Tuple[int, ...]:
    return tuple(int(b) - int(a) for a, b in box)


def box_contains(box, coord) -> bool:
    return all(a <= c < b for (a, b), c in zip(box, coord))


def box_coords(box):
    """All multi-indices of ``box`` in row-major order, as an (n, ndim) array."""
    shape = box_shape(box)
    if any(s <= 0 for s in shape):
        return np.zeros((0, len(box)), dtype=np.int64)
    grids = np.meshgrid(*[np.arange(a, b) for a, b in box], indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1).astype(np.int64)


@dataclass
class Block:
    full: Box
    data: Box
    fstep: Tuple[int, ...] = ()
    dstep: Tuple[int, ...] = ()

    def npoints(self, d: int) -> int:
        a, b = self.full[d]
        return max(0, -(-(b - a) // self.fstep[d]))

    def has_cell(self, coord) -> bool:
        return all(a <= c < b and (c - a) % st == 0 for (a, b), st, c in zip(self.full, self.fstep, coord))

    def has_data(self, coord) -> bool:
        return all(a <= c < b and (c - a) % st == 0 for (a, b), st, c in zip(self.data, self.dstep, coord))


class Grid:
    def __init__(self, lo: Sequence[int], hi: Sequence[int]):
        self.lo = [int(v) for v in lo]
        self.hi = [int(v) for v in hi]
        self.ndim = len(self.lo)
        self.blocks: List[Block] = []

    def add_block(self, full, data) -> int:
        """full / data: per dimension (start, stop) or (start, stop, step)."""
        fstep = tuple(int(s[2]) if len(s) > 2 else 1 for s in full)
        dstep = tuple(int(s[2]) if len(s) > 2 else 1 for s in data)
        full = [(int(s[0]), int(s[1])) for s in full]
        data = [(int(s[0]), int(s[1])) for s in data]
        assert len(full) == self.ndim and len(data) == self.ndim
        assert min(fstep + dstep) >= 1
        for (fa, fb), (da, db), lo, hi in zip(full, data, self.lo, self.hi):
            assert lo <= fa <= da < db <= fb <= hi, "data must lie inside full, full inside the global box"
        for blk in self.blocks:
            assert not all(max(a0, b0) < min(a1, b1) for (a0, a1), (b0, b1) in zip(blk.full, full)), \
                "block full regions must not overlap"
        self.blocks.append(Block(full, data, fstep, dstep))
        self._index = None
        return len(self.blocks) - 1

    def points(self, box) -> np.ndarray:
        """Cells of the grid inside a box of positions, row-major, as (n, ndim)
        coordinates.  Positions between the points of a stepped slice are
        skipped; a position outside every block's full range is an error."""
        coords = box_coords(box)
        if all(st == 1 for blk in self.blocks for st in blk.fstep):
            return coords
        keep = []
        for i, c in enumerate(coords):
            c = tuple(int(v) for v in c)
            if self.owner(c) >= 0:
                keep.append(i)
            elif not any(box_contains(blk.full, c) for blk in self.blocks):
                raise ValueError(f"position {c} lies outside every block")
        return coords[keep] if keep else np.zeros((0, self.ndim), dtype=np.int64)

    # ---- cell numbering ------------------------------------------------------
    def _build(self):
        bases, shapes = [], []
        n = 0
        for blk in self.blocks:
            shp = tuple(blk.npoints(d) for d in range(self.ndim))
            bases.append(n)
            shapes.append(shp)
            n += int(np.prod(shp))
        self._bases = bases
        self._shapes = shapes
        self._ncells = n
        is_data = np.zeros(n, dtype=bool)
        for b, blk in enumerate(self.blocks):
            pts = [blk.full[d][0] + blk.fstep[d] * np.arange(self._shapes[b][d]) for d in range(self.ndim)]
            m = np.ones(self._shapes[b], dtype=bool)
            for d in range(self.ndim):
                da, db = blk.data[d]
                ok = (pts[d] >= da) & (pts[d] < db) & ((pts[d] - da) % blk.dstep[d] == 0)
                shape = [1] * self.ndim
                shape[d] = -1
                m &= ok.reshape(shape)
            is_data[bases[b]: bases[b] + m.size] = m.reshape(-1)
        self._is_data = is_data
        self._data_cells = np.nonzero(is_data)[0]
        self._ghost_cells = np.nonzero(~is_data)[0]
        self._cell2col = np.full(n, -1, dtype=np.int64)
        self._cell2col[self._data_cells] = np.arange(self._data_cells.size)
        self._cell2row = np.full(n, -1, dtype=np.int64)
        self._cell2row[self._ghost_cells] = np.arange(self._ghost_cells.size)
        self._index = True

    def _ensure(self):
        if self._index is None:
            self._build()

    @property
    def is_data(self) -> np.ndarray:
        self._ensure()
        return self._is_data

    @property
    def data_cells(self) -> np.ndarray:
        """Cell numbers of all data cells, ascending (column order of A)."""
        self._ensure()
        return self._data_cells

    @property
    def ghost_cells(self) -> np.ndarray:
        """Cell numbers of all ghost cells, ascending (row order of A)."""
        self._ensure()
        return self._ghost_cells

    @property
    def cell2col(self) -> np.ndarray:
        self._ensure()
        return self._cell2col

    @property
    def cell2row(self) -> np.ndarray:
        self._ensure()
        return self._cell2row

    @property
    def ncells(self) -> int:
        self._ensure()
        return self._ncells

    @property
    def nghost(self) -> int:
        return int(self.ghost_cells.size)

    @property
    def ndata(self) -> int:
        return int(self.data_cells.size)

    def block_base(self, b: int) -> int:
        self._ensure()
        return self._bases[b]

    def block_shape(self, b: int):
        self._ensure()
        return self._shapes[b]

    def owner(self, coord) -> int:
        """Block one of whose cells is ``coord``, or -1."""
        for b, blk in enumerate(self.blocks):
            if blk.has_cell(coord):
                return b
        return -1

    def cell(self, coord) -> int:
        """Cell number of a global multi-index (must be a cell of some block)."""
        self._ensure()
        b = self.owner(coord)
        if b < 0:
            raise IndexError(f"coordinate {tuple(coord)} is not a cell of any block")
        blk = self.blocks[b]
        off = 0
        for d, c in enumerate(coord):
            off = off * blk.npoints(d) + (c - blk.full[d][0]) // blk.fstep[d]
        return self._bases[b] + off

    def cells_of_box(self, b: int, box) -> np.ndarray:
        """Cell numbers of block ``b``'s cells inside a box of positions, row-major."""
        self._ensure()
        blk = self.blocks[b]
        coords = np.array([c for c in box_coords(box) if blk.has_cell(tuple(c))], dtype=np.int64)
        coords = coords.reshape(-1, self.ndim)
        off = np.zeros(coords.shape[0], dtype=np.int64)
        for d in range(self.ndim):
            off = off * blk.npoints(d) + (coords[:, d] - blk.full[d][0]) // blk.fstep[d]
        return self._bases[b] + off

    def is_data_coord(self, coord) -> bool:
        b = self.owner(coord)
        return b >= 0 and self.blocks[b].has_data(coord)

    def coord_of_cell(self, cell: int):
        self._ensure()
        b = int(np.searchsorted(self._bases, cell, side="right") - 1)
        blk = self.blocks[b]
        off = cell - self._bases[b]
        out = []
        for d in reversed(range(self.ndim)):
            n = blk.npoints(d)
            out.append(blk.full[d][0] + blk.fstep[d] * (off % n))
            off //= n
        return b, tuple(reversed(out))
