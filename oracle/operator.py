"""Assembly and application of the affine BC operator (reference implementation).

Sec. III-B writes every boundary condition as ``F(x) = A x + b`` where ``x``
covers the data region and the rows of ``A`` / ``b`` are the full region of
the output.  Only ghost rows are produced here (the six kinds listed in
Sec. III-B all write ghost rows except block-edge averaging, which is not
modelled).  Sec. IV-A-3 and Tables II/III split ``A`` into basic
sub-matrices, each valid on a set of rows and giving a row iterator:

* ``MapSub``    a static list with one entry (column = fmap(row), weight):
                halo copy, circular / symmetric maps, rotated copies.
* ``ZeroSub``   a static empty list: padding with zeros.
* ``RowsSub``   a dynamic row iterator (nnz, then column and value of each
                entry): CSR / ELL user-defined interpolation.
* ``VectorSub`` a basic sub-vector: the ``b`` values of its rows.

A sub-matrix may carry a 2x2 signed permutation ``rot`` acting on the two
components of a vector field stored in the inner slots (Sec. V-A stores
multi-component vectors per grid point); scalar slots ignore it.

Overlapping sub-matrix rows are rejected unless ``allow_overlap_sum`` is set,
in which case their contributions add (the paper gives no priority rule for
overlapping valid sets).  Rows covered by no sub-matrix and no sub-vector are
left unchanged by ``apply``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

from .grid import Grid, box_contains, box_coords


@dataclass
class MapSub:
    rows: list
    fmap: Callable[[tuple], tuple]
    weight: float = 1.0
    rot: Optional[tuple] = None


@dataclass
class ZeroSub:
    rows: list


@dataclass
class RowsSub:
    rows: list
    entries: Callable[[tuple], List[Tuple[tuple, float]]]
    rot: Optional[tuple] = None


@dataclass
class VectorSub:
    rows: list
    values: np.ndarray  # (rows in box order,) or (rows, ninner)


def _rot_key(rot):
    if rot is None:
        return None
    r = np.asarray(rot, dtype=np.int64).reshape(2, 2)
    ok = (np.abs(r).sum(axis=0) == 1).all() and (np.abs(r).sum(axis=1) == 1).all()
    if not ok:
        raise ValueError("component rotation must be a signed permutation")
    return tuple(int(v) for v in r.reshape(-1))


@dataclass
class Operator:
    grid: Grid
    parts: Dict[Optional[tuple], sp.csr_matrix]   # rot key -> A restricted to rows of subs with that rot
    part_rows: Dict[Optional[tuple], np.ndarray]  # rot key -> bool mask over ghost rows
    b: Optional[np.ndarray]                       # (nghost, nb) or None
    has_b: np.ndarray                             # bool over ghost rows
    covered: np.ndarray                           # bool over ghost rows

    def dense(self) -> np.ndarray:
        """Sum of all parts as a dense (nghost, ndata) matrix (ignores rot)."""
        out = np.zeros((self.grid.nghost, self.grid.ndata))
        for A in self.parts.values():
            out += A.toarray()
        return out


def _ghost_row(grid: Grid, coord, block: int) -> int:
    blk = grid.blocks[block]
    if not blk.has_cell(coord):
        raise ValueError(f"row {coord} leaves block {block}")
    if blk.has_data(coord):
        raise ValueError(f"row {coord} is a data cell; only ghost rows are written")
    return int(grid.cell2row[grid.cell(coord)])


def _data_col(grid: Grid, coord) -> int:
    if not grid.is_data_coord(coord):
        raise ValueError(f"column {tuple(coord)} is not a data cell")
    return int(grid.cell2col[grid.cell(coord)])


def assemble(grid: Grid, subs: Sequence, allow_overlap_sum: bool = False) -> Operator:
    """Evaluate every row of every sub-matrix / sub-vector into (A, b)."""
    nG, nD = grid.nghost, grid.ndata
    coo: Dict[Optional[tuple], Tuple[list, list, list]] = {}
    part_rows: Dict[Optional[tuple], np.ndarray] = {}
    mat_count = np.zeros(nG, dtype=np.int64)
    vec_count = np.zeros(nG, dtype=np.int64)
    b = None
    for sub in subs:
        coords = grid.points(sub.rows)  # the grid's cells in the box (every point for step-1 slices)
        if coords.shape[0] == 0:
            continue
        block = grid.owner(tuple(coords[0]))
        if block < 0:
            raise ValueError("sub-matrix rows outside every block")
        rows = np.array([_ghost_row(grid, tuple(c), block) for c in coords], dtype=np.int64)
        if isinstance(sub, VectorSub):
            vals = np.asarray(sub.values, dtype=np.float64)
            if vals.ndim == 1:
                vals = vals[:, None]
            if vals.shape[0] != rows.size:
                raise ValueError("sub-vector values do not match its rows")
            if b is None:
                b = np.zeros((nG, vals.shape[1]))
            elif b.shape[1] != vals.shape[1]:
                raise ValueError("all sub-vectors need the same inner width")
            b[rows] += vals
            vec_count[rows] += 1
            continue
        key = _rot_key(getattr(sub, "rot", None))
        I, J, V = coo.setdefault(key, ([], [], []))
        mask = part_rows.setdefault(key, np.zeros(nG, dtype=bool))
        mask[rows] = True
        mat_count[rows] += 1
        for c, r in zip(coords, rows):
            c = tuple(int(v) for v in c)
            if isinstance(sub, ZeroSub):
                continue
            if isinstance(sub, MapSub):
                ents = [(sub.fmap(c), sub.weight)]
            elif isinstance(sub, RowsSub):
                ents = sub.entries(c)
            else:
                raise TypeError(type(sub))
            for col, w in ents:
                I.append(int(r))
                J.append(_data_col(grid, tuple(int(v) for v in col)))
                V.append(float(w))
    if not allow_overlap_sum and ((mat_count > 1).any() or (vec_count > 1).any()):
        raise ValueError("overlapping sub-matrix rows (enable allow_overlap_sum to add them)")
    parts = {}
    for key, (I, J, V) in coo.items():
        # duplicates are summed by the COO -> CSR conversion
        parts[key] = sp.coo_matrix((V, (I, J)), shape=(nG, nD)).tocsr()
    covered = (mat_count > 0) | (vec_count > 0)
    return Operator(grid, parts, part_rows, b, vec_count > 0, covered)


def _vec_slots(I: int, vec):
    if vec is None:
        return None
    lo, stride, length = vec
    u = np.arange(lo, lo + length)
    v = u + stride
    assert v[-1] < I if length else True
    return u, v


def _rotate(Z: np.ndarray, key, slots) -> np.ndarray:
    """Apply the signed permutation ``key`` to the vector slots of Z (exact)."""
    if key is None or slots is None:
        return Z
    r = np.array(key).reshape(2, 2)
    u, v = slots
    out = Z.copy()
    comps = (Z[:, u], Z[:, v])
    for a, dst in enumerate((u, v)):
        src = 0 if r[a, 0] != 0 else 1
        out[:, dst] = float(r[a, src]) * comps[src]
    return out


def apply(op: Operator, u: np.ndarray, vec=None) -> np.ndarray:
    """Return a copy of the full field ``u`` (ncells, I) with covered ghosts := A x + b."""
    g = op.grid
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 1:
        u = u[:, None]
    X = u[g.data_cells]
    slots = _vec_slots(u.shape[1], vec)
    Y = np.full((g.nghost, u.shape[1]), -0.0)
    for key, A in op.parts.items():
        Z = _rotate(A @ X, key, slots)
        m = op.part_rows[key]
        Y[m] += Z[m]
    if op.b is not None:
        if op.b.shape[1] not in (1, u.shape[1]):
            raise ValueError("sub-vector inner width must be 1 or the field's inner extent")
        Y[op.has_b] += op.b[op.has_b]
    out = u.copy()
    rows = g.ghost_cells[op.covered]
    out[rows] = Y[op.covered]
    return out


def _rotate_T(G: np.ndarray, key, slots) -> np.ndarray:
    if key is None or slots is None:
        return G
    r = np.array(key).reshape(2, 2).T
    return _rotate(G, tuple(int(v) for v in r.reshape(-1)), slots)


def vjp(op: Operator, ybar: np.ndarray, vec=None) -> np.ndarray:
    """Vector-Jacobian product of ``apply`` with respect to the full field.

    The forward keeps data cells, replaces covered ghosts by A x + b and keeps
    uncovered ghosts, so  ubar_D = ybar_D + A^T ybar_G(covered),
    ubar_G(covered) = 0,  ubar_G(uncovered) = ybar_G(uncovered).
    """
    g = op.grid
    ybar = np.asarray(ybar, dtype=np.float64)
    if ybar.ndim == 1:
        ybar = ybar[:, None]
    slots = _vec_slots(ybar.shape[1], vec)
    G = ybar[g.ghost_cells].copy()
    G[~op.covered] = 0.0
    out = ybar.copy()
    acc = np.zeros((g.ndata, ybar.shape[1]))
    for key, A in op.parts.items():
        Gm = np.where(op.part_rows[key][:, None], G, 0.0)
        acc += A.T @ _rotate_T(Gm, key, slots)
    out[g.data_cells] += acc
    out[g.ghost_cells[op.covered]] = 0.0
    return out
