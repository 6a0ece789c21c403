"""Pins of the reference's stepped slices (Sec. IV-A-1: step 2 for staggered
variables, step 2^k for multigrid levels).

A slice (start, stop, step) holds the points start + k*step < stop.  The
checks use closed forms (point counts, mirror and periodic images of a known
field, exact interpolation of a linear field) and the invariance of the
operator under relabelling the points by their index k.
"""
import math

import numpy as np
import pytest

from oracle import MapSub, RowsSub, ZeroSub, apply, assemble
from oracle.grid import Grid


def npts(a, b, s):
    return math.ceil((b - a) / s)


@pytest.mark.parametrize("full,data", [([(-1, 10, 2), (-3, 14, 4)], [(1, 8, 2), (1, 10, 4)]),
                                       ([(0, 7, 3), (2, 3, 1)], [(3, 6, 3), (2, 3, 1)])])
def test_point_counts(full, data):
    g = Grid([f[0] for f in full], [f[1] for f in full])
    g.add_block(full, data)
    nf = int(np.prod([npts(*f) for f in full]))
    nd = int(np.prod([npts(*d) for d in data]))
    assert g.ncells == nf and g.ndata == nd and g.nghost == nf - nd
    # every data cell is a point of the data slices
    for c in g.data_cells:
        _, coord = g.coord_of_cell(int(c))
        for (a, b, s), x in zip(data, coord):
            assert a <= x < b and (x - a) % s == 0


def staggered_1d(n):
    """Cell-centred variable on [0, 2n): points 1, 3, ..., 2n-1, one ghost each side."""
    g = Grid([-1], [2 * n + 2])
    g.add_block([(-1, 2 * n + 2, 2)], [(1, 2 * n, 2)])
    return g


def field_of(g, fn):
    u = np.full((g.ncells, 1), np.nan)
    for c in g.data_cells:
        _, (x,) = g.coord_of_cell(int(c))
        u[c, 0] = fn(x)
    return u


def test_staggered_mirror_closed_form():
    n = 5
    g = staggered_1d(n)
    # mirror about the faces x = 0 and x = 2n: ghost -1 takes point 1, ghost 2n+1 takes 2n-1
    subs = [MapSub([(-1, 0)], lambda c: (-c[0],)), MapSub([(2 * n, 2 * n + 2)], lambda c: (4 * n - c[0],))]
    out = apply(assemble(g, subs), field_of(g, lambda x: x * x + 3.0))
    assert out[g.cell((-1,)), 0] == 1.0 + 3.0
    assert out[g.cell((2 * n + 1,)), 0] == (2 * n - 1) ** 2 + 3.0
    # positions between the points hold no cells: the row box [2n, 2n+2) holds one row
    assert g.owner((2 * n,)) == -1 and g.nghost == 2


def test_multigrid_level_periodic():
    # level with step 4 over [0, 32) plus one ghost point on each side
    g = Grid([-4], [36])
    g.add_block([(-4, 36, 4)], [(0, 32, 4)])
    subs = [MapSub([(-4, 0)], lambda c: (c[0] + 32,)), MapSub([(32, 36)], lambda c: (c[0] - 32,))]
    out = apply(assemble(g, subs), field_of(g, lambda x: 10.0 + x))
    assert out[g.cell((-4,)), 0] == 10.0 + 28 and out[g.cell((32,)), 0] == 10.0 + 0


def test_linear_interpolation_on_staggered_points_is_exact():
    n = 6
    g = staggered_1d(n)
    # ghost at -1 extrapolated linearly from points 1 and 3: u(-1) = 2 u(1) - u(3)
    subs = [RowsSub([(-1, 0)], lambda c: [((1,), 2.0), ((3,), -1.0)]), ZeroSub([(2 * n, 2 * n + 2)])]
    out = apply(assemble(g, subs), field_of(g, lambda x: 0.5 * x - 2.0))
    assert out[g.cell((-1,)), 0] == 0.5 * -1 - 2.0
    assert out[g.cell((2 * n + 1,)), 0] == 0.0


def test_relabelling_by_index_gives_the_same_operator():
    # 2-D grid, step 2 along x (staggered), step 1 along y; the same BC on the
    # compact grid (positions replaced by their index) gives the same matrix
    nx, ny = 5, 4
    gs = Grid([-2, -1], [2 * nx + 2, ny + 1])
    gs.add_block([(-2, 2 * nx + 2, 2), (-1, ny + 1, 1)], [(0, 2 * nx, 2), (0, ny, 1)])
    gc = Grid([-1, -1], [nx + 1, ny + 1])
    gc.add_block([(-1, nx + 1), (-1, ny + 1)], [(0, nx), (0, ny)])
    assert gs.ncells == gc.ncells and np.array_equal(gs.data_cells, gc.data_cells)
    subs_s = [MapSub([(-2, 0), (0, ny)], lambda c: (c[0] + 2 * nx, c[1])),
              MapSub([(2 * nx, 2 * nx + 2), (0, ny)], lambda c: (c[0] - 2 * nx, c[1])),
              RowsSub([(0, 2 * nx), (-1, 0)], lambda c: [((c[0], 0), 0.75), ((c[0], 1), 0.25)]),
              ZeroSub([(0, 2 * nx), (ny, ny + 1)])]
    subs_c = [MapSub([(-1, 0), (0, ny)], lambda c: (c[0] + nx, c[1])),
              MapSub([(nx, nx + 1), (0, ny)], lambda c: (c[0] - nx, c[1])),
              RowsSub([(0, nx), (-1, 0)], lambda c: [((c[0], 0), 0.75), ((c[0], 1), 0.25)]),
              ZeroSub([(0, nx), (ny, ny + 1)])]
    A_s, A_c = assemble(gs, subs_s).dense(), assemble(gc, subs_c).dense()
    assert np.array_equal(A_s, A_c)
