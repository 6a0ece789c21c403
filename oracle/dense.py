"""Brute-force dense operators on tiny grids (reference).

Each entry ``A[i, j]`` (ghost row i, data column j) is evaluated on its own
from the definitions, in an O(#ghost x #data) double loop that does not use
the sparse assembly of ``oracle.operator``:

* Cartesian halo copy / zero padding (Sec. III-B): ``A[i, j] = 1`` exactly
  when the physical position of ghost i equals that of data cell j; ghosts
  outside the domain have no entry.
* Cubed-sphere rotated copy: ``A[i, j] = 1`` when data cell j lies at the same
  distance from a face edge as ghost i lies beyond it, on the neighbour face,
  and both project to the same point of that shared edge.
* Cubed-sphere Lagrange rows (Sec. III-B user-defined interpolation):
  ``A[i, j]`` is the Lagrange basis polynomial of node j evaluated at the
  ghost's projected angle, written as the product formula in angle space,
  when j is one of the four window nodes on the ghost's grid line.
"""
from __future__ import annotations

import math

import numpy as np

from . import cubed_sphere as cs
from .grid import Grid


def cartesian_halo(grid: Grid, nb: int, n: int) -> np.ndarray:
    """Dense A of the HPCG-shaped BC (blocks along the leading coordinate)."""
    G, D = grid.ghost_cells, grid.data_cells

    def phys(cell):
        b, c = grid.coord_of_cell(int(cell))
        bz, rem = divmod(b, nb * nb)
        by, bx = divmod(rem, nb)
        return (bz * n + c[1], by * n + c[2], bx * n + c[3])

    gpos = [phys(c) for c in G]
    dpos = [phys(c) for c in D]
    A = np.zeros((len(G), len(D)))
    for i, p in enumerate(gpos):
        for j, q in enumerate(dpos):
            if p == q:
                A[i, j] = 1.0
    return A


def _edge_point(f, j, i, N):
    """Point of the shared edge at the ghost's tangential coordinate, and layer."""
    side = cs.side_of(j, i, N)
    c, e1, e2 = cs.FRAMES[f]
    if side == cs.LEFT:
        return c - e1 + math.tan(cs.angle(N, j)) * e2, -1 - i
    if side == cs.RIGHT:
        return c + e1 + math.tan(cs.angle(N, j)) * e2, i - N
    if side == cs.BOTTOM:
        return c - e2 + math.tan(cs.angle(N, i)) * e1, -1 - j
    return c + e2 + math.tan(cs.angle(N, i)) * e1, j - N


def _data_edge_points(g, jj, ii, N):
    """For a data cell: [(edge point, distance from that edge)] for each of its face's edges."""
    c, e1, e2 = cs.FRAMES[g]
    tb = math.tan(cs.angle(N, jj))
    ta = math.tan(cs.angle(N, ii))
    return [
        (c - e1 + tb * e2, ii),
        (c + e1 + tb * e2, N - 1 - ii),
        (c - e2 + ta * e1, jj),
        (c + e2 + ta * e1, N - 1 - jj),
    ]


def cubed_sync(N: int, h: int) -> np.ndarray:
    gr = cs.grid(N, h)
    G, D = gr.ghost_cells, gr.data_cells
    dinfo = []
    for cell in D:
        _, (g, jj, ii) = gr.coord_of_cell(int(cell))
        dinfo.append((g, _data_edge_points(g, jj, ii, N)))
    A = np.zeros((len(G), len(D)))
    for r, cell in enumerate(G):
        _, (f, j, i) = gr.coord_of_cell(int(cell))
        if cs.is_corner(j, i, N):
            continue
        Q, k = _edge_point(f, j, i, N)
        for col, (g, eps) in enumerate(dinfo):
            if g == f:
                continue
            for q, dist in eps:
                if dist == k and np.abs(q - Q).max() < 1e-12:
                    A[r, col] = 1.0
    return A


def cubed_lagrange(N: int, h: int) -> np.ndarray:
    gr = cs.grid(N, h)
    G, D = gr.ghost_cells, gr.data_cells
    dcoord = [gr.coord_of_cell(int(c))[1] for c in D]
    Dang = math.pi / (2 * N)
    A = np.zeros((len(G), len(D)))
    for r, cell in enumerate(G):
        _, (f, j, i) = gr.coord_of_cell(int(cell))
        if cs.is_corner(j, i, N):
            continue
        P = cs.plane_point(f, j, i, N)
        g = int(np.argmax(cs.FRAMES[:, 0, :] @ P))
        cg, e1g, e2g = cs.FRAMES[g]
        a = math.atan(float(P @ e1g) / float(P @ cg))
        b = math.atan(float(P @ e2g) / float(P @ cg))
        # the ghost lies on the grid line of g whose centre angle matches a or b
        ka = (a + math.pi / 4) / Dang - 0.5
        kb = (b + math.pi / 4) / Dang - 0.5
        da, db = abs(ka - round(ka)), abs(kb - round(kb))
        if da <= cs.SNAP and db <= cs.SNAP:
            ra, rb = round(ka), round(kb)
            on_i = min(ra, N - 1 - ra) <= min(rb, N - 1 - rb)
        else:
            on_i = da <= db
        theta = b if on_i else a          # angle along the line
        s = (theta + math.pi / 4) / Dang - 0.5
        if abs(s - round(s)) <= cs.SNAP:
            s = float(round(s))
            theta = (s + 0.5) * Dang - math.pi / 4
        base = min(max(math.floor(s) - 1, 0), N - 4)
        nodes = [cs.angle(N, base + m) for m in range(4)]
        for col, (gg, jj, ii) in enumerate(dcoord):
            if gg != g:
                continue
            line, along = (ii, jj) if on_i else (jj, ii)
            if line != int(round(ka if on_i else kb)):
                continue
            m = along - base
            if not 0 <= m < 4:
                continue
            w = 1.0
            for n_ in range(4):
                if n_ != m:
                    w *= (theta - nodes[n_]) / (nodes[m] - nodes[n_])
            A[r, col] = w
    return A
