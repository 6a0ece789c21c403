"""Equiangular gnomonic cubed sphere: ghost rows from 3-D geometry (reference).

Sec. II-B describes the cubed-sphere ghost computation: the position of a
ghost cell is translated into the coordinates of the neighbouring panel and
interpolated there from that panel's data; Sec. III-B then treats the result
as a user-defined interpolation sub-matrix ``Itp`` of shape (#ghost, #data).
Sec. III-B also gives halo copying, and Alg. 1 a copy whose axes are rotated
between blocks.  Sec. V-A adds multi-component vectors per grid point.

The paper fixes neither the cube orientation nor the interpolation scheme, so
the choices below are readings (documented with the design):

* Six faces with frames (centre c, tangents e1, e2), each right-handed.
  Face f, index (j, i): i runs along e1 (angle alpha), j along e2 (beta),
  centre angles ``-pi/4 + (k + 1/2) * D`` with ``D = pi / (2N)``.
* An edge ghost (exactly one of i, j outside [0, N)) is the point
  ``P = c + tan(alpha_i) e1 + tan(beta_j) e2`` on f's extended plane.  Its
  neighbour is the face g maximising ``P . c_g``.  Seen from g,
  ``a = atan(P.e1_g / P.c_g)`` and ``b = atan(P.e2_g / P.c_g)`` give
  fractional indices ``(a + pi/4) / D - 1/2``; one of them is an integer
  (the grid line of g through the ghost), the other is ``s``.
* Lagrange rows: 4-point Lagrange interpolation in index space along that
  line, nodes ``base .. base + 3``, ``base = clamp(floor(s) - 1, 0, N - 4)``,
  after snapping ``s`` to an integer when within 1e-9.
* Sync (halo-copy) rows: the ghost at layer k and tangential index t copies the
  cell of g on the same line whose tangential index is that of the point of
  the shared edge at f's tangential coordinate t.
* Corner ghosts (both i and j outside) are zero rows.
* Vector components: a 2x2 signed permutation per face side, from the
  tangent directions of both faces at the midpoint of the shared edge,
  computed by finite differences of the 3-D maps.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from .grid import Grid
from .operator import MapSub, RowsSub, ZeroSub

FRAMES = np.array(
    [
        [[1, 0, 0], [0, 1, 0], [0, 0, 1]],
        [[0, 1, 0], [-1, 0, 0], [0, 0, 1]],
        [[-1, 0, 0], [0, -1, 0], [0, 0, 1]],
        [[0, -1, 0], [1, 0, 0], [0, 0, 1]],
        [[0, 0, 1], [0, 1, 0], [-1, 0, 0]],
        [[0, 0, -1], [0, 1, 0], [1, 0, 0]],
    ],
    dtype=np.float64,
)

LEFT, RIGHT, BOTTOM, TOP = 0, 1, 2, 3
SNAP = 1e-9


def angle(N: int, k: float) -> float:
    return -math.pi / 4 + (k + 0.5) * (math.pi / (2 * N))


def plane_point(f: int, j: float, i: float, N: int) -> np.ndarray:
    c, e1, e2 = FRAMES[f]
    return c + math.tan(angle(N, i)) * e1 + math.tan(angle(N, j)) * e2


def frac_index(P: np.ndarray, g: int, N: int) -> Tuple[float, float]:
    """(s_j, s_i): fractional (beta, alpha) indices of the ray through P on face g."""
    c, e1, e2 = FRAMES[g]
    pc = float(P @ c)
    a = math.atan(float(P @ e1) / pc)
    b = math.atan(float(P @ e2) / pc)
    D = math.pi / (2 * N)
    return (b + math.pi / 4) / D - 0.5, (a + math.pi / 4) / D - 0.5


def side_of(j: int, i: int, N: int) -> int:
    if i < 0:
        return LEFT
    if i >= N:
        return RIGHT
    if j < 0:
        return BOTTOM
    return TOP


def is_corner(j: int, i: int, N: int) -> bool:
    return not (0 <= i < N) and not (0 <= j < N)


def neighbour_line(f: int, j: int, i: int, N: int):
    """For an edge ghost: (g, axis, L, s).

    ``axis == 'i'`` means the line is i = L on face g (nodes vary in j);
    ``axis == 'j'`` means j = L (nodes vary in i).  ``s`` is the fractional
    index along the line.
    """
    P = plane_point(f, j, i, N)
    dots = FRAMES[:, 0, :] @ P
    g = int(np.argmax(dots))
    assert g != f
    sj, si = frac_index(P, g, N)
    di, dj = abs(si - round(si)), abs(sj - round(sj))
    if di <= SNAP and dj <= SNAP:
        # both indices integral (the middle line of an odd-sized face): the grid
        # line is the one nearer to a face edge, i.e. across from the ghost
        ri, rj = int(round(si)), int(round(sj))
        use_i = min(ri, N - 1 - ri) <= min(rj, N - 1 - rj)
    else:
        use_i = di <= dj
    if use_i:
        return g, "i", int(round(si)), sj
    return g, "j", int(round(sj)), si


def lagrange_weights(s: float, N: int):
    """Stencil base and the 4 Lagrange weights for fractional index s."""
    if abs(s - round(s)) <= SNAP:
        s = float(round(s))
    base = min(max(math.floor(s) - 1, 0), N - 4)
    d = [s - (base + n) for n in range(4)]
    w = [
        -d[1] * d[2] * d[3] / 6.0,
        d[0] * d[2] * d[3] / 2.0,
        -d[0] * d[1] * d[3] / 2.0,
        d[0] * d[1] * d[2] / 6.0,
    ]
    return base, w, s


def _node(g: int, axis: str, L: int, k: int):
    return (g, k, L) if axis == "i" else (g, L, k)


def lagrange_entries(f: int, j: int, i: int, N: int):
    """Row of the user-defined interpolation sub-matrix for edge ghost (f, j, i)."""
    g, axis, L, s = neighbour_line(f, j, i, N)
    base, w, _ = lagrange_weights(s, N)
    return [(_node(g, axis, L, base + m), w[m]) for m in range(4)]


def sync_source(f: int, j: int, i: int, N: int):
    """Source cell of the rotated halo copy for edge ghost (f, j, i)."""
    g, axis, L, _ = neighbour_line(f, j, i, N)
    side = side_of(j, i, N)
    c, e1, e2 = FRAMES[f]
    if side in (LEFT, RIGHT):
        n = -e1 if side == LEFT else e1
        Q = c + n + math.tan(angle(N, j)) * e2
    else:
        n = -e2 if side == BOTTOM else e2
        Q = c + n + math.tan(angle(N, i)) * e1
    sj, si = frac_index(Q, g, N)
    t = sj if axis == "i" else si
    tg = int(round(t))
    assert abs(t - tg) < 1e-6
    return _node(g, axis, L, tg)


def _tangents(f: int, a: float, b: float, eps: float = 1e-6):
    c, e1, e2 = FRAMES[f]

    def X(a_, b_):
        p = c + math.tan(a_) * e1 + math.tan(b_) * e2
        return p / np.linalg.norm(p)

    ta = (X(a + eps, b) - X(a - eps, b)) / (2 * eps)
    tb = (X(a, b + eps) - X(a, b - eps)) / (2 * eps)
    return ta / np.linalg.norm(ta), tb / np.linalg.norm(tb), X(a, b)


def side_neighbour(f: int, side: int) -> int:
    c, e1, e2 = FRAMES[f]
    n = {LEFT: -e1, RIGHT: e1, BOTTOM: -e2, TOP: e2}[side]
    return int(np.argmax(FRAMES[:, 0, :] @ n))


def rside(f: int, side: int) -> np.ndarray:
    """2x2 integer matrix R with (u, v)_ghost = R (u', v')_neighbour."""
    q = math.pi / 4
    a, b = {LEFT: (-q, 0.0), RIGHT: (q, 0.0), BOTTOM: (0.0, -q), TOP: (0.0, q)}[side]
    taf, tbf, Q = _tangents(f, a, b)
    g = side_neighbour(f, side)
    cg, e1g, e2g = FRAMES[g]
    pc = float(Q @ cg)
    ag = math.atan(float(Q @ e1g) / pc)
    bg = math.atan(float(Q @ e2g) / pc)
    tag, tbg, _ = _tangents(g, ag, bg)
    R = np.array([[taf @ tag, taf @ tbg], [tbf @ tag, tbf @ tbg]])
    Ri = np.rint(R).astype(np.int64)
    assert np.abs(R - Ri).max() < 1e-6
    return Ri


def grid(N: int, h: int) -> Grid:
    """Six blocks along the leading (face) coordinate, full [-h, N+h)^2, data [0, N)^2."""
    gr = Grid([0, -h, -h], [6, N + h, N + h])
    for f in range(6):
        gr.add_block([(f, f + 1), (-h, N + h), (-h, N + h)], [(f, f + 1), (0, N), (0, N)])
    return gr


def side_box(f: int, side: int, N: int, h: int):
    fb = (f, f + 1)
    return {
        LEFT: [fb, (0, N), (-h, 0)],
        RIGHT: [fb, (0, N), (N, N + h)],
        BOTTOM: [fb, (-h, 0), (0, N)],
        TOP: [fb, (N, N + h), (0, N)],
    }[side]


def corner_boxes(f: int, N: int, h: int):
    fb = (f, f + 1)
    lo, hi = (-h, 0), (N, N + h)
    return [[fb, a, b] for a in (lo, hi) for b in (lo, hi)]


def subs(N: int, h: int, mode: str = "lagrange", vector: bool = False) -> List:
    """Basic sub-matrices of the cubed-sphere BC programs.

    ``mode='lagrange'``: 24 interpolation sub-matrices (one per face side) +
    24 zero corners.  ``mode='sync'``: 24 rotated halo-copy sub-matrices + 24
    zero corners.  With ``vector`` each side carries its component rotation.
    """
    out = []
    for f in range(6):
        for side in (LEFT, RIGHT, BOTTOM, TOP):
            rot = tuple(int(v) for v in rside(f, side).reshape(-1)) if vector else None
            box = side_box(f, side, N, h)
            if mode == "lagrange":
                out.append(RowsSub(box, lambda c, f=f: lagrange_entries(f, c[1], c[2], N), rot=rot))
            elif mode == "sync":
                out.append(MapSub(box, lambda c, f=f: sync_source(f, c[1], c[2], N), 1.0, rot=rot))
            else:
                raise ValueError(mode)
        for box in corner_boxes(f, N, h):
            out.append(ZeroSub(box))
    return out


def ghost_point_unit(f: int, j: int, i: int, N: int) -> np.ndarray:
    P = plane_point(f, j, i, N)
    return P / np.linalg.norm(P)


def local_tangents_at_cell(f: int, j: float, i: float, N: int):
    """Unit tangents (alpha, beta directions) of face f at cell (j, i)."""
    ta, tb, _ = _tangents(f, angle(N, i), angle(N, j))
    return ta, tb
