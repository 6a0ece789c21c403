"""Wide interpolation rows: cell averages by quadrature of a tensor-product
reconstruction (reference implementation).

Sec. III-B describes HOPE's ghost computation as the product of two linear
maps, ``Itp = Agg . Recons``: a tensor-product polynomial reconstruction of
the neighbour's data at a set of points, and a Gaussian quadrature that
aggregates those point values into the ghost cell's value.  Users hand the
product to the library as a (wide) sparse row per ghost.

The instance modelled here (readings, documented with the design): the ghost
cell (f, j, i) of an edge strip covers ``[alpha_i - D/2, alpha_i + D/2] x
[beta_j - D/2, beta_j + D/2]`` in f's angles (D = pi / 2N); a q x q
Gauss-Legendre rule on that square (q = 2: nodes at +-1/(2 sqrt 3) cell
widths, weights 1/4) gives points, each projected onto the neighbour face g
across that side, where a 4 x 4 tensor-product Lagrange stencil in g's index
space (base ``clamp(floor(s) - 1, 0, N - 4)`` per direction) reconstructs the
value.  The row is the union of the stencils with the weights summed, in
ascending cell order.  Corner ghosts are zero rows.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

from .cubed_sphere import (BOTTOM, FRAMES, LEFT, RIGHT, TOP, angle, corner_boxes, frac_index, rside, side_box,
                           side_neighbour, side_of)
from .operator import RowsSub, ZeroSub


def gauss_legendre(q: int) -> Tuple[np.ndarray, np.ndarray]:
    """Nodes (in cell widths, on [-1/2, 1/2]) and weights (summing to 1)."""
    x, w = np.polynomial.legendre.leggauss(q)
    return x / 2.0, w / 2.0


def lagrange4(s: float, N: int):
    """Base and the 4 Lagrange weights of nodes base .. base + 3 at s."""
    base = min(max(math.floor(s) - 1, 0), N - 4)
    d = [s - (base + n) for n in range(4)]
    return base, [-d[1] * d[2] * d[3] / 6.0, d[0] * d[2] * d[3] / 2.0, -d[0] * d[1] * d[3] / 2.0,
                  d[0] * d[1] * d[2] / 6.0]


def quad_points(f: int, j: int, i: int, N: int, q: int = 2):
    """(g, s_j, s_i, weight) of every quadrature point of ghost cell (f, j, i)."""
    side = side_of(j, i, N)
    g = side_neighbour(f, side)
    x, w = gauss_legendre(q)
    D = math.pi / (2 * N)
    c, e1, e2 = FRAMES[f]
    out = []
    for xb, wb in zip(x, w):
        for xa, wa in zip(x, w):
            a = angle(N, i) + xa * D
            b = angle(N, j) + xb * D
            P = c + math.tan(a) * e1 + math.tan(b) * e2
            assert int(np.argmax(FRAMES[:, 0, :] @ P)) == g
            sj, si = frac_index(P, g, N)
            out.append((g, sj, si, wa * wb))
    return out


def quad_entries(f: int, j: int, i: int, N: int, q: int = 2):
    acc: Dict[tuple, float] = {}
    for g, sj, si, wq in quad_points(f, j, i, N, q):
        bj, wj = lagrange4(sj, N)
        bi, wi = lagrange4(si, N)
        for a in range(4):
            for b in range(4):
                key = (g, bj + a, bi + b)
                acc[key] = acc.get(key, 0.0) + wq * wj[a] * wi[b]
    return sorted(acc.items())


def subs(N: int, h: int, q: int = 2, vector: bool = False) -> List:
    out = []
    for f in range(6):
        for side in (LEFT, RIGHT, BOTTOM, TOP):
            rot = tuple(int(v) for v in rside(f, side).reshape(-1)) if vector else None
            out.append(RowsSub(side_box(f, side, N, h), lambda c, f=f: quad_entries(f, c[1], c[2], N, q), rot=rot))
        for box in corner_boxes(f, N, h):
            out.append(ZeroSub(box))
    return out
