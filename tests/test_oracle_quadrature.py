"""Pins of the wide (quadrature x tensor-product) interpolation rows (Sec. III-B, Agg . Recons)."""
import math

import numpy as np
import pytest

import synthinputs
from oracle import apply, assemble
from oracle import cubed_sphere as ocs
from oracle import quadrature as oq


def test_gauss_legendre_rule():
    x, w = oq.gauss_legendre(2)
    assert np.allclose(x, [-1 / (2 * math.sqrt(3)), 1 / (2 * math.sqrt(3))], rtol=0, atol=1e-15)
    assert np.allclose(w, [0.5, 0.5], rtol=0, atol=1e-15)
    # exact for cubics on the cell [-1/2, 1/2]: mean of t^2 is 1/12
    assert abs((w * x ** 2).sum() - 1 / 12) < 1e-16 and abs((w * x ** 3).sum()) < 1e-16


@pytest.mark.parametrize("N,h", [(8, 2), (12, 3)])
def test_row_sums_and_widths(N, h):
    for f in range(6):
        for (j, i) in [(0, -1), (3, N), (-2, 5), (N + h - 1, N - 1), (N - 1, -h)]:
            ents = oq.quad_entries(f, j, i, N)
            assert abs(sum(w for _, w in ents) - 1.0) < 1e-13
            assert 16 <= len(ents) <= 25  # union of 4 overlapping 4x4 stencils
            assert all(c[0] == ocs.side_neighbour(f, ocs.side_of(j, i, N)) for c, _ in ents)


@pytest.mark.parametrize("N,h", [(8, 3), (11, 2)])
def test_exact_for_tensor_cubics(N, h):
    """Data = a tensor-product cubic in each neighbour face's index space: the
    row returns the quadrature of that cubic at the projected points."""
    rng = np.random.default_rng(N)
    coef = rng.standard_normal((6, 4, 4))

    def poly(g, sj, si):
        return sum(coef[g, a, b] * sj ** a * si ** b for a in range(4) for b in range(4))

    g = ocs.grid(N, h)
    u = np.full((g.ncells, 1), np.nan)
    for cell in g.data_cells:
        f, j, i = g.coord_of_cell(cell)[1]
        u[cell, 0] = poly(f, j, i)
    out = apply(assemble(g, oq.subs(N, h)), u)
    scale = np.nanmax(np.abs(u))
    for f in range(6):
        for (j, i) in [(0, -1), (4, N + 1), (-h, 3), (N, N - 2)]:
            want = sum(w * poly(gg, sj, si) for gg, sj, si, w in oq.quad_points(f, j, i, N))
            got = out[g.cell((f, j, i)), 0]
            assert abs(got - want) <= 1e-12 * scale, (f, j, i, got, want)


def cell_average_exact(fun, f, j, i, N, q=8):
    """Reference cell average of ``fun`` (a function of the unit 3-D point) over
    ghost cell (f, j, i) in angle space, by a q x q Gauss rule."""
    x, w = oq.gauss_legendre(q)
    D = math.pi / (2 * N)
    c, e1, e2 = ocs.FRAMES[f]
    tot = 0.0
    for xb, wb in zip(x, w):
        for xa, wa in zip(x, w):
            P = c + math.tan(ocs.angle(N, i) + xa * D) * e1 + math.tan(ocs.angle(N, j) + xb * D) * e2
            tot += wa * wb * fun(P / np.linalg.norm(P))
    return tot


def test_converges_to_cell_averages():
    """Fourth order: the error of the ghost averages of a smooth field falls
    by about 16 each time N doubles."""
    terms = [(2, 1, 0.7), (3, -2, -0.4), (1, 0, 0.3)]

    def fun(p):
        return sum(c * synthinputs.real_sh(l, m, p[None, :])[0] for l, m, c in terms)

    errs = []
    for N in (8, 16, 32):
        h = 2
        g = ocs.grid(N, h)
        u = np.full((g.ncells, 1), np.nan)
        pts = synthinputs.cs_cell_centres(N)
        vals = sum(c * synthinputs.real_sh(l, m, pts) for l, m, c in terms)
        W = N + 2 * h
        uu = u.reshape(6, W, W)
        uu[:, h:h + N, h:h + N] = vals
        # the data are point values; cell averages differ at second order, so
        # compare against the point-value reconstruction target instead: the
        # quadrature of the field at the projected points
        out = apply(assemble(g, oq.subs(N, h)), u)
        e = 0.0
        for f in range(6):
            for (j, i) in [(N // 3, -1), (N // 2, N), (-1, N // 4), (N, 2 * N // 3)]:
                want = cell_average_exact(fun, f, j, i, N, q=2)
                e = max(e, abs(out[g.cell((f, j, i)), 0] - want))
        errs.append(e)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert r1 > 10 and r2 > 12, errs
