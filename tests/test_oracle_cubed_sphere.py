"""Pins of the CPU reference's cubed-sphere rows (not GPU).

* connectivity: each of the 24 face sides has a unique partner side and the
  relation is symmetric; the ghost's grid line is at the mirrored layer;
* rotated copy rows: exact permutation rows, brute-force dense agreement;
* Lagrange rows: partition of unity, first moment, cubic reproduction,
  fourth-order convergence to a smooth field, brute-force dense agreement;
* component rotation: signed permutations with det +1, and a solid-body
  rotation velocity field reproduced to first order in the mesh width with
  tangents written analytically here (not the reference's finite
  differences).
"""
import math

import numpy as np
import pytest

from oracle import apply, assemble
from oracle import cubed_sphere as cs
from oracle import dense


def edge_ghosts(N, h):
    for f in range(6):
        for j in range(-h, N + h):
            for i in range(-h, N + h):
                if (0 <= i < N and 0 <= j < N) or cs.is_corner(j, i, N):
                    continue
                yield f, j, i


def layer(j, i, N):
    side = cs.side_of(j, i, N)
    return {cs.LEFT: -1 - i, cs.RIGHT: i - N, cs.BOTTOM: -1 - j, cs.TOP: j - N}[side]


@pytest.mark.parametrize("N", [8, 13, 48])
def test_connectivity_is_an_involution(N):
    h = 3
    partner = {}
    for f, j, i in edge_ghosts(N, h):
        g, axis, L, s = cs.neighbour_line(f, j, i, N)
        k = layer(j, i, N)
        assert L in (k, N - 1 - k)
        if N - 1 - k == k:
            continue
        gside = {("i", k): cs.LEFT, ("i", N - 1 - k): cs.RIGHT, ("j", k): cs.BOTTOM, ("j", N - 1 - k): cs.TOP}[(axis, L)]
        key = (f, cs.side_of(j, i, N))
        assert partner.setdefault(key, (g, gside)) == (g, gside)
    assert len(partner) == 24
    assert len(set(partner.values())) == 24
    for (f, side), (g, gside) in partner.items():
        assert partner[(g, gside)] == (f, side)
        assert g == cs.side_neighbour(f, side)


@pytest.mark.parametrize("N,h", [(4, 1), (5, 2), (6, 3), (8, 3)])
def test_sync_rows_match_bruteforce(N, h):
    g = cs.grid(N, h)
    op = assemble(g, cs.subs(N, h, "sync"))
    A = op.dense()
    B = dense.cubed_sync(N, h)
    assert np.array_equal(A, B)
    # permutation rows: one entry 1.0 per edge ghost, none per corner ghost
    nnz = (A != 0).sum(axis=1)
    assert set(np.unique(A)) <= {0.0, 1.0}
    assert int((nnz == 1).sum()) == 6 * 4 * h * N and int((nnz == 0).sum()) == 6 * 4 * h * h


@pytest.mark.parametrize("N,h", [(4, 1), (5, 2), (6, 3), (8, 3)])
def test_lagrange_rows_match_bruteforce(N, h):
    g = cs.grid(N, h)
    op = assemble(g, cs.subs(N, h, "lagrange"))
    A = op.dense()
    B = dense.cubed_lagrange(N, h)
    assert np.array_equal(A != 0, B != 0)
    assert np.abs(A - B).max() <= 1e-14


@pytest.mark.parametrize("N", [8, 24, 96])
def test_lagrange_row_invariants_and_cubic_reproduction(N):
    h = 3
    rng = np.random.default_rng(N)
    for f, j, i in edge_ghosts(N, h):
        g, axis, L, s = cs.neighbour_line(f, j, i, N)
        ents = cs.lagrange_entries(f, j, i, N)
        along = [c[1] if axis == "i" else c[2] for c, _ in ents]
        lines = {c[2] if axis == "i" else c[1] for c, _ in ents}
        assert lines == {L} and all(c[0] == g for c, _ in ents)
        assert along == list(range(along[0], along[0] + 4))
        w = np.array([v for _, v in ents])
        assert abs(w.sum() - 1.0) <= 1e-15 * 8
        assert abs(float(w @ np.array(along)) - s) <= 1e-12 * max(1.0, abs(s))
        p = rng.standard_normal(4)
        pv = np.polyval(p, np.array(along, dtype=float))
        exact = np.polyval(p, s)
        scale = np.abs(np.polyval(np.abs(p), max(abs(s), along[-1])))
        assert abs(float(w @ pv) - exact) <= 1e-13 * scale


def smooth(P):
    x, y, z = P[..., 0], P[..., 1], P[..., 2]
    return np.sin(2.0 * x + 0.3) * np.cos(1.5 * y) + 0.5 * z * z * x + np.exp(0.7 * z)


def interp_error(N, h=3):
    g = cs.grid(N, h)
    op = assemble(g, cs.subs(N, h, "lagrange"))
    u = np.full((g.ncells, 1), np.nan)
    exact = {}
    for cell in g.data_cells:
        _, (f, j, i) = g.coord_of_cell(int(cell))
        u[cell, 0] = smooth(cs.ghost_point_unit(f, j, i, N))
    out = apply(op, u)
    err = 0.0
    for cell in g.ghost_cells:
        _, (f, j, i) = g.coord_of_cell(int(cell))
        if cs.is_corner(j, i, N):
            assert out[cell, 0] == 0.0
            continue
        err = max(err, abs(out[cell, 0] - smooth(cs.ghost_point_unit(f, j, i, N))))
    return err


@pytest.mark.slow
def test_lagrange_fourth_order_convergence():
    errs = [interp_error(N) for N in (12, 24, 48, 96)]
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    assert all(r > 8.0 for r in ratios), ratios
    assert ratios[-1] > 13.0, ratios


def test_rside_signed_permutation_det_one():
    for f in range(6):
        for side in range(4):
            R = cs.rside(f, side)
            assert (np.abs(R).sum(axis=0) == 1).all() and (np.abs(R).sum(axis=1) == 1).all()
            assert round(np.linalg.det(R)) == 1


def analytic_tangents(f, j, i, N):
    """Unit tangents of face f's alpha / beta lines at index (j, i) (analytic derivative)."""
    c, e1, e2 = cs.FRAMES[f]
    t1, t2 = math.tan(cs.angle(N, i)), math.tan(cs.angle(N, j))
    P = c + t1 * e1 + t2 * e2
    n2 = float(P @ P)
    ta = e1 - (t1 / n2) * P
    tb = e2 - (t2 / n2) * P
    return ta / np.linalg.norm(ta), tb / np.linalg.norm(tb), P / math.sqrt(n2)


def rotation_error(N, mode, h=2):
    omega = np.array([0.3, -0.5, 0.8])
    g = cs.grid(N, h)
    op = assemble(g, cs.subs(N, h, mode, vector=True))
    u = np.full((g.ncells, 2), np.nan)
    for cell in g.data_cells:
        _, (f, j, i) = g.coord_of_cell(int(cell))
        ta, tb, X = analytic_tangents(f, j, i, N)
        V = np.cross(omega, X)
        u[cell] = (V @ ta, V @ tb)
    out = apply(op, u, vec=(0, 1, 1))
    err = 0.0
    for cell in g.ghost_cells:
        _, (f, j, i) = g.coord_of_cell(int(cell))
        if cs.is_corner(j, i, N):
            continue
        # the gnomonic coordinate lines are orthogonal only on the mid-lines of a
        # face, so the signed permutation is exact only near the edge midpoint:
        # compare the ghosts whose tangential index is next to the middle
        t = j if cs.side_of(j, i, N) in (cs.LEFT, cs.RIGHT) else i
        if abs(t - (N - 1) / 2) > 1.0:
            continue
        ta, tb, X = analytic_tangents(f, j, i, N)
        V = np.cross(omega, X)
        err = max(err, float(np.abs(out[cell] - (V @ ta, V @ tb)).max()))
    return err


@pytest.mark.parametrize("mode", ["sync", "lagrange"])
def test_component_rotation_solid_body(mode):
    e = [rotation_error(N, mode) for N in (12, 24, 48)]
    # a wrong sign or swapped component gives an O(1) error; the right one is O(mesh width)
    assert e[0] < 0.5 and e[1] < 0.6 * e[0] and e[2] < 0.6 * e[1], e
