"""Pins of the consumer-footprint restriction of the CPU reference (Sec. IV-C).

Counts are tied to closed forms of the grid shapes, and the restriction to
its purpose: the consumer's output is unchanged, and dropped ghosts are
never written.
"""
import numpy as np
import pytest

from oracle import apply, assemble
from oracle import cubed_sphere as ocs
from oracle import footprint as ofp
from oracle import hpcg as ohpcg


def cross(r):
    """Offsets (0, dj, di) of a 2-D cross of radius r on the cubed sphere."""
    out = [(0, 0, 0)]
    for k in range(1, r + 1):
        out += [(0, k, 0), (0, -k, 0), (0, 0, k), (0, 0, -k)]
    return out


@pytest.mark.parametrize("N,h,r", [(6, 3, 1), (8, 3, 2), (5, 2, 2), (7, 1, 1)])
def test_cross_live_ghosts_closed_form(N, h, r):
    g = ocs.grid(N, h)
    live = ofp.live_ghost_mask(g, cross(r))
    # per face: r layers of each of the 4 strips, no corners
    assert live.sum() == 6 * 4 * min(r, h) * N


def test_box_stencil_reaches_corners_and_cartesian_faces():
    g = ocs.grid(6, 2)
    box = [(0, a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)]
    live = ofp.live_ghost_mask(g, box)
    # one full ring around each face: 4 N + 4 corners
    assert live.sum() == 6 * (4 * 6 + 4)
    hg = ohpcg.grid(2, 4)
    seven = [(0, 0, 0, 0)] + [tuple(s * (k == d) for k in range(4)) for d in (1, 2, 3) for s in (1, -1)]
    live = ofp.live_ghost_mask(hg, seven)
    assert live.sum() == 8 * 6 * 4 * 4  # faces only, no edges or corners


def cross_sum(u, N, h, r):
    """sum over the cross offsets of the field, at every data cell of every face."""
    W = N + 2 * h
    v = u.reshape(6, W, W, -1)
    s = slice(h, h + N)
    out = v[:, s, s].copy()
    for k in range(1, r + 1):
        out = out + v[:, h + k:h + k + N, s] + v[:, h - k:h - k + N, s]
        out = out + v[:, s, h + k:h + k + N] + v[:, s, h - k:h - k + N]
    return out


@pytest.mark.parametrize("mode", ["sync", "lagrange"])
def test_consumer_output_unchanged_and_dead_ghosts_untouched(mode):
    N, h, r = 8, 3, 2
    g = ocs.grid(N, h)
    rng = np.random.default_rng(1)
    u = np.full((g.ncells, 2), np.nan)
    u[g.data_cells] = rng.standard_normal((g.ndata, 2))
    op = assemble(g, ocs.subs(N, h, mode))
    live = ofp.live_ghost_mask(g, cross(r))
    full = apply(op, u)
    part = apply(ofp.restrict(op, live), u)
    assert np.array_equal(cross_sum(full, N, h, r), cross_sum(part, N, h, r))
    G = g.ghost_cells
    assert np.isnan(part[G][~live]).all()
    assert np.array_equal(part[G][live], full[G][live])
    # a smaller footprint than the consumer's would change the output
    small = ofp.live_ghost_mask(g, cross(r - 1))
    bad = apply(ofp.restrict(op, small), u)
    assert np.isnan(cross_sum(bad, N, h, r)).any()
