"""Pins of the consumer reference (oracle.consumer.stencil_after_bc), the
stencil evaluated on the field after the BC (Sec. IV-C).

* With the HPCG halo program and the 27 offsets of weight 26 (centre) / -1,
  it is the 27-point operator of oracle.hpcg on the ghosted blocks, itself
  pinned by closed forms and by numpy.pad of the whole domain.
* On tiny cubed spheres it equals the dense composition S_D x_D + S_G (A x_D + b)
  with A the brute-force dense operator (oracle.dense, entry by entry from
  the geometry) and S the stencil written out as a matrix by enumeration.
* It never reads a ghost no offset reaches: the operator restricted to the
  consumer footprint (oracle.footprint) gives the same result, with NaN in
  every dropped ghost.
* A zero-sum stencil of a constant field is 0 whenever the BC reproduces
  constants (copy and Lagrange rows).
"""
import itertools

import numpy as np
import pytest

import synthinputs
from oracle import VectorSub, apply, assemble
from oracle import cubed_sphere as ocs
from oracle import dense as odense
from oracle import footprint as ofp
from oracle import hpcg as ohpcg
from oracle.consumer import stencil_after_bc

CROSS = [(0, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
CROSS_W = [-4.0, 1.0, 1.0, 1.0, 1.0]


@pytest.mark.parametrize("nb,n", [(2, 5), (1, 4), (3, 3)])
def test_reduces_to_the_27_point_operator(nb, n):
    g = ohpcg.grid(nb, n)
    op = assemble(g, ohpcg.subs(nb, n))
    x = synthinputs.uniform((nb * n,) * 3, seed=3)
    blocks = ohpcg.ghosted_blocks(x, nb)
    full = np.full(g.ncells, np.nan)
    for b in range(nb ** 3):
        full[g.cells_of_box(b, g.blocks[b].data)] = blocks[b][1:-1, 1:-1, 1:-1].reshape(-1)
    offs = [(0,) + d for d in itertools.product((-1, 0, 1), repeat=3)]
    w = [26.0 if d == (0, 0, 0, 0) else -1.0 for d in offs]
    y = stencil_after_bc(op, full, offs, w)[:, 0]
    want = np.concatenate([ohpcg.stencil27(b).reshape(-1) for b in blocks])
    bound = np.concatenate([ohpcg.abs_row_sum(b).reshape(-1) for b in blocks])
    assert (np.abs(y - want) <= 64 * 2.0 ** -53 * bound).all()
    # and the unsplit domain
    assert np.allclose(np.concatenate([ohpcg.stencil27_padded(x)[bz * n:(bz + 1) * n, by * n:(by + 1) * n,
                                                                  bx * n:(bx + 1) * n].reshape(-1)
                                       for bz in range(nb) for by in range(nb) for bx in range(nb)]),
                       y, rtol=0, atol=1e-12)


@pytest.mark.parametrize("N,h,offs,w", [(5, 2, CROSS, CROSS_W),
                                        (6, 2, [(0, 0, 0), (0, 2, 0), (0, -1, -1), (0, 0, 2)], [0.5, -1.0, 2.0, 0.25])])
def test_matches_dense_composition_on_tiny_cubed_spheres(N, h, offs, w):
    g = ocs.grid(N, h)
    rng = np.random.default_rng(N)
    bvals = rng.standard_normal((h * N, 1))
    subs = ocs.subs(N, h, "lagrange") + [VectorSub(ocs.side_box(1, ocs.TOP, N, h), bvals)]
    op = assemble(g, subs)
    u = rng.standard_normal((g.ncells, 1))
    y = stencil_after_bc(op, u, offs, w)[:, 0]
    # brute force: dense A (entry by entry from the geometry) and the stencil
    # matrix over all cells, rows = data cells in order
    A = odense.cubed_lagrange(N, h)
    G, D = g.ghost_cells, g.data_cells
    b = np.zeros(len(G))
    gi = {int(c): r for r, c in enumerate(G)}
    for k, (j, i) in enumerate((j, i) for j in range(N, N + h) for i in range(N)):
        b[gi[g.cell((1, j, i))]] += bvals[k, 0]
    S = np.zeros((len(D), g.ncells))
    for r, c in enumerate(D):
        _, coord = g.coord_of_cell(int(c))
        for o, wo in zip(offs, w):
            S[r, g.cell(tuple(a + s for a, s in zip(coord, o)))] += wo
    want = S[:, D] @ u[D, 0] + S[:, G] @ (A @ u[D, 0] + b)
    assert np.abs(y - want).max() <= 1e-13 * (np.abs(S) @ np.abs(np.concatenate([u[:, 0]]))).max() * 10


def test_footprint_restriction_changes_nothing():
    N, h = 8, 3
    g = ocs.grid(N, h)
    op = assemble(g, ocs.subs(N, h, "lagrange", vector=True))
    u = np.full((g.ncells, 4), np.nan)
    u[g.data_cells] = synthinputs.cs_sh_field(N, 4, 1, seed=4).reshape(-1, 4)
    live = ofp.live_ghost_mask(g, CROSS)
    assert 0 < live.sum() < g.nghost
    y_full = stencil_after_bc(op, u, CROSS, CROSS_W, vec=(2, 1, 1))
    y_live = stencil_after_bc(ofp.restrict(op, live), u, CROSS, CROSS_W, vec=(2, 1, 1))
    assert np.isfinite(y_full).all()
    assert np.array_equal(y_full, y_live)


@pytest.mark.parametrize("mode", ["sync", "lagrange"])
def test_zero_sum_stencil_of_a_constant_is_zero(mode):
    N, h = 12, 2
    g = ocs.grid(N, h)
    op = assemble(g, ocs.subs(N, h, mode))
    u = np.full((g.ncells, 1), 3.25)
    y = stencil_after_bc(op, u, CROSS, CROSS_W)
    assert np.abs(y).max() <= 1e-13


def test_reads_outside_a_block_are_refused():
    g = ocs.grid(6, 1)
    op = assemble(g, ocs.subs(6, 1, "sync"))
    with pytest.raises(ValueError):
        stencil_after_bc(op, np.zeros((g.ncells, 1)), [(0, 2, 0)], [1.0])
