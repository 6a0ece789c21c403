"""Pins of the CPU reference's HPCG-shaped case (not GPU).

* closed form: on x = 1 the 27-point operator (26 on the diagonal, -1 off it)
  with zero padding gives 27 minus the number of in-domain points of the
  3x3x3 box: 0 inside, 9 on faces, 15 on edges, 19 at corners;
* split invariance: 2x2x2 blocks with halo copies equal the unsplit
  zero-padded domain;
* the generic sub-matrix assembly of the same BC equals the block split and
  a brute-force dense A built from physical positions.
"""
import numpy as np
import pytest

from oracle import apply, assemble
from oracle import dense, hpcg


@pytest.mark.parametrize("nd", [4, 6, 16])
def test_closed_form_on_ones(nd):
    x = np.ones((nd, nd, nd))
    idx = np.arange(nd)
    on_b = ((idx == 0) | (idx == nd - 1)).astype(int)
    cnt = on_b[:, None, None] + on_b[None, :, None] + on_b[None, None, :]
    want = np.select([cnt == 0, cnt == 1, cnt == 2, cnt == 3], [0.0, 9.0, 15.0, 19.0])
    assert np.array_equal(hpcg.stencil27_padded(x), want)
    ys = [hpcg.stencil27(b) for b in hpcg.ghosted_blocks(x, 2)]
    assert np.array_equal(assemble_blocks(ys, 2), want)


def assemble_blocks(ys, nb):
    n = ys[0].shape[0]
    out = np.empty((nb * n,) * 3)
    for bz in range(nb):
        for by in range(nb):
            for bx in range(nb):
                out[bz * n:(bz + 1) * n, by * n:(by + 1) * n, bx * n:(bx + 1) * n] = ys[hpcg.block_index(nb, bz, by, bx)]
    return out


@pytest.mark.parametrize("nd", [8, 32])
def test_split_invariance(nd):
    x = np.random.default_rng(3).uniform(-1, 1, (nd, nd, nd))
    ys = [hpcg.stencil27(b) for b in hpcg.ghosted_blocks(x)]
    assert np.array_equal(assemble_blocks(ys, 2), hpcg.stencil27_padded(x))


def test_generic_assembly_equals_blocks_and_bruteforce():
    nb, n = 2, 4
    g = hpcg.grid(nb, n)
    op = assemble(g, hpcg.subs(nb, n))
    assert op.covered.all()
    A = op.dense()
    assert np.array_equal(A, dense.cartesian_halo(g, nb, n))
    x = np.random.default_rng(5).uniform(-1, 1, (nb * n,) * 3)
    u = np.full((g.ncells, 1), np.nan)
    blocks = hpcg.ghosted_blocks(x, nb)
    for b in range(nb ** 3):
        cells = g.cells_of_box(b, g.blocks[b].data)
        u[cells, 0] = blocks[b][1:-1, 1:-1, 1:-1].reshape(-1)
    out = apply(op, u)
    for b in range(nb ** 3):
        cells = g.cells_of_box(b, g.blocks[b].full)
        assert np.array_equal(out[cells, 0].reshape((n + 2,) * 3), blocks[b])
    # copy rows: one entry 1.0; rows outside the domain: empty
    nnz = (A != 0).sum(axis=1)
    assert set(np.unique(nnz)) == {0, 1}
