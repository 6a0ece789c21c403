"""Pins of the block-edge averaging rows of the CPU reference (Sec. III-B).

The co-located sets are found by 3-D position; these tests tie them to the
topology of the cube and the rows to what averaging must do, without
re-stating the reference's construction.
"""
import numpy as np
import pytest

from oracle import averaging as oav
from oracle import cubed_sphere as ocs
from oracle import assemble, apply


@pytest.mark.parametrize("Np", [3, 4, 7, 10])
def test_distinct_positions_match_cube_vertex_count(Np):
    # a cube surface cut into (Np-1)^2 quads per face has 6 (Np-1)^2 + 2
    # vertices (Euler: V - E + F = 2 with F = 6 n^2, E = 12 n^2)
    n = Np - 1
    assert len(oav.colocated_sets(Np, which="all")) == 6 * n * n + 2


@pytest.mark.parametrize("Np", [3, 5, 9])
def test_set_sizes_are_cube_edges_and_corners(Np):
    sizes = sorted(len(s) for s in oav.colocated_sets(Np))
    # 12 cube edges with Np-2 interior points shared by 2 faces, 8 corners shared by 3
    assert sizes.count(2) == 12 * (Np - 2)
    assert sizes.count(3) == 8
    assert set(sizes) <= {2, 3}
    # every copy of a set is a boundary point of a different face
    for s in oav.colocated_sets(Np):
        assert len({f for f, _, _ in s}) == len(s)
        for f, j, i in s:
            assert i in (0, Np - 1) or j in (0, Np - 1)


def _field(Np, h, seed, I=2):
    g = ocs.grid(Np, h)
    rng = np.random.default_rng(seed)
    u = np.full((g.ncells, I), np.nan)
    u[g.data_cells] = rng.standard_normal((g.ndata, I))
    return g, u


def _sets_as_cells(g, Np):
    return [[g.cell(m) for m in s] for s in oav.colocated_sets(Np) if len(s) > 1]


def test_rows_average_to_a_consensus():
    Np, h = 6, 2
    g, u = _field(Np, h, 1)
    op = assemble(g, [])
    dop = oav.assemble_data(g, oav.edge_average_subs(Np))
    out = oav.apply_with_data_rows(op, dop, u)
    for cells in _sets_as_cells(g, Np):
        vals = out[cells]
        # every copy holds the mean of the input copies (within rounding)
        want = u[cells].mean(axis=0)
        assert np.allclose(vals, want[None, :], rtol=0, atol=4e-16 * np.abs(u[cells]).sum())
        assert np.abs(vals - vals[0]).max() <= 4e-16 * np.abs(u[cells]).sum()
    # interior points and ghosts are untouched
    inner = np.ones(g.ncells, dtype=bool)
    for cells in _sets_as_cells(g, Np):
        inner[cells] = False
    assert np.array_equal(out[inner], u[inner], equal_nan=True)


def test_constant_and_zero_sum_perturbations():
    Np, h = 5, 1
    g, u = _field(Np, h, 2)
    sets = _sets_as_cells(g, Np)
    c = 1.75
    u[g.data_cells] = c
    rng = np.random.default_rng(3)
    for cells in sets:
        d = rng.standard_normal((len(cells), u.shape[1]))
        d -= d.mean(axis=0)  # zero-sum perturbation of the copies
        u[cells] = c + d
    dop = oav.assemble_data(g, oav.edge_average_subs(Np))
    out = oav.apply_with_data_rows(assemble(g, []), dop, u)
    for cells in sets:
        assert np.abs(out[cells] - c).max() <= 1e-14


def test_rows_read_the_input_not_updated_values():
    # two applications of an averaging map: the second changes nothing, the
    # first uses only input values (a row computed from already-averaged
    # copies would differ for sets of 3)
    Np, h = 4, 1
    g, u = _field(Np, h, 4, I=1)
    dop = oav.assemble_data(g, oav.edge_average_subs(Np))
    op = assemble(g, [])
    once = oav.apply_with_data_rows(op, dop, u)
    twice = oav.apply_with_data_rows(op, dop, once)
    for cells in _sets_as_cells(g, Np):
        assert np.abs(twice[cells] - once[cells]).max() <= 4e-16 * np.abs(u[cells]).sum()
        assert np.abs(once[cells] - u[cells].mean()).max() <= 4e-16 * np.abs(u[cells]).sum()


def test_ghost_rows_use_the_input_data_values():
    # a ghost sync program next to averaging rows: ghosts copy the *input*
    # values of their source cells, even where those cells are averaged
    Np, h = 5, 2
    g, u = _field(Np, h, 5, I=1)
    op = assemble(g, ocs.subs(Np, h, "sync"))
    dop = oav.assemble_data(g, oav.edge_average_subs(Np))
    both = oav.apply_with_data_rows(op, dop, u)
    ghosts_only = apply(op, u)
    G = g.ghost_cells
    assert np.array_equal(both[G], ghosts_only[G])


def test_rejects_ghost_rows_and_duplicates():
    Np, h = 4, 1
    g = ocs.grid(Np, h)
    with pytest.raises(ValueError):
        oav.assemble_data(g, [oav.DataRowsSub([(0, -1, 0)], [[((0, 0, 0), 1.0)]])])
    with pytest.raises(ValueError):
        oav.assemble_data(g, [oav.DataRowsSub([(0, 0, 0), (0, 0, 0)], [[((0, 0, 1), 1.0)]] * 2)])
