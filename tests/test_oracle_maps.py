"""Pins of the CPU reference's generic assembly (not GPU).

* zero / circular / symmetric padding against ``numpy.pad`` ('constant',
  'wrap', 'symmetric'), with the left-side index maps of Sec. III-B and their
  mirror on the right side;
* the Alg. 1 worked example (regions, rotated map, zero region incl. corners);
* overlap rejection / summation, uncovered rows, sub-vectors;
* the dot-product identity for the vector-Jacobian product.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import Grid, MapSub, RowsSub, VectorSub, ZeroSub, assemble, apply, vjp

HERE = os.path.dirname(os.path.abspath(__file__))


def one_block(n0, n1, h):
    g = Grid([0, -h, -h], [1, n0 + h, n1 + h])
    g.add_block([(0, 1), (-h, n0 + h), (-h, n1 + h)], [(0, 1), (0, n0), (0, n1)])
    return g


def fmap_1d(kind, n):
    """Index map of one axis for a ghost coordinate r (Sec. III-B left side; mirrored right)."""
    def f(r):
        if 0 <= r < n:
            return r
        if kind == "symmetric":
            return -r - 1 if r < 0 else 2 * n - 1 - r
        if kind == "circular":
            return n + r if r < 0 else r - n
        raise ValueError(kind)
    return f


def padding_program(n0, n1, h, kind0, kind1):
    """8 ghost boxes of one block; each axis is 'zero', 'symmetric' or 'circular'."""
    ranges = {0: [(-h, 0), (0, n0), (n0, n0 + h)], 1: [(-h, 0), (0, n1), (n1, n1 + h)]}
    f0 = fmap_1d(kind0, n0) if kind0 != "zero" else None
    f1 = fmap_1d(kind1, n1) if kind1 != "zero" else None
    subs = []
    for a, ra in enumerate(ranges[0]):
        for b, rb in enumerate(ranges[1]):
            if a == 1 and b == 1:
                continue
            box = [(0, 1), ra, rb]
            zero = (a != 1 and f0 is None) or (b != 1 and f1 is None)
            if zero:
                subs.append(ZeroSub(box))
            else:
                subs.append(MapSub(box, lambda c, f0=f0, f1=f1: (0, f0(c[1]) if f0 else c[1], f1(c[2]) if f1 else c[2])))
    return subs


def full_field(g, data2d, ghost_fill=np.nan):
    u = np.full((g.ncells, 1), ghost_fill)
    u[g.data_cells, 0] = data2d.reshape(-1)
    return u


NP_MODE = {"zero": "constant", "symmetric": "symmetric", "circular": "wrap"}


@pytest.mark.parametrize("kind0,kind1", [
    ("zero", "zero"), ("symmetric", "symmetric"), ("circular", "circular"),
    ("zero", "circular"), ("symmetric", "zero"), ("circular", "symmetric"),
])
@pytest.mark.parametrize("n0,n1,h", [(5, 7, 1), (6, 4, 3), (9, 9, 2)])
def test_padding_matches_numpy_pad(kind0, kind1, n0, n1, h):
    g = one_block(n0, n1, h)
    data = np.random.default_rng(0).standard_normal((n0, n1))
    op = assemble(g, padding_program(n0, n1, h, kind0, kind1))
    out = apply(op, full_field(g, data))[:, 0].reshape(n0 + 2 * h, n1 + 2 * h)
    ref = np.pad(data, ((0, 0), (h, h)), mode=NP_MODE[kind1])
    ref = np.pad(ref, ((h, h), (0, 0)), mode=NP_MODE[kind0])
    assert np.array_equal(out, ref)
    # copy rows are exact permutation rows; zero rows are empty
    A = op.dense()
    assert set(np.unique(A)) <= {0.0, 1.0}
    assert (A.sum(axis=1) <= 1).all()


def test_alg1_worked_example():
    fx = json.load(open(os.path.join(HERE, "golden", "alg1_example.json")))
    g = Grid([0, -1, -1], [3, 6, 6])
    for i in range(3):
        g.add_block([(i, i + 1), (-1, 6), (-1, 6)], [(i, i + 1), (0, 5), (0, 5)])
    assert g.ncells == 3 * fx["full_cells_per_block"]
    assert g.ndata == 3 * fx["data_cells_per_block"]
    right = [tuple(r) for r in fx["right_ghost_block1"]]
    left = [tuple(r) for r in fx["left_ghost_block1"]]
    rmap = MapSub(right, lambda c: (2, 9 - c[2], c[1]), 1.0)
    for row, col in fx["derived_right_map_entries"]:
        assert rmap.fmap(tuple(row)) == tuple(col)
    # left ghost: a CSR sub-matrix reading block 0 (values chosen here: 2-point averages)
    ptr = np.arange(0, 11, 2)
    cols = [(0, r, c) for r in range(5) for c in (3, 4)]
    vals = np.full(10, 0.5)
    lsub = RowsSub(left, lambda c: [(cols[k], vals[k]) for k in range(ptr[c[1]], ptr[c[1] + 1])])
    # zero = full minus data minus left minus right, split into boxes (top/bottom rows with corners)
    zeros = [ZeroSub([(1, 2), (-1, 0), (-1, 6)]), ZeroSub([(1, 2), (5, 6), (-1, 6)])]
    op = assemble(g, [rmap, lsub] + zeros)
    assert int(op.covered.sum()) == 49 - 25
    nz_rows = sum(int(np.prod([b - a for a, b in z.rows])) for z in zeros)
    assert nz_rows == fx["zero_rows_block1"]
    rng = np.random.default_rng(1)
    u = rng.standard_normal((g.ncells, 1))
    out = apply(op, u)
    for r in range(5):
        assert out[g.cell((1, r, 5)), 0] == u[g.cell((2, 4, r)), 0]
        assert out[g.cell((1, r, -1)), 0] == pytest.approx(0.5 * (u[g.cell((0, r, 3)), 0] + u[g.cell((0, r, 4)), 0]), rel=1e-15)
    for z in zeros:
        for c in oracle.grid.box_coords(z.rows):
            v = out[g.cell(tuple(c)), 0]
            assert v == 0.0 and not np.signbit(v)
    # blocks 0 and 2 have no sub-matrices: their ghosts are untouched
    for b in (0, 2):
        cells = g.cells_of_box(b, g.blocks[b].full)
        assert np.array_equal(out[cells], u[cells])


def test_overlap_rejected_and_summed():
    g = one_block(4, 4, 1)
    a = MapSub([(0, 1), (-1, 0), (0, 4)], lambda c: (0, 0, c[2]), 1.0)
    b = MapSub([(0, 1), (-1, 0), (2, 4)], lambda c: (0, 1, c[2]), 2.0)
    with pytest.raises(ValueError):
        assemble(g, [a, b])
    op = assemble(g, [a, b], allow_overlap_sum=True)
    u = np.random.default_rng(2).standard_normal((g.ncells, 1))
    out = apply(op, u)
    for x in range(4):
        want = u[g.cell((0, 0, x)), 0] + (2.0 * u[g.cell((0, 1, x)), 0] if x >= 2 else 0.0)
        assert out[g.cell((0, -1, x)), 0] == want


def test_subvector_and_uncovered_rows():
    g = one_block(4, 5, 2)
    rows = [(0, 1), (-2, 0), (0, 5)]
    vals = np.arange(10, dtype=float).reshape(10, 1) + 0.25
    op = assemble(g, [VectorSub(rows, vals), MapSub(rows, lambda c: (0, -c[1] - 1, c[2]))])
    u = np.random.default_rng(3).standard_normal((g.ncells, 1))
    out = apply(op, u)
    k = 0
    for y in range(-2, 0):
        for x in range(5):
            assert out[g.cell((0, y, x)), 0] == u[g.cell((0, -y - 1, x)), 0] + vals[k, 0]
            k += 1
    covered = g.ghost_cells[op.covered]
    rest = np.setdiff1d(g.ghost_cells, covered)
    assert np.array_equal(out[rest], u[rest]) and rest.size == g.nghost - 10
    with pytest.raises(ValueError):
        assemble(g, [MapSub([(0, 1), (0, 1), (0, 1)], lambda c: c)])  # data row
    with pytest.raises(ValueError):
        assemble(g, [MapSub([(0, 1), (-1, 0), (0, 1)], lambda c: (0, -1, 0))])  # ghost column


def test_vjp_dot_product_identity():
    """<F(u) - F(0), w> = <u, F*(w)> for the full-field map, with vector slots."""
    from oracle import cubed_sphere as cs
    N, h, I = 6, 2, 5
    vec = (1, 2, 2)  # u slots {1, 2}, v slots {3, 4}
    g = cs.grid(N, h)
    subs = cs.subs(N, h, "lagrange", vector=True)
    rng = np.random.default_rng(4)
    rows = cs.side_box(0, cs.LEFT, N, h)
    nrow = N * h
    subs.append(VectorSub(rows, rng.standard_normal((nrow, I))))
    op = assemble(g, subs)
    u = rng.standard_normal((g.ncells, I))
    w = rng.standard_normal((g.ncells, I))
    Fu = apply(op, u, vec) - apply(op, np.zeros_like(u), vec)
    lhs = float(np.sum(Fu * w))
    rhs = float(np.sum(u * vjp(op, w, vec)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_magnitude_operator_drops_rotation_signs():
    """The bound helper of the GPU tests: for a negated copy with a component
    rotation that flips a sign, plus b, applying it to |u| gives
    |w| |u[mapped cell, permuted slot]| + |b| per value (no cancellation
    between the negated part and b)."""
    from helpers import magnitude_operator
    g = Grid([0, -1], [1, 4])
    g.add_block([(0, 1), (-1, 4)], [(0, 1), (0, 3)])
    rows = [(0, 1), (-1, 0)]
    rot = (0, -1, 1, 0)  # slot pairs swapped, one of them negated
    b = np.array([[0.5, -0.25, 2.0, -1.0]])
    op = assemble(g, [MapSub(rows, lambda c: (c[0], 2), weight=-3.0, rot=rot), VectorSub(rows, b)])
    vec = (0, 2, 2)  # components at slots {0, 1} and {2, 3}
    u = np.arange(1.0, 21.0).reshape(5, 4) * np.array([1, -1, 1, -1])
    mag = apply(magnitude_operator(op), np.abs(u), vec)
    src = np.abs(u[3])  # cell (0, 2): the mapped data cell
    want = 3.0 * src[[2, 3, 0, 1]] + np.abs(b[0])
    assert np.array_equal(mag[0], want)
    val = apply(op, u, vec)[0]
    assert (np.abs(val) <= mag[0]).all()
