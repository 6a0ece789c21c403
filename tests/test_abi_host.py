"""C-ABI library checks that need no GPU (plans compiled host-only).

* the library loads and exports every function ``include/hbc.h`` declares;
* the plan compiler's rows equal the oracle's A on tiny grids (cubed-sphere
  copy and Lagrange programs, the HPCG halo program, padding maps);
* validation errors: rows outside the ghost region, columns outside the
  data region, overlaps, strict cover, bad slices, bad rotations;
* segment / row counts of the workload programs.
"""
import os
import re

import numpy as np
import pytest

import paper_2605_14780_amd as hb
from helpers import closed_form_weights
from oracle import assemble
from oracle import cubed_sphere as ocs
from oracle import hpcg as ohpcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hbc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hbc_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = hb.lib()
    names = declared_functions()
    assert len(names) >= 40
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(hb.SIGNATURES), set(names) ^ set(hb.SIGNATURES)


def compare_plan_with_oracle(plan, og, op, tol=0.0):
    A = op.dense()
    for r, cell in enumerate(og.ghost_cells):
        kind, cols, vals, b, rot = plan.row(int(cell))
        nz = np.nonzero(A[r])[0]
        ref = {int(og.data_cells[j]): A[r, j] for j in nz}
        got = {c: v for c, v in zip(cols, vals) if v != 0.0}
        assert set(got) == set(ref), (cell, got, ref)
        for c in ref:
            assert abs(got[c] - ref[c]) <= tol, (cell, c, got[c], ref[c])


@pytest.mark.parametrize("N,h", [(4, 1), (4, 2), (6, 3), (13, 3), (24, 2), (5, 2), (8, 4)])
def test_cs_sync_plan_equals_oracle(N, h):
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add(N, h, hb.CS_SYNC, vector=True)
    plan = hb.Plan(p, inner=1, host_only=True)
    og = ocs.grid(N, h)
    compare_plan_with_oracle(plan, og, assemble(og, ocs.subs(N, h, "sync")))
    # component rotation per side equals the oracle's finite-difference rotation
    for f in range(6):
        for side in range(4):
            box = ocs.side_box(f, side, N, h)
            c = og.cell((f, box[1][0], box[2][0]))
            rot = plan.row(c)[4]
            R = ocs.rside(f, side)
            sw = R[0, 0] == 0
            code = int(sw) | ((R[0, 1 if sw else 0] < 0) << 1) | ((R[1, 0 if sw else 1] < 0) << 2)
            assert rot == code, (f, side, rot, R)


@pytest.mark.parametrize("N,h", [(4, 1), (4, 2), (6, 3), (13, 3), (24, 2), (5, 2), (8, 4)])
def test_cs_lagrange_plan_equals_oracle(N, h):
    base, w = closed_form_weights(N, h)
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add(N, h, hb.CS_LAGRANGE, vector=False, base=base, w=w)
    plan = hb.Plan(p, inner=1, host_only=True)
    st = plan.stats()
    assert st["rows_ell"] == 24 * h * N and st["rows_zero"] == 24 * h * h and st["nnz"] == 4 * 24 * h * N
    og = ocs.grid(N, h)
    compare_plan_with_oracle(plan, og, assemble(og, ocs.subs(N, h, "lagrange")), tol=64 * N * 2.0 ** -53)


@pytest.mark.parametrize("nb,n", [(2, 4), (1, 5), (3, 3)])
def test_hpcg_plan_equals_oracle(nb, n):
    g = hb.Grid.cartesian([nb] * 3, [n] * 3, 1)
    p = hb.Program(g)
    p.cart_add_halo([nb] * 3, [n] * 3, 1)
    plan = hb.Plan(p, inner=1, host_only=True)
    og = ohpcg.grid(nb, n)
    compare_plan_with_oracle(plan, og, assemble(og, ohpcg.subs(nb, n)))


def test_workload_program_sizes():
    # cubed sphere C384, halo 3: 24 Lagrange strips + 24 corners
    N, h = 384, 3
    base, w = closed_form_weights(N, h)
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add(N, h, hb.CS_LAGRANGE, True, base, w)
    st = hb.Plan(p, inner=256, vec=(128, 64, 64), host_only=True).stats()
    assert st["segments"] == 48 and st["rows_ell"] == 27648 and st["nnz"] == 110592
    assert st["rows_zero"] == 216 and st["ghost_values"] == 7133184
    assert st["unique_sources"] == 6 * (4 * h * N - 4 * h * h)
    # HPCG-shaped: 2x2x2 blocks of 128^3, halo 1
    g = hb.Grid.cartesian([2] * 3, [128] * 3, 1)
    p = hb.Program(g)
    p.cart_add_halo([2] * 3, [128] * 3, 1)
    st = hb.Plan(p, inner=1, host_only=True).stats()
    assert st["segments"] == 208 and st["rows_map"] == 396296 and st["rows_zero"] == 402488
    assert st["unique_sources"] == 390152


def one_block(n0, n1, h):
    g = hb.Grid([0, -h, -h], [1, n0 + h, n1 + h])
    g.add_block([(0, 1), (-h, n0 + h), (-h, n1 + h)], [(0, 1), (0, n0), (0, n1)])
    return g


def test_validation_errors():
    g = one_block(4, 4, 1)
    I3 = np.eye(3, dtype=np.int64)
    p = hb.Program(g)
    p.add_map([(0, 1), (0, 1), (0, 4)], I3, [0, 0, 0])  # data rows
    with pytest.raises(hb.HbcError) as e:
        hb.Plan(p, host_only=True)
    assert e.value.code == hb.ERANGE
    p = hb.Program(g)
    p.add_map([(0, 1), (-1, 0), (0, 4)], I3, [0, 0, 0])  # copies a ghost
    with pytest.raises(hb.HbcError) as e:
        hb.Plan(p, host_only=True)
    assert e.value.code == hb.ERANGE
    p = hb.Program(g)
    p.add_zero([(0, 1), (-1, 0), (0, 4)])
    p.add_zero([(0, 1), (-1, 0), (3, 5)])
    with pytest.raises(hb.HbcError) as e:
        hb.Plan(p, host_only=True)
    assert e.value.code == hb.EOVERLAP
    p = hb.Program(g)
    p.add_zero([(0, 1), (-1, 0), (0, 4)])
    p.set_flags(hb.STRICT_COVER)
    with pytest.raises(hb.HbcError) as e:
        hb.Plan(p, host_only=True)
    assert e.value.code == hb.EUNCOVERED
    p = hb.Program(g)
    with pytest.raises(hb.HbcError):
        p.add_map([(0, 1), (-1, 0), (0, 4)], I3, [0, 0, 0], rot=[[1, 1], [0, 1]])
    p = hb.Program(g)
    p.add_ell([(0, 1), (-1, 0), (0, 1)], 2, [7, 10 ** 6], [0.5, 0.5])
    with pytest.raises(hb.HbcError) as e:
        hb.Plan(p, host_only=True)
    assert e.value.code == hb.ERANGE
    with pytest.raises(hb.HbcError) as e:
        g.add_block([(0, 1), (0, 2, 2), (0, 2)], [(0, 1), (0, 2, 2), (0, 2)])
    gg = hb.Grid([0], [10])
    gg.add_block([(0, 5)], [(1, 4)])
    with pytest.raises(hb.HbcError):
        gg.add_block([(4, 8)], [(5, 7)])  # overlaps the first block


def test_zero_rest_partition_covers_ghost_ring():
    g = one_block(5, 5, 2)
    p = hb.Program(g)
    p.add_map([(0, 1), (0, 5), (5, 7)], np.diag([1, 1, -1]), [0, 0, 9])
    p.add_zero_rest(0)
    p.set_flags(hb.STRICT_COVER)
    st = hb.Plan(p, host_only=True).stats()
    assert st["rows_uncovered"] == 0
    assert st["rows_map"] == 10 and st["rows_zero"] == 81 - 25 - 10


# ---- data rows: block-edge averaging -------------------------------------------------------
@pytest.mark.parametrize("Np,h", [(4, 1), (6, 2), (11, 3)])
def test_edge_average_plan_equals_oracle(Np, h):
    from oracle import averaging as oav
    g = hb.Grid.cubed_sphere(Np, h)
    p = hb.Program(g)
    p.cs_add_edge_average(Np)
    plan = hb.Plan(p, inner=3, host_only=True)
    st = plan.stats()
    assert st["rows_data"] == 24 * Np - 24
    og = ocs.grid(Np, h)
    dop = oav.assemble_data(og, oav.edge_average_subs(Np))
    S = dop.S.toarray()
    for r in np.nonzero(dop.rows)[0]:
        cell = int(og.data_cells[r])
        kind, cols, vals, b, rot = plan.row(cell)
        assert kind == hb.SEG_DATA_ROW
        ref = {int(og.data_cells[j]): S[r, j] for j in np.nonzero(S[r])[0]}
        assert dict(zip(cols, vals)) == ref, (cell, cols, vals, ref)
    # interior points are no rows
    inner = og.data_cells[~dop.rows][0]
    assert plan.row(int(inner))[0] == -1


def test_data_rows_validation():
    Np, h = 5, 1
    g = hb.Grid.cubed_sphere(Np, h)
    W = Np + 2 * h

    def lin(f, j, i):
        return (f * W + (j + h)) * W + (i + h)

    p = hb.Program(g)
    p.add_data_csr([(0, 1), (0, 1), (0, 2)], [0, 1, 2], [lin(0, 1, 1), lin(0, 1, 1)], [1.0, 1.0])
    p.add_data_csr([(0, 1), (0, 1), (1, 3)], [0, 1, 2], [lin(0, 1, 1), lin(0, 1, 1)], [1.0, 1.0])
    with pytest.raises(hb.HbcError) as e:
        hb.Plan(p, inner=1, host_only=True)
    assert e.value.code == hb.EOVERLAP
    p = hb.Program(g)
    p.add_data_csr([(0, 1), (-1, 0), (0, 1)], [0, 1], [lin(0, 1, 1)], [1.0])  # a ghost row
    with pytest.raises(hb.HbcError) as e:
        hb.Plan(p, inner=1, host_only=True)
    assert e.value.code == hb.ERANGE
    p = hb.Program(g)
    p.add_data_csr([(0, 1), (0, 1), (0, 1)], [0, 1], [lin(0, -1, 0)], [1.0])  # a ghost column
    with pytest.raises(hb.HbcError) as e:
        hb.Plan(p, inner=1, host_only=True)
    assert e.value.code == hb.ERANGE
    p = hb.Program(g)
    p.cs_add_edge_average(Np)
    with pytest.raises(hb.HbcError) as e:
        hb.Plan(p, inner=2, order=hb.PLANE_MAJOR, host_only=True)
    assert e.value.code == hb.EUNSUPPORTED
    with pytest.raises(hb.HbcError) as e:
        hb.Program(hb.Grid.cubed_sphere(Np + 1, h)).cs_add_edge_average(Np)
    assert e.value.code == hb.EINVAL


# ---- consumer footprint ------------------------------------------------------------------
@pytest.mark.parametrize("N,h,r,mode", [(8, 3, 1, "sync"), (9, 3, 2, "lagrange"), (6, 2, 2, "sync")])
def test_consumer_footprint_plan_equals_oracle(N, h, r, mode):
    from oracle import footprint as ofp
    offs = [(0, 0, 0)] + [o for k in range(1, r + 1) for o in ((0, k, 0), (0, -k, 0), (0, 0, k), (0, 0, -k))]
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    if mode == "sync":
        p.cs_add(N, h, hb.CS_SYNC)
    else:
        base, w = closed_form_weights(N, h)
        p.cs_add(N, h, hb.CS_LAGRANGE, False, base, w)
    p.set_consumer(offs)
    plan = hb.Plan(p, inner=1, host_only=True)
    st = plan.stats()
    og = ocs.grid(N, h)
    live = ofp.live_ghost_mask(og, offs)
    assert st["ghost_cells_live"] == live.sum() == 6 * 4 * r * N
    assert st["rows_covered"] == live.sum()
    assert st["rows_dead"] == 6 * (4 * h * N + 4 * h * h) - live.sum()
    A = assemble(og, ocs.subs(N, h, mode)).dense()
    for row, cell in enumerate(og.ghost_cells):
        kind, cols, vals, b, rot = plan.row(int(cell))
        assert (kind >= 0) == bool(live[row]), cell
        if not live[row]:
            continue
        ref = {int(og.data_cells[j]): A[row, j] for j in np.nonzero(A[row])[0]}
        got = {c: v for c, v in zip(cols, vals) if v != 0.0}
        assert set(got) == set(ref), (cell, got, ref)
        assert max(abs(got[c] - ref[c]) for c in ref) <= 1e-13
    # strict cover asks only for the live ghosts
    p.set_flags(hb.STRICT_COVER)
    hb.Plan(p, inner=1, host_only=True)
    p.set_consumer([])
    assert hb.Plan(p, inner=1, host_only=True).stats()["rows_dead"] == 0


# ---- wide rows: quadrature of tensor-product reconstructions --------------------------------
@pytest.mark.parametrize("N,h,q", [(8, 2, 2), (12, 3, 2), (9, 1, 3), (6, 2, 1)])
def test_quadrature_plan_equals_oracle(N, h, q):
    from oracle import quadrature as oq
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add_quadrature(N, h, q)
    plan = hb.Plan(p, inner=1, host_only=True)
    og = ocs.grid(N, h)
    st = plan.stats()
    assert st["rows_csr"] == 24 * h * N and st["rows_zero"] == 24 * h * h
    compare_plan_with_oracle(plan, og, assemble(og, oq.subs(N, h, q)), tol=1e-13)


@pytest.mark.parametrize("inner,dtype,order,wide", [(16, "f64", hb.POINT_MAJOR, True), (8, "f64", hb.POINT_MAJOR, False),
                                                   (32, "f32", hb.POINT_MAJOR, True), (16, "f32", hb.POINT_MAJOR, False),
                                                   (64, "f64", hb.PLANE_MAJOR, False)])
def test_wide_row_selection(inner, dtype, order, wide):
    """Rows of >= 128 bytes in point-major plans go to the LDS-staged kernel;
    every CSR row is served exactly once (tiles hold at most 32 rows, so the
    24 halo strips of h * N rows need at least ceil(h * N / 32) tiles each)."""
    N, h = 20, 3
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add_quadrature(N, h, 2)
    dt = hb.F64 if dtype == "f64" else hb.F32
    st = hb.Plan(p, inner=inner, dtype=dt, order=order, host_only=True).stats()
    if wide:
        assert st["rows_wide"] == st["rows_csr"] == 24 * h * N
        assert st["wide_tiles"] >= 24 * -(-h * N // 32)
    else:
        assert st["rows_wide"] == 0 and st["wide_tiles"] == 0
    assert st["rows_narrow"] == 0


@pytest.mark.parametrize("inner,dtype,order,narrow", [(3, "f64", hb.POINT_MAJOR, True), (4, "f64", hb.POINT_MAJOR, False),
                                                     (7, "f32", hb.POINT_MAJOR, True), (8, "f32", hb.POINT_MAJOR, False),
                                                     (1, "f64", hb.PLANE_MAJOR, False)])
def test_narrow_row_selection(inner, dtype, order, narrow):
    """CSR rows of >= 8 entries and < 32 bytes in point-major plans go to the
    entry-splitting kernel; everything else stays on the other paths."""
    N, h = 12, 2
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add_quadrature(N, h, 2)
    dt = hb.F64 if dtype == "f64" else hb.F32
    st = hb.Plan(p, inner=inner, dtype=dt, order=order, host_only=True).stats()
    assert st["rows_narrow"] == (st["rows_csr"] if narrow else 0)
    assert st["rows_wide"] == 0


@pytest.mark.parametrize("inner,dtype,order,with_b,windowed", [
    (32, "f64", hb.POINT_MAJOR, False, True),    # 256-byte rows: windows
    (64, "f32", hb.POINT_MAJOR, False, True),
    (16, "f64", hb.POINT_MAJOR, False, False),   # 128 bytes: the row kernel
    (32, "f64", hb.POINT_MAJOR, True, False),    # b on every strip: windows from 512 bytes only
    (64, "f64", hb.POINT_MAJOR, True, True),
    (64, "f64", hb.PLANE_MAJOR, False, False),
])
def test_window_row_selection(inner, dtype, order, with_b, windowed):
    """Interpolation rows of the face-edge strips take the window kernel in
    point-major plans of >= 256-byte rows (>= 512 with b values).  The
    default launch shape follows: runs of WIN_DEFAULT_ROWS rows where windows
    are taken, else the row kernel's own tile (a plan whose window-shaped rows
    all fall under the b threshold keeps the row tiles of a plan built
    without windows)."""
    N, h = 24, 3
    base, w = closed_form_weights(N, h)
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add(N, h, hb.CS_LAGRANGE, vector=False, base=base, w=w)
    if with_b:
        for f in range(6):
            for side in (ocs.LEFT, ocs.RIGHT, ocs.BOTTOM, ocs.TOP):
                p.add_vector(ocs.side_box(f, side, N, h), np.full((N * h, 1), 0.25), ninner=1)
    dt = hb.F64 if dtype == "f64" else hb.F32
    plan = hb.Plan(p, inner=inner, dtype=dt, order=order, host_only=True)
    st = plan.stats()
    ref = hb.Plan(p, inner=inner, dtype=dt, order=order, host_only=True, windows=False)
    assert ref.stats()["rows_window"] == 0
    if windowed:
        assert st["rows_window"] == st["rows_ell"] == 24 * h * N
        assert st["window_runs"] >= 24 * h * -(-N // 8)
        assert plan.tune["rows_per_tile"] == 8
    else:
        assert st["rows_window"] == 0 and st["window_runs"] == 0
        assert plan.tune == ref.tune


def test_smoke_entry_is_importable_and_shapes_consistent():
    """smoke() needs a GPU; here only its module imports and its field layout
    matches the oracle grid (cells face by face, inner trailing)."""
    import __graft_entry__ as ge
    assert callable(ge.smoke) and callable(ge.build)
    og = ocs.grid(12, 3)
    assert og.ncells == 6 * 18 * 18


# ---- stepped slices (staggered variables, multigrid levels) ----------------------------
def _stepped_programs(nx=5, ny=4):
    from oracle import MapSub as OMap, RowsSub as ORows, ZeroSub as OZero, VectorSub as OVec
    from oracle.grid import Grid as OGrid
    lo, hi = [-2, -1], [2 * nx + 2, ny + 1]
    full, data = [(-2, 2 * nx + 2, 2), (-1, ny + 1, 1)], [(0, 2 * nx, 2), (0, ny, 1)]
    g = hb.Grid(lo, hi)
    g.add_block(full, data)
    p = hb.Program(g)
    og = OGrid(lo, hi)
    og.add_block(full, data)
    W = hi[1] - lo[1]

    def lin(x, y):  # row-major linear index over the global box of positions
        return (x - lo[0]) * W + (y - lo[1])

    p.add_map([(-2, 0), (0, ny)], np.eye(2, dtype=np.int64), [2 * nx, 0])
    p.add_map([(2 * nx, 2 * nx + 2), (0, ny)], np.eye(2, dtype=np.int64), [-2 * nx, 0], weight=-0.5)
    xs = list(range(0, 2 * nx, 2))
    p.add_csr([(0, 2 * nx), (-1, 0)], np.arange(0, 2 * len(xs) + 1, 2),
              [c for x in xs for c in (lin(x, 0), lin(x, 1))], [0.75, 0.25] * len(xs))
    p.add_zero([(0, 2 * nx), (ny, ny + 1)])
    bvals = 0.125 * (1.0 + np.arange(len(xs)))
    p.add_vector([(0, 2 * nx), (ny, ny + 1)], bvals)
    subs = [OMap([(-2, 0), (0, ny)], lambda c: (c[0] + 2 * nx, c[1])),
            OMap([(2 * nx, 2 * nx + 2), (0, ny)], lambda c: (c[0] - 2 * nx, c[1]), -0.5),
            ORows([(0, 2 * nx), (-1, 0)], lambda c: [((c[0], 0), 0.75), ((c[0], 1), 0.25)]),
            OZero([(0, 2 * nx), (ny, ny + 1)]),
            OVec([(0, 2 * nx), (ny, ny + 1)], bvals)]
    return g, p, og, subs


def test_stepped_grid_plan_equals_oracle():
    g, p, og, subs = _stepped_programs()
    assert g.cells == og.ncells
    plan = hb.Plan(p, inner=1, host_only=True)
    op = assemble(og, subs)
    compare_plan_with_oracle(plan, og, op)
    st = plan.stats()
    assert st["rows_covered"] == int(op.covered.sum())
    # b of the top rows
    for r, cell in enumerate(og.ghost_cells):
        if op.has_b[r]:
            assert plan.row(int(cell))[3] == op.b[r, 0]


def test_stepped_grid_errors():
    g = hb.Grid([0, 0], [16, 8])
    g.add_block([(0, 8, 2), (0, 8, 1)], [(2, 6, 2), (1, 7, 1)])
    with pytest.raises(hb.HbcError) as e:  # a second block on another lattice
        g.add_block([(9, 16, 2), (0, 8, 1)], [(11, 15, 2), (1, 7, 1)])
    assert e.value.code == hb.EUNSUPPORTED
    p = hb.Program(g)
    with pytest.raises(hb.HbcError) as e:  # a column between the lattice points
        p.add_csr([(0, 1), (0, 1)], [0, 1], [3 * 8 + 1], [1.0])
    assert e.value.code == hb.ERANGE
    with pytest.raises(hb.HbcError) as e:  # a map that leaves the lattice
        p.add_map([(0, 1), (0, 8)], np.eye(2, dtype=np.int64), [1, 0])
    assert e.value.code == hb.EINVAL
    with pytest.raises(hb.HbcError) as e:  # consumer offsets must be whole steps
        p.set_consumer([[1, 0]])
    assert e.value.code == hb.EINVAL
    p.set_consumer([[2, 0], [-2, 0], [0, 1], [0, -1]])


def test_cell_count_limit():
    """Cell numbers are 32-bit on the device: a grid of 2^31 - 2 cells
    compiles (host work is per row, not per cell), one more cell is refused."""
    n = (1 << 31) - 2
    g = hb.Grid([-1], [n - 1])
    g.add_block([(-1, n - 1)], [(0, n - 2)])
    p = hb.Program(g)
    p.add_zero([(-1, 0)])
    p.add_map([(n - 2, n - 1)], [[1]], [-1])
    plan = hb.Plan(p, inner=1, host_only=True)
    assert g.cells == n and plan.stats()["rows_covered"] == 2
    g2 = hb.Grid([-1], [n])
    g2.add_block([(-1, n)], [(0, n - 1)])
    p2 = hb.Program(g2)
    p2.add_zero([(-1, 0)])
    with pytest.raises(hb.HbcError) as e:
        hb.Plan(p2, inner=1, host_only=True)
    assert e.value.code == hb.EUNSUPPORTED


def test_rejected_first_block_leaves_the_grid_unchanged():
    g = hb.Grid([0, 0], [16, 8])
    with pytest.raises(hb.HbcError):  # data outside full: rejected
        g.add_block([(0, 8, 2), (0, 8, 1)], [(2, 10, 2), (1, 7, 1)])
    assert g.cells == 0
    g.add_block([(0, 16, 1), (0, 8, 1)], [(1, 15, 1), (1, 7, 1)])  # another lattice is still possible
    assert g.cells == 16 * 8


@pytest.mark.parametrize("N,h", [(5, 3), (8, 5), (8, 8)])
def test_cubed_sphere_halo_limited_to_half_a_face(N, h):
    """Ghost layer k sits at angle pi/4 + (k + 1/2) pi/(2N) in its face's frame;
    from k = N/2 on it passes pi/2 and leaves the face's gnomonic chart, so
    every cubed-sphere entry point refuses h > N/2."""
    import math
    assert math.pi / 4 + (h - 0.5) * math.pi / (2 * N) > math.pi / 2 - 1e-12
    with pytest.raises(hb.HbcError) as e:
        hb.Grid.cubed_sphere(N, h)
    assert e.value.code == hb.EINVAL
    g = hb.Grid.cubed_sphere(N, N // 2)
    p = hb.Program(g)
    with pytest.raises(hb.HbcError):
        p.cs_add(N, h, hb.CS_SYNC)
    with pytest.raises(hb.HbcError):
        p.cs_add_quadrature(N, h, 2)


def _set_vector_program(b1, b2, b3, I):
    """One 4^3 block, halo 1: zero halo rows, a b of width I on the z = -1
    face, a b of width 1 on part of it (summed), a b of width I on z = 4."""
    g = hb.Grid.cartesian([1, 1, 1], [4, 4, 4], 1)
    p = hb.Program(g)
    p.set_flags(hb.ALLOW_OVERLAP_SUM)
    p.cart_add_halo([1, 1, 1], [4, 4, 4], 1)
    s1 = p.add_vector([(0, 1), (-1, 0), (0, 4), (0, 4)], b1, ninner=I)
    s2 = p.add_vector([(0, 1), (-1, 0), (1, 3), (0, 4)], b2, ninner=1)
    s3 = p.add_vector([(0, 1), (4, 5), (0, 4), (0, 4)], b3, ninner=I)
    return g, p, (s1, s2, s3)


@pytest.mark.parametrize("order", [hb.POINT_MAJOR, hb.PLANE_MAJOR])
def test_set_vector_gives_the_b_of_a_plan_built_with_the_new_values(order):
    """Sec. III-B (b of F): new values for sub-vectors of a compiled plan give,
    row by row and slot by slot, the b a plan compiled from those values has
    (sums over overlapping sub-vectors included); matrix rows are unchanged."""
    I = 3
    rng = np.random.default_rng(21)
    b1, b2, b3 = rng.standard_normal((16, I)), rng.standard_normal(8), rng.standard_normal((16, I))
    n2, n3 = rng.standard_normal(8), rng.standard_normal((16, I))
    g, p, (s1, s2, s3) = _set_vector_program(b1, b2, b3, I)
    plan = hb.Plan(p, inner=I, order=order, host_only=True)
    plan.set_vector(s2, n2)
    plan.set_vector(s3, n3)
    _, pf, _ = _set_vector_program(b1, n2, n3, I)
    fresh = hb.Plan(pf, inner=I, order=order, host_only=True)
    _, po, _ = _set_vector_program(b1, b2, b3, I)
    old = hb.Plan(po, inner=I, order=order, host_only=True)
    changed = 0
    for cell in range(g.cells):
        for l in range(I):
            got, want, before = plan.row(cell, l), fresh.row(cell, l), old.row(cell, l)
            assert got == want, (cell, l)
            changed += got[3] != before[3]
    assert changed == (8 + 16) * I  # the rows of s2 and s3, every slot
    with pytest.raises(hb.HbcError, match="not a sub-vector"):
        plan.set_vector(0, n2)  # a halo sub-matrix
    with pytest.raises(hb.HbcError, match="not a sub-vector"):
        plan.set_vector(s3 + 1, n2)


def test_set_vector_with_a_consumer_footprint():
    """A sub-vector over a whole halo strip of which the consumer footprint
    keeps one layer: new values reach the kept rows (as in a plan built with
    them) and the dropped rows stay uncovered; a sub-vector whose rows are all
    dropped takes new values without error."""
    N, h = 8, 3
    box = ocs.side_box(0, ocs.LEFT, N, h)  # the h layers of face 0's left strip
    outer_layer = [box[0], (-h, -h + 1), box[2]] if box[1][0] < 0 else [box[0], box[1], (-h, -h + 1)]
    rng = np.random.default_rng(4)
    b0, b1 = rng.standard_normal(h * N), rng.standard_normal(h * N)
    o0, o1 = rng.standard_normal(N), rng.standard_normal(N)
    offs = [(0, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]

    def build(bv, ov):
        g = hb.Grid.cubed_sphere(N, h)
        p = hb.Program(g)
        p.set_flags(hb.ALLOW_OVERLAP_SUM)
        p.cs_add(N, h, hb.CS_SYNC)
        s_strip = p.add_vector(box, bv)
        s_outer = p.add_vector(outer_layer, ov)
        p.set_consumer(offs)
        return g, hb.Plan(p, inner=1, host_only=True), s_strip, s_outer

    g, plan, s_strip, s_outer = build(b0, o0)
    plan.set_vector(s_strip, b1)
    plan.set_vector(s_outer, o1)  # every row of it is dropped
    _, fresh, _, _ = build(b1, o1)
    og = ocs.grid(N, h)
    kept = 0
    for cell in og.cells_of_box(0, box):
        got, want = plan.row(int(cell)), fresh.row(int(cell))
        assert got == want, cell
        kept += got[0] >= 0
    assert kept == N  # one layer of the strip
    assert all(plan.row(int(c))[0] == -1 for c in og.cells_of_box(0, outer_layer))


def test_binding_checks_host_array_lengths():
    """The binding refuses host arrays whose length does not match what the
    C ABI will read (it copies rows x width values from the pointer), before
    calling the library; the box row count comes from the library itself
    (lattice points on stepped grids)."""
    g = hb.Grid.cubed_sphere(8, 2)
    p = hb.Program(g)
    box = [(0, 1), (0, 8), (-2, 0)]
    assert p.box_rows(box) == 16
    with pytest.raises(ValueError):
        p.add_vector(box, np.zeros(15))
    with pytest.raises(ValueError):
        p.add_ell(box, 4, np.zeros(63, dtype=np.int64), np.zeros(64))
    with pytest.raises(ValueError):
        p.add_csr(box, np.zeros(16, dtype=np.int64), [], [])
    with pytest.raises(ValueError):
        p.add_map(box, np.eye(2, dtype=np.int64), [0, 0, 0])
    sid = p.add_vector(box, np.ones((16, 3)), ninner=3)
    p.add_zero_rest(0)
    plan = hb.Plan(p, inner=3, host_only=True)
    with pytest.raises(ValueError):
        plan.set_vector(sid, np.ones(47))
    with pytest.raises(hb.HbcError, match="not a sub-vector"):
        plan.set_vector(sid + 1, np.ones(48))
    plan.set_vector(sid, np.full(48, 2.0))
    # stepped slices: the box selects lattice points only
    gs = hb.Grid([0, 0], [1, 20])
    gs.add_block([(0, 1), (0, 20, 2)], [(0, 1), (4, 16, 2)])
    ps = hb.Program(gs)
    assert ps.box_rows([(0, 1), (0, 4)]) == 2


@pytest.mark.parametrize("N,h", [(6, 1), (12, 3), (20, 2)])
def test_consumer_compiled_on_a_host_only_plan(N, h):
    """A consumer of a host-only cubed-sphere Lagrange plan is compiled on the
    host (applies need a device plan).  Its composed boundary rows in closed
    form: the cells next to a face edge, 4N - 4 per face; for the cross, 8
    entries on an edge (4 data reads, one ghost's 4 Lagrange entries) and 11
    at a corner cell (two ghosts); for the 9-point box, 6 data reads plus 3
    ghosts on an edge (18), and at a corner 4 data reads, 4 edge ghosts and
    the zero corner ghost (20)."""
    base, w = closed_form_weights(N, h)
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add(N, h, hb.CS_LAGRANGE, vector=False, base=base, w=w)
    plan = hb.Plan(p, inner=4, host_only=True)
    cross = [(0, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    box9 = [(0, a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)]
    for offs, edge, corner in ((cross, 8, 11), (box9, 18, 20)):
        st = hb.Consumer(plan, offs, [1.0] * len(offs)).stats()
        assert st["boundary_rows"] == 6 * (4 * N - 4)
        assert st["boundary_entries"] == 6 * ((4 * N - 8) * edge + 4 * corner)
    c = hb.Consumer(plan, cross, [1.0] * 5)
    # an apply is refused (host-only plan) before any pointer is read
    assert hb.lib().hbc_consumer_apply(c._h, None, 0, None, 0, 1, None) == hb.EINVAL
