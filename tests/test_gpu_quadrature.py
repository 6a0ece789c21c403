"""GPU checks of wide rows (Sec. III-B Agg . Recons: 16..25 entries per row)
against the oracle: FP64 within the weights' agreement (1e-13 per entry,
pinned host-side) plus summation rounding; FP32 within a stated bound."""
import numpy as np
import pytest

from helpers import cs_full_field, gpu_available
from oracle import apply as o_apply, assemble
from oracle import cubed_sphere as ocs
from oracle import quadrature as oq

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_2605_14780_amd as hb


def wide_bounds(op, full, og, vec):
    """Per ghost value: sum of |x| over the row's entries, and sum |w x|, with
    the component rotation applied (a rotated slot takes the other component)."""
    from dataclasses import replace
    G = og.ghost_cells
    ax = np.nan_to_num(np.abs(full))
    op_pat = replace(op, parts={k: (abs(A) > 0).astype(np.float64) for k, A in op.parts.items()}, b=None)
    op_mag = replace(op, parts={k: abs(A) for k, A in op.parts.items()}, b=None)
    pat = np.abs(o_apply(op_pat, ax, vec))[G]
    mag = np.abs(o_apply(op_mag, ax, vec))[G]
    return pat, mag


@pytest.mark.parametrize("N,h,nf,nl,q,dtype", [(12, 3, 4, 2, 2, "f64"), (9, 2, 1, 5, 3, "f64"), (16, 2, 4, 1, 2, "f64"),
                                               (12, 3, 4, 4, 2, "f32")])
def test_quadrature_rows(N, h, nf, nl, q, dtype):
    I = nf * nl
    vec = (2 * nl, nl, nl) if nf == 4 else None
    dt = hb.F64 if dtype == "f64" else hb.F32
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add_quadrature(N, h, q, vector=vec is not None)
    plan = hb.Plan(p, inner=I, vec=vec, dtype=dt)
    full = cs_full_field(N, h, nf, nl, seed=N + q)
    t = torch.from_numpy(full.astype(np.float64 if dt == hb.F64 else np.float32)).cuda()
    hb.apply(plan, t)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.float64)
    og = ocs.grid(N, h)
    op = assemble(og, oq.subs(N, h, q, vector=vec is not None))
    ref = o_apply(op, full, vec)
    G = og.ghost_cells
    pat, mag = wide_bounds(op, full, og, vec)
    if dt == hb.F64:
        tol = 1e-13 * pat + 64 * 2.0 ** -53 * mag
    else:
        tol = 1e-13 * pat + 64 * 2.0 ** -24 * mag
    d = np.abs(got[G] - ref[G])
    assert (d <= tol).all(), float((d / np.maximum(tol, 1e-300)).max())
    corners = np.isin(G, np.concatenate([og.cells_of_box(f, b) for f in range(6) for b in ocs.corner_boxes(f, N, h)]))
    assert (got[G][corners] == 0).all()


@pytest.mark.parametrize("nl,dtype", [(8, "f64"), (16, "f32"), (12, "f64"), (6, "f64")])
def test_quadrature_rows_staged(nl, dtype):
    """Rows of >= 128 bytes take the LDS-staged wide-row kernel (several
    inner-value slices per tile, partial last slice for nl = 12; FP64 slices
    of 256 bytes for nl = 8 and 12, of 128 bytes for nl = 6, whose vector
    components are not 4-aligned)."""
    N, h, nf, q = 10, 3, 4, 2
    I = nf * nl
    vec = (2 * nl, nl, nl)
    dt = hb.F64 if dtype == "f64" else hb.F32
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add_quadrature(N, h, q, vector=True)
    rng = np.random.default_rng(nl)
    b = rng.standard_normal((N * h, I))
    p.add_vector(ocs.side_box(3, ocs.RIGHT, N, h), b, ninner=I)
    plan = hb.Plan(p, inner=I, vec=vec, dtype=dt)
    full = cs_full_field(N, h, nf, nl, seed=30 + nl)
    t = torch.from_numpy(full.astype(np.float64 if dt == hb.F64 else np.float32)).cuda()
    hb.apply(plan, t)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.float64)
    og = ocs.grid(N, h)
    from oracle import VectorSub
    op = assemble(og, oq.subs(N, h, q, vector=True) + [VectorSub(ocs.side_box(3, ocs.RIGHT, N, h), b)])
    ref = o_apply(op, full, vec)
    G = og.ghost_cells
    pat, mag = wide_bounds(op, full, og, vec)
    ulp = 2.0 ** -53 if dt == hb.F64 else 2.0 ** -24
    tol = 1e-13 * pat + 64 * ulp * (mag + np.abs(ref[G]))
    d = np.abs(got[G] - ref[G])
    assert (d <= tol).all(), float((d / np.maximum(tol, 1e-300)).max())
    # the adjoint through the same plan: dot-product identity
    y = torch.randn(g.cells, I, dtype=t.dtype, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    x = torch.from_numpy(np.nan_to_num(full, nan=0.0).astype(np.float64 if dt == hb.F64 else np.float32)).cuda()
    Ax, z, Aty = x.clone(), torch.zeros_like(x), y.clone()
    hb.apply(plan, Ax)
    hb.apply(plan, z)
    hb.apply_adjoint(plan, Aty)
    torch.cuda.synchronize()
    lhs = float(((Ax.double() - z.double()) * y.double()).sum())
    rhs = float((x.double() * Aty.double()).sum())
    assert abs(lhs - rhs) <= (1e-12 if dt == hb.F64 else 1e-5) * max(abs(lhs), abs(rhs))


@pytest.mark.parametrize("dtype,h,I", [("f64", 4, 64), ("f32", 3, 64), ("f64", 3, 24)])
def test_wide_kernel_matches_general_rows_bitwise(dtype, h, I):
    """The staged wide-row kernel (rows of >= 128 bytes: many tiles per side,
    every ghost layer of a position in one tile; FP64 slices of 256 bytes for
    64 inner values, of 128 bytes for 24) sums each row in the same order as
    the general row path (rows of 32 to 127 bytes): applying one program to I
    inner values, and to the same values 8 at a time, gives equal bits."""
    N, q = 20, 2
    dt, npdt = (hb.F64, np.float64) if dtype == "f64" else (hb.F32, np.float32)
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add_quadrature(N, h, q)
    wide = hb.Plan(p, inner=I, dtype=dt)
    narrow = hb.Plan(p, inner=8, dtype=dt)
    sw, sn = wide.stats(), narrow.stats()
    assert sw["rows_wide"] == sw["rows_csr"] and sw["wide_tiles"] > 24
    assert sn["rows_wide"] == 0 and sn["rows_narrow"] == 0
    full = cs_full_field(N, h, 1, I, seed=11 + h).astype(npdt)
    t = torch.from_numpy(full.copy()).cuda()
    hb.apply(wide, t)
    k = 8  # rows of 64 or 32 bytes: the general row path
    parts = []
    for c0 in range(0, I, k):
        s = torch.from_numpy(np.ascontiguousarray(full[:, c0:c0 + k])).cuda()
        hb.apply(narrow, s)
        parts.append(s)
    torch.cuda.synchronize()
    got_wide = t.cpu().numpy()
    got_narrow = torch.cat(parts, dim=1).cpu().numpy()
    assert np.array_equal(got_wide.view(np.uint64 if dt == hb.F64 else np.uint32),
                          got_narrow.view(np.uint64 if dt == hb.F64 else np.uint32))


@pytest.mark.parametrize("I,vector,dtype", [(3, True, "f64"), (1, False, "f64"), (7, False, "f32"),
                                            (3, True, "f32")])
def test_quadrature_rows_narrow(I, vector, dtype):
    """Rows of < 32 bytes (the shallow-water (h, u, v) case) take the kernel
    that splits a row's entries over 16 lanes and adds the partial sums by a
    butterfly: oracle parity with b on one side and the (u, v) rotation,
    determinism over repeated applies, and the adjoint's dot-product identity
    (its ghost reset goes through the same kernel)."""
    N, h, q = 14, 3, 2
    vec = (1, 1, 1) if vector else None
    dt, npdt = (hb.F64, np.float64) if dtype == "f64" else (hb.F32, np.float32)
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add_quadrature(N, h, q, vector=vector)
    rng = np.random.default_rng(I)
    b = rng.standard_normal((N * h, I))
    p.add_vector(ocs.side_box(2, ocs.TOP, N, h), b, ninner=I)
    plan = hb.Plan(p, inner=I, vec=vec, dtype=dt)
    st = plan.stats()
    assert st["rows_narrow"] == st["rows_csr"] == 24 * h * N and st["rows_wide"] == 0
    full = cs_full_field(N, h, I, 1, seed=50 + I)
    t = torch.from_numpy(full.astype(npdt)).cuda()
    hb.apply(plan, t)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.float64)
    og = ocs.grid(N, h)
    from oracle import VectorSub
    op = assemble(og, oq.subs(N, h, q, vector=vector) + [VectorSub(ocs.side_box(2, ocs.TOP, N, h), b)])
    ref = o_apply(op, full, vec)
    G = og.ghost_cells
    pat, mag = wide_bounds(op, full, og, vec)
    ulp = 2.0 ** -53 if dt == hb.F64 else 2.0 ** -24
    tol = 1e-13 * pat + 64 * ulp * (mag + np.abs(ref[G]))
    d = np.abs(got[G] - ref[G])
    assert (d <= tol).all(), float((d / np.maximum(tol, 1e-300)).max())
    corners = np.isin(G, np.concatenate([og.cells_of_box(f, bx) for f in range(6) for bx in ocs.corner_boxes(f, N, h)]))
    assert (got[G][corners] == 0).all()
    for _ in range(3):  # same bits on every apply
        t2 = torch.from_numpy(full.astype(npdt)).cuda()
        hb.apply(plan, t2)
        torch.cuda.synchronize()
        assert np.array_equal(t2.cpu().numpy().astype(np.float64), got, equal_nan=True)
    y = torch.randn(g.cells, I, dtype=t.dtype, device="cuda", generator=torch.Generator("cuda").manual_seed(4))
    x = torch.from_numpy(np.nan_to_num(full, nan=0.0).astype(npdt)).cuda()
    Ax, z, Aty = x.clone(), torch.zeros_like(x), y.clone()
    hb.apply(plan, Ax)
    hb.apply(plan, z)
    hb.apply_adjoint(plan, Aty)
    torch.cuda.synchronize()
    lhs = float(((Ax.double() - z.double()) * y.double()).sum())
    rhs = float((x.double() * Aty.double()).sum())
    assert abs(lhs - rhs) <= (1e-12 if dt == hb.F64 else 1e-5) * max(abs(lhs), abs(rhs))
    Gm = torch.from_numpy(og.ghost_cells).cuda()
    assert (Aty[Gm] == 0).all()  # covered ghosts cleared


@pytest.mark.parametrize("I,dtype", [(32, "f64"), (3, "f64"), (64, "f32")])
def test_wide_and_narrow_kernels_under_graph_replays(I, dtype):
    """Applies and adjoints of plans served by the LDS-staged (rows >= 128
    bytes) and entry-splitting (rows < 32 bytes) kernels, captured in HIP
    graphs and replayed several times with eager work in between: every
    replay equals the eager result."""
    N, h = 12, 3
    dt, tdt = (hb.F64, torch.float64) if dtype == "f64" else (hb.F32, torch.float32)
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add_quadrature(N, h, 2)
    plan = hb.Plan(p, inner=I, dtype=dt)
    st = plan.stats()
    assert st["rows_wide"] + st["rows_narrow"] == st["rows_csr"] > 0
    src = torch.from_numpy(np.nan_to_num(cs_full_field(N, h, 1, I, seed=70 + I), nan=1.5)).to(tdt).cuda()
    want = src.clone()
    hb.apply(plan, want)
    want_adj = src.clone()
    hb.apply_adjoint(plan, want_adj)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for op, ref in ((hb.OP_APPLY, want), (hb.OP_ADJOINT, want_adj)):
            bufs = [src.clone() for _ in range(2)]
            graph = hb.ApplyGraph(plan, bufs, 2, stream=s.cuda_stream, op=op)  # one call per field
            for rep in range(3):
                for b in bufs:
                    b.copy_(src)
                torch.cuda.synchronize()
                graph.launch(s.cuda_stream)
                torch.cuda.synchronize()
                for b in bufs:
                    assert torch.equal(b, ref), (op, rep)
            del graph
