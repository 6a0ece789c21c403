"""GPU parity of the BC apply against the CPU oracle, through the C ABI.

Bar: copies, rotations and zero padding bit-exact (+0.0 for zeros); FP64
interpolated ghosts within 1e-13 * max(|ref|, sum_m |w_m x_m|) per value when
the library applies the oracle's own weights (the kernel's arithmetic), and
the library's FP64 weights within DS_ULPS ulp(N) of the oracle's position s
(the geometry); end to end, the sum of the two.  Data cells never written;
NaN-poisoned ghosts all overwritten.
"""
import math

import numpy as np
import pytest

import synthinputs
from helpers import (DS_ULPS, cs_full_field, gpu_available, lagrange_dw, lagrange_tolerance, normwise_error,
                     oracle_weights_program, ulp_n)
from oracle import apply as o_apply, assemble, vjp as o_vjp
from oracle import cubed_sphere as ocs
from oracle import hpcg as ohpcg

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_2605_14780_amd as hb


def run_apply(plan, full, order=0, dtype=np.float64):
    import torch
    I = full.shape[1]
    arr = full if order == 0 else np.ascontiguousarray(full.T)
    t = torch.from_numpy(np.ascontiguousarray(arr.astype(dtype))).cuda()
    hb.apply(plan, t)
    torch.cuda.synchronize()
    out = t.cpu().numpy().astype(np.float64)
    return out if order == 0 else np.ascontiguousarray(out.T)


def interp_bound(op, X):
    acc = 0.0
    for A in op.parts.values():
        acc = acc + abs(A) @ np.abs(X)
    return acc


def check_cs(N, h, nf, nl, mode, vector, seed=1, noise=0.0, order=0):
    I = nf * nl
    vec = (2 * nl, nl, nl) if vector else None
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE if mode == "lagrange" else hb.CS_SYNC, vector=vector)
    plan = hb.Plan(prog, inner=I, order=order, vec=vec)
    full = cs_full_field(N, h, nf, nl, seed, noise)
    got = run_apply(plan, full, order)
    og = ocs.grid(N, h)
    op = assemble(og, ocs.subs(N, h, mode, vector=vector))
    ref = o_apply(op, full, vec)
    G, Dc = og.ghost_cells, og.data_cells
    assert np.array_equal(got[Dc], full[Dc]), "data cells were written"
    assert np.isfinite(got[G]).all(), "a ghost was left unwritten"
    corner = np.array([ocs.is_corner(*og.coord_of_cell(int(c))[1][1:], N) for c in G])
    zc = got[G][corner]
    assert (zc == 0).all() and not np.signbit(zc).any(), "corner ghosts must be +0.0"
    if mode == "sync":
        assert np.array_equal(got[G], ref[G])
        return 0.0
    tol = lagrange_tolerance(N, h, full, ref, vec if vector else None)
    diff = np.abs(got[G] - ref[G])
    assert (diff <= tol).all(), float((diff / np.maximum(tol, 1e-300)).max())
    nw = normwise_error(got[G], ref[G], full[Dc])
    assert nw <= 1e-13, nw
    return nw


@pytest.mark.parametrize("N,h,nf,nl,vector", [(8, 3, 1, 1, False), (12, 3, 4, 2, True), (13, 2, 4, 3, True),
                                              (48, 3, 1, 1, False), (4, 2, 4, 1, True)])
def test_cs_sync_bit_exact(N, h, nf, nl, vector):
    check_cs(N, h, nf, nl, "sync", vector)


@pytest.mark.parametrize("N,h,nf,nl,vector", [(8, 3, 1, 1, False), (12, 3, 4, 2, True), (13, 2, 4, 3, True),
                                              (48, 3, 1, 1, False), (48, 3, 4, 8, True), (4, 2, 4, 1, True),
                                              (5, 2, 1, 2, False)])
def test_cs_lagrange_fp64(N, h, nf, nl, vector):
    check_cs(N, h, nf, nl, "lagrange", vector, noise=1e-3)


@pytest.mark.parametrize("mode", ["sync", "lagrange"])
def test_cs_plane_major(mode):
    check_cs(12, 3, 4, 2, mode, True, order=hb.PLANE_MAJOR)


def weight_bound(s, base, N):
    """|w_gpu - w_oracle| allowed per node: the position s held to DS_ULPS
    ulp(N) moves w_m by at most that times |dw_m/ds|; 16 eps for the roundings
    of the weight formula on either side."""
    return [DS_ULPS * ulp_n(N) * abs(dw) + 16 * 2.0 ** -53 for dw in lagrange_dw(s, base)]


def test_cs_weights_match_oracle():
    for N, h in [(8, 3), (13, 3), (48, 3), (384, 3), (768, 4)]:
        base, w = hb.cs_lagrange_weights(N, h)
        torch.cuda.synchronize()
        base, w = base.cpu().numpy(), w.cpu().numpy().reshape(h, N, 4)
        base = base.reshape(h, N)
        # face 0, right side: ghost (j = t, i = N + k) reads face 1's line i = k, nodes along j
        for k in range(h):
            for t in range(N):
                g, axis, L, s = ocs.neighbour_line(0, t, N + k, N)
                ob, ow, s = ocs.lagrange_weights(s, N)
                if abs(s - round(s)) > 1e-9:
                    assert base[k, t] == ob, (N, k, t)
                    bnd = weight_bound(s, ob, N)
                    assert (np.abs(w[k, t] - np.array(ow)) <= bnd).all(), (N, k, t)
                else:
                    node = int(round(s))
                    assert w[k, t][node - base[k, t]] == 1.0


@pytest.mark.parametrize("N,h", [(8, 3), (13, 3), (48, 3), (384, 3), (768, 3)])
def test_cs_weights_in_plan_match_oracle_all_sides(N, h):
    """The weights the library builds on the GPU, as they land in the compiled
    plan on every one of the 24 face sides (orientation tables included):
    columns identical to the oracle's, weights within the position bound."""
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE)
    plan = hb.Plan(prog, inner=1, host_only=False)
    W = N + 2 * h
    worst = 0.0
    for f in range(6):
        for side in (ocs.LEFT, ocs.RIGHT, ocs.BOTTOM, ocs.TOP):
            box = ocs.side_box(f, side, N, h)
            for j in range(*box[1]):
                for i in range(*box[2]):
                    kind, cols, vals, b, rot = plan.row((f * W + (j + h)) * W + (i + h))
                    g, axis, L, s = ocs.neighbour_line(f, j, i, N)
                    ob, ow, s = ocs.lagrange_weights(s, N)
                    node = (lambda m: (g, m, L)) if axis == "i" else (lambda m: (g, L, m))
                    cell = [(gg * W + (jj + h)) * W + (ii + h) for gg, jj, ii in (node(ob + m) for m in range(4))]
                    got = dict(zip(cols, vals))
                    assert kind == 2 and len(cols) == 4, (f, j, i, kind)
                    if abs(s - round(s)) <= 1e-9:
                        # snapped to a node (R7): weight 1 there, 0 elsewhere; on a
                        # side whose index runs against the neighbour's, the stencil
                        # is the other one of the two around that node (same value)
                        nz = {c: v for c, v in got.items() if v != 0}
                        assert nz == {cell[list(ow).index(1.0)]: 1.0}, (f, j, i, got)
                        continue
                    assert set(got) == set(cell), (f, j, i)
                    bnd = weight_bound(s, ob, N)
                    dw = lagrange_dw(s, ob)
                    for m in range(4):
                        err = abs(got[cell[m]] - ow[m])
                        assert err <= bnd[m], (f, j, i, m, err, bnd[m])
                        if abs(dw[m]) > 0.1:
                            worst = max(worst, err / abs(dw[m]) / ulp_n(N))
    print(f"C{N}: largest implied position difference {worst:.2f} ulp(N)")


@pytest.mark.parametrize("N,h,nf,nl,vector", [(48, 3, 4, 8, True), (48, 3, 4, 16, True), (48, 3, 1, 1, False),
                                              (13, 2, 4, 3, True), (5, 2, 1, 2, False), (96, 3, 4, 64, True)])
def test_cs_lagrange_kernel_arithmetic_plain_bound(N, h, nf, nl, vector):
    """The kernel's arithmetic alone, held to the plain bound
    1e-13 * max(|ref|, sum_m |w_m x_m|) with no position term: the program
    carries the oracle's own columns and weights (add_ell, one sub-matrix per
    face side with its rotation), so the library and the oracle apply the same
    A and differ only in the rounding of the sums.  Rows of 512 bytes and more
    run the window kernel, shorter ones the row kernel."""
    I = nf * nl
    vec = (2 * nl, nl, nl) if vector else None
    grid, prog = oracle_weights_program(hb, N, h, vector)
    plan = hb.Plan(prog, inner=I, vec=vec)
    full = cs_full_field(N, h, nf, nl, seed=1, noise=1e-3)
    got = run_apply(plan, full)
    og = ocs.grid(N, h)
    ref = o_apply(assemble(og, ocs.subs(N, h, "lagrange", vector=vector)), full, vec)
    G, Dc = og.ghost_cells, og.data_cells
    assert np.array_equal(got[Dc], full[Dc])
    tol = lagrange_tolerance(N, h, full, ref, vec, ds=0.0)
    diff = np.abs(got[G] - ref[G])
    assert (diff <= tol).all(), float((diff / np.maximum(tol, 1e-300)).max())


def test_unit_vector_probing_recovers_A():
    N, h = 6, 2
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE)
    plan = hb.Plan(prog, inner=1)
    og = ocs.grid(N, h)
    A = assemble(og, ocs.subs(N, h, "lagrange")).dense()
    G, Dc = og.ghost_cells, og.data_cells
    nD = len(Dc)
    # probe many columns at once: inner slot k carries e_{j} for j = k (batched probing via inner extent)
    plan_b = hb.Plan(prog, inner=nD)
    full = np.zeros((og.ncells, nD))
    full[Dc, np.arange(nD)] = 1.0
    got = run_apply(plan_b, full)
    Ag = got[G]
    assert np.array_equal(Ag != 0, A != 0)
    assert np.abs(Ag - A).max() <= 1e-14


def hpcg_field(nb, n, x):
    g = ohpcg.grid(nb, n)
    blocks = ohpcg.ghosted_blocks(x, nb)
    full = np.full(g.ncells, np.nan)
    for b in range(nb ** 3):
        cells = g.cells_of_box(b, g.blocks[b].data)
        full[cells] = blocks[b][1:-1, 1:-1, 1:-1].reshape(-1)
    return g, blocks, full


@pytest.mark.parametrize("nb,n", [(2, 8), (2, 13), (2, 128), (1, 16), (3, 9)])
def test_hpcg_bc_and_stencil(nb, n):
    x = synthinputs.uniform((nb * n,) * 3, seed=3)
    g, blocks, full = hpcg_field(nb, n, x)
    hg = hb.Grid.cartesian([nb] * 3, [n] * 3, 1)
    prog = hb.Program(hg)
    prog.cart_add_halo([nb] * 3, [n] * 3, 1)
    plan = hb.Plan(prog, inner=1)
    st = plan.stats()
    assert st["rows_uncovered"] == 0 and st["segments"] == nb ** 3 * 26
    xt = torch.from_numpy(full.copy()).cuda()
    # fused first: it reads through the BC and materialises the ghosts
    y_f = torch.empty(nb ** 3 * n ** 3, dtype=torch.float64, device="cuda")
    hb.fused_stencil27(plan, xt, y_f)
    torch.cuda.synchronize()
    xf = xt.cpu().numpy()
    want = np.concatenate([b.reshape(-1) for b in blocks])
    assert np.array_equal(xf, want), "fused ghosts differ from the oracle's halo"
    # read-only fused: same y, x (ghosts NaN) left untouched
    xt_ro = torch.from_numpy(full.copy()).cuda()
    y_ro = torch.empty_like(y_f)
    hb.fused_stencil27(plan, xt_ro, y_ro, write_ghosts=False)
    torch.cuda.synchronize()
    assert torch.equal(y_ro, y_f)
    assert np.array_equal(xt_ro.cpu().numpy(), full, equal_nan=True)
    # unfused: BC apply then stencil on a fresh copy
    xt2 = torch.from_numpy(full.copy()).cuda()
    hb.apply(plan, xt2)
    y_u = torch.empty_like(y_f)
    hb.stencil27(plan, xt2, y_u)
    torch.cuda.synchronize()
    assert np.array_equal(xt2.cpu().numpy(), want), "BC apply ghosts differ from the oracle's halo"
    yref = np.concatenate([ohpcg.stencil27(b).reshape(-1) for b in blocks])
    bound = np.concatenate([ohpcg.abs_row_sum(b).reshape(-1) for b in blocks])
    tol = 64 * 2.0 ** -53 * bound
    for y in (y_f, y_u):
        d = np.abs(y.cpu().numpy() - yref)
        assert (d <= tol).all(), float((d / np.maximum(bound, 1e-300)).max())


FACE7 = [(0, 0, 0, 0), (0, 1, 0, 0), (0, -1, 0, 0), (0, 0, 1, 0), (0, 0, -1, 0), (0, 0, 0, 1), (0, 0, 0, -1)]


@pytest.mark.parametrize("nb,n", [(2, 24), (3, 9)])
def test_hpcg_fused_with_uncovered_regions(nb, n):
    """A plan that drops the edge and corner rows (a 7-point consumer
    footprint): the fused form reads those regions from x itself and neither
    form writes them.  Fused (with and without ghost stores) equals BC apply +
    stencil bit for bit, in y and in x."""
    x = synthinputs.uniform((nb * n,) * 3, seed=5)
    g, blocks, full = hpcg_field(nb, n, x)
    want = np.concatenate([b.reshape(-1) for b in blocks])
    W = n + 2
    c = np.arange(W)
    on = ((c == 0) | (c == W - 1)).astype(int)
    cnt = on[:, None, None] + on[None, :, None] + on[None, None, :]
    edge = np.broadcast_to(cnt >= 2, (nb ** 3, W, W, W)).reshape(-1)
    pre = full.copy()
    pre[edge] = want[edge]  # edge / corner ghosts hold the halo values; face ghosts stay NaN
    hg = hb.Grid.cartesian([nb] * 3, [n] * 3, 1)
    prog = hb.Program(hg)
    prog.cart_add_halo([nb] * 3, [n] * 3, 1)
    prog.set_consumer(FACE7)
    plan = hb.Plan(prog, inner=1)
    assert plan.stats()["rows_dead"] > 0
    ny = nb ** 3 * n ** 3
    xa = torch.from_numpy(pre.copy()).cuda()
    ya = torch.empty(ny, dtype=torch.float64, device="cuda")
    hb.apply(plan, xa)
    hb.stencil27(plan, xa, ya)
    xf = torch.from_numpy(pre.copy()).cuda()
    yf = torch.empty_like(ya)
    hb.fused_stencil27(plan, xf, yf)
    xr = torch.from_numpy(pre.copy()).cuda()
    yr = torch.empty_like(ya)
    hb.fused_stencil27(plan, xr, yr, write_ghosts=False)
    torch.cuda.synchronize()
    assert np.array_equal(xa.cpu().numpy(), want)  # faces from the BC, edges as they were
    assert np.array_equal(xf.cpu().numpy(), want)
    assert np.array_equal(xr.cpu().numpy(), pre, equal_nan=True)
    assert torch.equal(yf, ya) and torch.equal(yr, ya)
    yref = np.concatenate([ohpcg.stencil27(b).reshape(-1) for b in blocks])
    bound = np.concatenate([ohpcg.abs_row_sum(b).reshape(-1) for b in blocks])
    assert (np.abs(ya.cpu().numpy() - yref) <= 64 * 2.0 ** -53 * bound).all()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nb,n,periodic", [((2, 1, 3), (70, 9, 37), 0), ((1, 2, 2), (5, 17, 130), 5)])
def test_hpcg_noncubic_blocks(nb, n, periodic, dtype):
    """Blocks of unequal extents: z chunks with a 6-plane tail, partial x and
    y tiles, an x tile two values wide; zero padding or periodic wrap per
    dimension.  The fused forms equal BC apply + stencil bit for bit (y and
    x's ghosts), and y matches a plain numpy 27-point operator on the padded
    global field within 64 roundings of the absolute row sum."""
    tdt, dt, eps = (torch.float64, hb.F64, 2.0 ** -53) if dtype == "f64" else (torch.float32, hb.F32, 2.0 ** -24)
    N = [nb[d] * n[d] for d in range(3)]
    g = np.random.default_rng(11).standard_normal(N)
    if dtype == "f32":
        g = g.astype(np.float32).astype(np.float64)
    W = [n[d] + 2 for d in range(3)]
    full = np.full((nb[0] * nb[1] * nb[2], W[0], W[1], W[2]), np.nan)
    blocks = []
    for bz in range(nb[0]):
        for by in range(nb[1]):
            for bx in range(nb[2]):
                sl = tuple(slice(c * n[d], (c + 1) * n[d]) for d, c in enumerate((bz, by, bx)))
                full[(bz * nb[1] + by) * nb[2] + bx, 1:-1, 1:-1, 1:-1] = g[sl]
                blocks.append(sl)
    pad = g
    for d in range(3):
        widths = [(1, 1) if i == d else (0, 0) for i in range(3)]
        pad = np.pad(pad, widths, mode="wrap" if periodic >> d & 1 else "constant")
    box = np.zeros(N)
    abox = np.zeros(N)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                v = pad[dz:dz + N[0], dy:dy + N[1], dx:dx + N[2]]
                box += v
                abox += np.abs(v)
    yref_g = 27 * g - box
    bound_g = 26 * np.abs(g) + (abox - np.abs(g))
    yref = np.concatenate([yref_g[sl].reshape(-1) for sl in blocks])
    bound = np.concatenate([bound_g[sl].reshape(-1) for sl in blocks])
    hg = hb.Grid.cartesian(list(nb), list(n), 1)
    prog = hb.Program(hg)
    prog.cart_add_halo(list(nb), list(n), 1, periodic)
    plan = hb.Plan(prog, inner=1, dtype=dt)
    src = torch.from_numpy(full.reshape(-1)).to(tdt).cuda()
    ny = int(np.prod(N))
    xa, ya = src.clone(), torch.empty(ny, dtype=tdt, device="cuda")
    hb.apply(plan, xa)
    hb.stencil27(plan, xa, ya)
    xf, yf = src.clone(), torch.empty_like(ya)
    hb.fused_stencil27(plan, xf, yf)
    xr, yr = src.clone(), torch.empty_like(ya)
    hb.fused_stencil27(plan, xr, yr, write_ghosts=False)
    torch.cuda.synchronize()
    assert torch.equal(yf, ya) and torch.equal(yr, ya)
    assert np.array_equal(xf.cpu().numpy(), xa.cpu().numpy(), equal_nan=True)
    assert np.array_equal(xr.cpu().numpy(), src.cpu().numpy(), equal_nan=True)
    d = np.abs(ya.cpu().numpy().astype(np.float64) - yref)
    assert (d <= 64 * eps * bound).all(), float((d / np.maximum(bound, 1e-300)).max())


def test_hpcg_partly_covered_region_refuses_the_fused_form():
    """One ghost region covered for half its cells: the fused form would read
    the other half through the BC, so it is refused; the unfused form runs."""
    n = 8
    hg = hb.Grid.cartesian([1, 1, 1], [n] * 3, 1)
    prog = hb.Program(hg)
    prog.add_map([(0, 1), (0, n), (0, n // 2), (-1, 0)], np.eye(4, dtype=np.int64), [0, 0, 0, n])
    plan = hb.Plan(prog, inner=1)
    xt = torch.zeros(hg.cells, dtype=torch.float64, device="cuda")
    y = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    hb.stencil27(plan, xt, y)
    torch.cuda.synchronize()
    assert torch.equal(y, torch.zeros_like(y))
    for wg in (True, False):
        with pytest.raises(hb.HbcError) as e:
            hb.fused_stencil27(plan, xt, y, write_ghosts=wg)
        assert e.value.code == hb.EUNSUPPORTED and "partly covered" in str(e.value)


def test_hpcg_closed_form_on_ones():
    nb, n = 2, 16
    x = np.ones((nb * n,) * 3)
    g, blocks, full = hpcg_field(nb, n, x)
    hg = hb.Grid.cartesian([nb] * 3, [n] * 3, 1)
    prog = hb.Program(hg)
    prog.cart_add_halo([nb] * 3, [n] * 3, 1)
    plan = hb.Plan(prog, inner=1)
    xt = torch.from_numpy(full.copy()).cuda()
    y = torch.empty(nb ** 3 * n ** 3, dtype=torch.float64, device="cuda")
    hb.fused_stencil27(plan, xt, y)
    torch.cuda.synchronize()
    yb = y.cpu().numpy().reshape(nb, nb, nb, n, n, n).transpose(0, 3, 1, 4, 2, 5).reshape((nb * n,) * 3)
    nd = nb * n
    idx = np.arange(nd)
    on_b = ((idx == 0) | (idx == nd - 1)).astype(int)
    cnt = on_b[:, None, None] + on_b[None, :, None] + on_b[None, None, :]
    want = np.select([cnt == 0, cnt == 1, cnt == 2, cnt == 3], [0.0, 9.0, 15.0, 19.0])
    assert np.array_equal(yb, want)


NP_MODE = {"zero": "constant", "symmetric": "symmetric", "circular": "wrap"}


def fmap1(kind, n):
    """(M, o) of one axis: symmetric / circular index maps of a ghost side."""
    if kind == "symmetric":
        return {"lo": (-1, -1), "hi": (-1, 2 * n - 1)}
    return {"lo": (1, n), "hi": (1, -n)}


@pytest.mark.parametrize("k0,k1", [("zero", "symmetric"), ("circular", "circular"), ("symmetric", "circular"),
                                   ("symmetric", "symmetric")])
@pytest.mark.parametrize("n0,n1,h,I", [(5, 7, 1, 1), (6, 9, 3, 3), (17, 4, 2, 8)])
def test_padding_modes_match_numpy_pad(k0, k1, n0, n1, h, I):
    g = hb.Grid([0, -h, -h], [1, n0 + h, n1 + h])
    g.add_block([(0, 1), (-h, n0 + h), (-h, n1 + h)], [(0, 1), (0, n0), (0, n1)])
    prog = hb.Program(g)
    ranges = [[(-h, 0), (0, n0), (n0, n0 + h)], [(-h, 0), (0, n1), (n1, n1 + h)]]
    kinds = [k0, k1]
    ns = [n0, n1]
    for a in range(3):
        for b in range(3):
            if a == 1 and b == 1:
                continue
            box = [(0, 1), ranges[0][a], ranges[1][b]]
            if (a != 1 and k0 == "zero") or (b != 1 and k1 == "zero"):
                prog.add_zero(box)
                continue
            M = np.zeros((3, 3), dtype=np.int64)
            o = np.zeros(3, dtype=np.int64)
            for d, side in ((0, a), (1, b)):
                if side == 1:
                    M[d + 1, d + 1] = 1
                    continue
                m, off = fmap1(kinds[d], ns[d])["lo" if side == 0 else "hi"]
                M[d + 1, d + 1] = m
                o[d + 1] = off
            prog.add_map(box, M, o)
    plan = hb.Plan(prog, inner=I)
    data = np.random.default_rng(7).standard_normal((n0, n1, I))
    full = np.full((n0 + 2 * h, n1 + 2 * h, I), np.nan)
    full[h:h + n0, h:h + n1] = data
    got = run_apply(plan, full.reshape(-1, I)).reshape(full.shape)
    ref = np.pad(data, ((0, 0), (h, h), (0, 0)), mode=NP_MODE[k1])
    ref = np.pad(ref, ((h, h), (0, 0), (0, 0)), mode=NP_MODE[k0])
    assert np.array_equal(got, ref)


def test_alg1_example_with_csr():
    g = hb.Grid([0, -1, -1], [3, 6, 6])
    for i in range(3):
        g.add_block([(i, i + 1), (-1, 6), (-1, 6)], [(i, i + 1), (0, 5), (0, 5)])
    prog = hb.Program(g)
    # right ghost of block 1: col = [2, 9 - i[2], i[1]]
    M = np.array([[0, 0, 0], [0, 0, -1], [0, 1, 0]])
    prog.add_map([(1, 2), (0, 5), (5, 6)], M, [2, 9, 0])
    # left ghost: CSR rows reading block 0 (2-point averages)
    lin = lambda b, r, c: (b * 7 + (r + 1)) * 7 + (c + 1)
    ptr = np.arange(0, 11, 2)
    cols = [lin(0, r, c) for r in range(5) for c in (3, 4)]
    prog.add_csr([(1, 2), (0, 5), (-1, 0)], ptr, cols, np.full(10, 0.5))
    prog.add_zero_rest(1)
    plan = hb.Plan(prog, inner=2)
    st = plan.stats()
    assert st["rows_covered"] == 24 and st["rows_zero"] == 14 and st["rows_map"] == 5 and st["rows_csr"] == 5
    u = np.random.default_rng(1).standard_normal((3 * 49, 2))
    got = run_apply(plan, u)
    cell = lambda b, r, c: b * 49 + (r + 1) * 7 + (c + 1)
    for r in range(5):
        assert np.array_equal(got[cell(1, r, 5)], u[cell(2, 4, r)])
        assert np.allclose(got[cell(1, r, -1)], 0.5 * (u[cell(0, r, 3)] + u[cell(0, r, 4)]), rtol=1e-15, atol=0)
    untouched = [c for b in (0, 2) for c in range(b * 49, b * 49 + 49)]
    assert np.array_equal(got[untouched], u[untouched])


def test_subvector_overlap_sum_and_ragged():
    n0, n1, h, I = 7, 5, 2, 3  # I = 3: no 16-byte vector path, ragged rows
    g = hb.Grid([0, -h, -h], [1, n0 + h, n1 + h])
    g.add_block([(0, 1), (-h, n0 + h), (-h, n1 + h)], [(0, 1), (0, n0), (0, n1)])
    prog = hb.Program(g)
    prog.set_flags(hb.ALLOW_OVERLAP_SUM)
    rows = [(0, 1), (-h, 0), (0, n1)]
    M = np.diag([1, -1, 1])
    prog.add_map(rows, M, [0, -1, 0], weight=1.0)            # symmetric copy
    prog.add_map([(0, 1), (-1, 0), (1, 4)], np.diag([1, 0, 1]), [0, 3, 0], weight=0.25)  # overlaps: adds
    b = np.random.default_rng(2).standard_normal((h * n1, I))
    prog.add_vector(rows, b, ninner=I)
    prog.add_vector([(0, 1), (n0, n0 + 1), (0, 1)], [2.5], ninner=1)  # pure-function ghost (b only)
    plan = hb.Plan(prog, inner=I)
    u = np.random.default_rng(3).standard_normal((g.cells, I))
    got = run_apply(plan, u)
    W = n1 + 2 * h
    cell = lambda y, x: (y + h) * W + (x + h)
    k = 0
    for y in range(-h, 0):
        for x in range(n1):
            want = u[cell(-y - 1, x)].copy()
            if y == -1 and 1 <= x < 4:
                want = want + 0.25 * u[cell(3, x)]
            want = want + b[k]
            assert np.allclose(got[cell(y, x)], want, rtol=1e-15, atol=1e-15), (y, x)
            k += 1
    assert (got[cell(n0, 0)] == 2.5).all()
    st = plan.stats()
    assert st["rows_uncovered"] == (g.cells - n0 * n1) - (h * n1 + 1)


def test_empty_program_is_a_no_op():
    g = hb.Grid.cubed_sphere(4, 1)
    prog = hb.Program(g)
    plan = hb.Plan(prog, inner=2)
    assert plan.stats()["rows_covered"] == 0
    u = np.random.default_rng(0).standard_normal((g.cells, 2))
    assert np.array_equal(run_apply(plan, u), u)


def test_size_and_alignment_errors():
    grid, prog = hb.cs_program(8, 2, hb.CS_SYNC)
    plan = hb.Plan(prog, inner=2)
    t = torch.zeros(grid.cells * 2 - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(hb.HbcError):
        hb.apply(plan, t)
    t = torch.zeros(grid.cells * 2 + 1, dtype=torch.float64, device="cuda")[1:]
    with pytest.raises(hb.HbcError):
        hb.apply(plan, t)


@pytest.mark.parametrize("I,order,dtype", [(3, 0, "f64"), (8, 0, "f64"), (32, 0, "f64"), (64, 0, "f32"),
                                           (4, 1, "f64"), (7, 0, "f32")])
def test_csr_segments_with_empty_rows(I, order, dtype):
    """CSR rows alternating 16 entries and none (8 per row on average), with
    b on half of them: the segment goes to the entry-splitting kernel (rows
    < 32 bytes), the general row path, the LDS-staged kernel (rows >= 128
    bytes) or the plane-major kernel; empty rows give 0 (+ b)."""
    from oracle import RowsSub, VectorSub
    from oracle.grid import Grid as OGrid
    n0, n1, h = 40, 24, 2
    lo, hi = [-h, -h], [n0 + h, n1 + h]
    g = hb.Grid(lo, hi)
    g.add_block([(-h, n0 + h), (-h, n1 + h)], [(0, n0), (0, n1)])
    og = OGrid(lo, hi)
    og.add_block([(-h, n0 + h), (-h, n1 + h)], [(0, n0), (0, n1)])
    rows = [(-h, 0), (0, n1)]
    nrows = h * n1
    rng = np.random.default_rng(I)
    W = hi[1] - lo[1]
    ptr, cols, vals, ents = [0], [], [], []
    for r in range(nrows):
        e = []
        if r % 2 == 0:
            for _ in range(16):
                x, y = int(rng.integers(0, n0)), int(rng.integers(0, n1))
                w = float(rng.standard_normal())
                e.append(((x, y), w))
                cols.append((x - lo[0]) * W + (y - lo[1]))
                vals.append(w)
        ptr.append(len(cols))
        ents.append(e)
    p = hb.Program(g)
    p.add_csr(rows, ptr, cols, vals)
    b_rows = [(-1, 0), (0, n1)]
    b = rng.standard_normal((n1, I))
    p.add_vector(b_rows, b, ninner=I)
    dt, npdt = (hb.F64, np.float64) if dtype == "f64" else (hb.F32, np.float32)
    plan = hb.Plan(p, inner=I, order=order, dtype=dt)
    st = plan.stats()
    if order == 0 and I * np.dtype(npdt).itemsize < 32:
        assert st["rows_narrow"] == nrows
    elif order == 0 and I * np.dtype(npdt).itemsize >= 128:
        assert st["rows_wide"] == nrows
    else:
        assert st["rows_narrow"] == 0 and st["rows_wide"] == 0
    order_of = {}
    for k, (x, y) in enumerate((x, y) for x in range(-h, 0) for y in range(0, n1)):
        order_of[(x, y)] = k
    sub = RowsSub(rows, lambda c: ents[order_of[(c[0], c[1])]])
    op = assemble(og, [sub, VectorSub(b_rows, b)])
    full = rng.standard_normal((og.ncells, I)).astype(npdt).astype(np.float64)  # inputs as the GPU holds them
    ref = o_apply(op, full)
    got = run_apply(plan, full, order, npdt)
    G = og.ghost_cells
    eps = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    mag = np.abs(op.dense()) @ np.abs(full[og.data_cells])
    mag = mag + (np.abs(op.b) if op.b is not None else 0.0)
    err = np.abs(got[G] - ref[G])
    bad = np.argwhere(err > 32 * eps * mag + 1e-300)
    assert bad.size == 0, (bad[:5].tolist(), err[tuple(bad[0])], mag[tuple(bad[0])], got[G][tuple(bad[0])],
                           ref[G][tuple(bad[0])], og.coord_of_cell(int(G[bad[0][0]])))
    empty = np.array([len(e) == 0 for e in ents])
    cells = og.cells_of_box(0, rows)
    no_b = og.cells_of_box(0, [(-h, -1), (0, n1)])
    assert (got[np.intersect1d(cells[empty], no_b)] == 0).all()
