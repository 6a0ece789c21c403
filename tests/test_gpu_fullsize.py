"""Full-size GPU checks in the launch configurations the bench times.

* C384, halo 3, 256 inner values (4 fields x 64 levels, (u, v) rotated),
  FP64, after the autotuner has picked the launch shape: sampled ghost rows
  (all 256 values of each; edge strips and corners) against the rows the
  oracle evaluates one by one from the geometry (arithmetic bound plus the
  position bound of the library's FP64 weights); and every ghost of the
  program built from the oracle's own weights at the plain arithmetic bound;
* C768, halo 3, 32 levels, with a sub-vector b on every side: the adjoint
  against the forward through the dot-product identity, and sampled source
  rows of A^T y against the oracle's (FP64 and FP32); finite differences of
  a loss through one linearised shallow-water RK4 step with (h, u, v);
* C384 wide interpolation rows (16..25 entries, LDS-staged kernel): sampled
  rows against the oracle's;
* the 64-grid FP32 batch in its autotuned graph launch: bit identity with
  plain applies and sampled rows against the oracle's;
* a field beyond 4 GiB (C384 x 768 FP64): window kernel, row kernel and
  adjoint on sampled rows and cells at the plain bound;
* the radius-1 cross consumer on the full C384 x 256 field (plan compiled
  with the cross's footprint, the default launch shape the bench times),
  fused and unfused: sampled data cells (every cell along two faces' edges,
  whose stencils reach ghosts, and random interior cells) against the
  oracle's stencil over its BC.
"""

import numpy as np
import pytest

import synthinputs
from helpers import (DS_ULPS, gpu_available, lagrange_dw, lagrange_tolerance, magnitude_operator,
                     oracle_lagrange_rows, oracle_weights_program, ulp_n)
from oracle import apply as o_apply, assemble
from oracle import cubed_sphere as ocs

pytestmark = [pytest.mark.gpu]

U64 = 2.0 ** -53

if gpu_available():
    import torch

    import paper_2605_14780_amd as hb


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c384_sampled_rows_tuned_shape(tmp_path, dtype):
    """The bench's C384 operator (4-point Lagrange rows, (u, v) rotated) in the
    autotuned launch shape: sampled ghost rows against the oracle's rows
    evaluated one by one, corners +0 (FP32: weights rounded from FP64, four
    FP32 terms summed)."""
    N, h, nf, nl = 384, 3, 4, 64
    I = nf * nl
    vec = (2 * nl, nl, nl)
    W = N + 2 * h
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE, vector=True)
    dt, tdt = (hb.F64, torch.float64) if dtype == "f64" else (hb.F32, torch.float32)
    plan = hb.Plan(prog, inner=I, vec=vec, dtype=dt)
    data = synthinputs.cs_sh_field_torch(N, nf, nl, seed=2, device="cuda")
    full = torch.full((6, W, W, I), float("nan"), dtype=tdt, device="cuda")
    full[:, h:h + N, h:h + N] = data.to(tdt)
    full = full.reshape(-1, I)
    del data
    plan.autotune([full.clone() for _ in range(2)], str(tmp_path / "tune.jsonl"))
    out = full.clone()
    hb.apply(plan, out)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all(), "a ghost was left unwritten"
    rng = np.random.default_rng(0)
    u_sl = np.arange(vec[0], vec[0] + vec[2])
    v_sl = u_sl + vec[1]
    rows = corners = 0
    while rows < 1500:
        f = int(rng.integers(6))
        j, i = (int(v) for v in rng.integers(-h, N + h, size=2))
        if 0 <= j < N and 0 <= i < N:
            continue
        got = out[(f * W + (j + h)) * W + (i + h)].cpu().numpy().astype(np.float64)
        if ocs.is_corner(j, i, N):
            assert (got == 0).all() and not np.signbit(got).any(), (f, j, i)
            corners += 1
            continue
        ents = ocs.lagrange_entries(f, j, i, N)
        src = [(g * W + (jj + h)) * W + (ii + h) for (g, jj, ii), _ in ents]
        w = np.array([wv for _, wv in ents])
        X = full[torch.tensor(src, device="cuda")].cpu().numpy().astype(np.float64)  # inputs as the GPU holds them
        y = w @ X
        R = ocs.rside(f, ocs.side_of(j, i, N))
        ref = y.copy()
        ref[u_sl] = R[0, 0] * y[u_sl] + R[0, 1] * y[v_sl]
        ref[v_sl] = R[1, 0] * y[u_sl] + R[1, 1] * y[v_sl]
        # arithmetic: 1e-13 of sum |w x|; position: the library's s is held
        # to DS_ULPS ulp(N) of the oracle's, which moves the value by that
        # times sum |dw/ds| |x| (nodes as the oracle orders them)
        _, _, _, s_or = ocs.neighbour_line(f, j, i, N)
        base, _, s_or = ocs.lagrange_weights(s_or, N)
        dw = np.abs(np.array(lagrange_dw(s_or, base)))
        wx = np.abs(w) @ np.abs(X)
        bnd = 1e-13 * np.maximum(wx, 1e-300) + DS_ULPS * ulp_n(N) * (dw @ np.abs(X))
        if dt == hb.F32:  # weight rounding (1 ulp each) and four FP32 roundings of the sum
            bnd = bnd + 8 * 2.0 ** -24 * wx
        bnd_rot = bnd.copy()
        bnd_rot[u_sl] = np.maximum(bnd[u_sl], bnd[v_sl])
        bnd_rot[v_sl] = bnd_rot[u_sl]
        assert (np.abs(got - ref) <= bnd_rot).all(), (f, j, i)
        rows += 1
    assert corners > 0


def test_c384_oracle_weights_every_ghost_plain_bound(tmp_path):
    """The kernel's arithmetic on the full C384 x 256 FP64 field ((u, v)
    rotated, SH fields + N(0, 1e-3) noise, 9 cold copies for the autotuner):
    the program carries the oracle's own columns and weights, so every ghost
    value must lie within the plain bound 1e-13 * max(|ref|, sum |w x|)."""
    from helpers import cs_full_field
    N, h, nf, nl = 384, 3, 4, 64
    I = nf * nl
    vec = (2 * nl, nl, nl)
    grid, prog = oracle_weights_program(hb, N, h, True)
    plan = hb.Plan(prog, inner=I, vec=vec, dtype=hb.F64)
    st = plan.stats()
    assert st["rows_window"] == st["rows_ell"] == 24 * h * N
    full = cs_full_field(N, h, nf, nl, seed=2, noise=1e-3)
    x = torch.from_numpy(full).cuda()
    plan.autotune([x.clone() for _ in range(3)], str(tmp_path / "tune.jsonl"))
    out = x.clone()
    hb.apply(plan, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    del out, x
    og = ocs.grid(N, h)
    ref = o_apply(assemble(og, ocs.subs(N, h, "lagrange", vector=True)), full, vec)
    G, Dc = og.ghost_cells, og.data_cells
    assert np.array_equal(got[Dc], full[Dc])
    tol = lagrange_tolerance(N, h, full, ref, vec, ds=0.0)
    ratio = np.abs(got[G] - ref[G]) / np.maximum(tol, 1e-300)
    assert ratio.max() <= 1.0, (float(ratio.max()), plan.tune)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c768_adjoint_sampled_source_rows(dtype):
    """The adjoint at C768, halo 3, 32 levels (b on every ghost, as the bench
    runs it), in the bench's launch, element by element on sampled source
    rows against the oracle's VJP: xbar_j = ybar_j + sum_i A_ij ybar_i over the
    ghost rows i that read j, with A the oracle's own rows (the program carries
    them, so only the sums differ).  FP64: 1e-13 of the sum of magnitudes;
    FP32 (weights rounded to FP32, FP32 sums of at most 12 terms): 16 FP32
    roundings of it.  Covered ghosts end at +0."""
    N, h, L = 768, 3, 32
    W = N + 2 * h
    rows = oracle_lagrange_rows(N, h)
    rng = np.random.default_rng(5)
    b = []
    for f in range(6):
        for side in (ocs.LEFT, ocs.RIGHT, ocs.BOTTOM, ocs.TOP):
            b.append((ocs.side_box(f, side, N, h), rng.normal(size=(N * h, L))))
        for box in ocs.corner_boxes(f, N, h):
            b.append((box, rng.normal(size=(h * h, L))))
    grid, prog = oracle_weights_program(hb, N, h, False, rows=rows, b=b)
    dt, tdt, eps, k = (hb.F64, torch.float64, 2.0 ** -53, 1e-13 / 2.0 ** -53) if dtype == "f64" else \
        (hb.F32, torch.float32, 2.0 ** -24, 16.0)
    plan = hb.Plan(prog, inner=L, dtype=dt)
    gen = torch.Generator(device="cuda").manual_seed(7)
    y = torch.randn(grid.cells * L, dtype=tdt, device="cuda", generator=gen)
    aty = y.clone()
    hb.apply_adjoint(plan, aty)
    torch.cuda.synchronize()
    ybar = y.view(-1, L).cpu().numpy().astype(np.float64)
    got = aty.view(-1, L).cpu().numpy().astype(np.float64)
    # the transpose of the oracle's rows: source cell -> [(ghost cell, weight)]
    cols = {}
    for (f, side), (box, ents) in rows.items():
        r = 0
        for j in range(*box[1]):
            for i in range(*box[2]):
                gcell = (f * W + (j + h)) * W + (i + h)
                for (gg, jj, ii), wv in ents[r]:
                    wv = float(np.float32(wv)) if dt == hb.F32 else wv
                    cols.setdefault((gg * W + (jj + h)) * W + (ii + h), []).append((gcell, wv))
                r += 1
    srcs = np.array(sorted(cols))
    pick = rng.choice(srcs, size=3000, replace=False)
    for c in pick:
        ents = cols[int(c)]
        gi = np.array([g for g, _ in ents])
        wv = np.array([w for _, w in ents])
        ref = ybar[c] + wv @ ybar[gi]
        mag = np.abs(ybar[c]) + np.abs(wv) @ np.abs(ybar[gi])
        assert (np.abs(got[c] - ref) <= k * eps * mag).all(), (int(c), len(ents))
    # data cells no ghost reads keep their gradient; covered ghosts are +0
    interior = (3 * W + (N // 2 + h)) * W + (N // 2 + h)
    assert interior not in cols and np.array_equal(got[interior], ybar[interior])
    G = np.ones((6, W, W), dtype=bool)
    G[:, h:h + N, h:h + N] = False
    gg = got.reshape(6, W, W, L)[G]
    assert (gg == 0).all() and not np.signbit(gg).any()


def test_c768_fd_linearised_swe_step_hUV():
    """Finite differences of a loss through one linearised shallow-water RK4
    step at C768, halo 3, 32 levels with (h, u, v) (u, v rotated across faces,
    b on one side), the BC applied before every stage through bc_apply: the
    step is affine in the state, so the centred difference with eps = 1 is
    exact up to rounding and must equal <grad, d> to 1e-12 of the sums'
    magnitudes."""
    from swe import make_step
    N, h, L = 768, 3, 32
    I = 3 * L
    W = N + 2 * h
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE, vector=True)
    rng = np.random.default_rng(11)
    prog.add_vector(ocs.side_box(2, ocs.TOP, N, h), rng.standard_normal((N * h, I)), ninner=I)
    plan = hb.Plan(prog, inner=I, vec=(L, L, L))
    step = make_step(lambda t: hb.bc_apply(plan, t), N, h, L, dx=np.pi / (2 * N), dt=0.2 * np.pi / (2 * N))
    u0 = torch.zeros((6, W, W, I), dtype=torch.float64, device="cuda")
    u0[:, h:h + N, h:h + N] = synthinputs.cs_sh_field_torch(N, 3, L, seed=12, device="cuda")
    u0 = u0.reshape(-1, I)
    gen = torch.Generator("cuda").manual_seed(1)
    wgt = torch.randn(grid.cells, I, dtype=torch.float64, device="cuda", generator=gen)
    d = torch.randn(grid.cells, I, dtype=torch.float64, device="cuda", generator=gen)

    def loss(u):
        return (step(u) * wgt).sum()

    u = u0.clone().requires_grad_(True)
    loss(u).backward()
    gd = float((u.grad * d).sum())
    mag_g = float((u.grad * d).abs().sum())
    del u
    with torch.no_grad():
        lp, lm = step(u0 + d) * wgt, step(u0 - d) * wgt
        fd = (float(lp.sum()) - float(lm.sum())) / 2.0
        mag_f = (float(lp.abs().sum()) + float(lm.abs().sum())) / 2.0
    assert abs(fd - gd) <= 1e-12 * (mag_g + mag_f), (fd, gd, mag_g, mag_f)
    assert abs(gd) > 1e-9 * mag_g


def test_c768_adjoint_dot_product():
    N, h, L = 768, 3, 32
    W = N + 2 * h
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE)
    rng = np.random.default_rng(5)
    for f in range(6):
        for side in (ocs.LEFT, ocs.RIGHT, ocs.BOTTOM, ocs.TOP):
            prog.add_vector(ocs.side_box(f, side, N, h), rng.normal(size=(N * h, L)), ninner=L)
    plan = hb.Plan(prog, inner=L, dtype=hb.F64)
    x = torch.zeros((6, W, W, L), dtype=torch.float64, device="cuda")
    x[:, h:h + N, h:h + N] = synthinputs.cs_sh_field_torch(N, 1, L, seed=5, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(7)
    y = torch.randn(x.shape, dtype=torch.float64, device="cuda", generator=gen)
    y[:, h:h + N, h:h + N] = 0.0      # only the BC part enters the identity
    x, y = x.reshape(-1), y.reshape(-1)
    Ax, b = x.clone(), torch.zeros_like(x)
    hb.apply(plan, Ax)
    hb.apply(plan, b)
    Aty = y.clone()
    hb.apply_adjoint(plan, Aty)
    torch.cuda.synchronize()
    Ax -= b
    lhs_t, rhs_t = Ax * y, x * Aty
    lhs, rhs = float(lhs_t.sum()), float(rhs_t.sum())
    scale = float(lhs_t.abs().sum() + rhs_t.abs().sum())
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    assert abs(lhs) > 1e-6 * scale
    # covered ghosts of the adjoint are cleared
    G = torch.ones((6, W, W), dtype=torch.bool, device="cuda")
    G[:, h:h + N, h:h + N] = False
    assert (Aty.reshape(6, W, W, L)[G] == 0).all()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c384_wide_rows_sampled(dtype):
    """Wide interpolation rows (2x2 Gauss average of cubic reconstructions,
    16..25 entries) at C384, halo 3, 256 inner values with (u, v) rotated,
    through the LDS-staged kernel in the bench's launch (FP64: 256-byte
    slices, FP32: 128-byte slices): sampled ghost rows against the oracle's
    rows evaluated one by one (FP32: weights and sums in FP32)."""
    from oracle import quadrature as oq
    N, h, nf, nl = 384, 3, 4, 64
    I = nf * nl
    vec = (2 * nl, nl, nl)
    W = N + 2 * h
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    p.cs_add_quadrature(N, h, 2, vector=True)
    dt, tdt, eps = (hb.F64, torch.float64, U64) if dtype == "f64" else (hb.F32, torch.float32, 2.0 ** -24)
    plan = hb.Plan(p, inner=I, vec=vec, dtype=dt)
    st = plan.stats()
    assert st["rows_wide"] == st["rows_csr"] == 24 * h * N
    full = torch.full((6, W, W, I), float("nan"), dtype=tdt, device="cuda")
    full[:, h:h + N, h:h + N] = synthinputs.cs_sh_field_torch(N, nf, nl, seed=3, device="cuda").to(tdt)
    full = full.reshape(-1, I)
    out = full.clone()
    hb.apply(plan, out)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all(), "a ghost was left unwritten"
    rng = np.random.default_rng(1)
    u_sl = np.arange(vec[0], vec[0] + vec[2])
    v_sl = u_sl + vec[1]
    rows = 0
    while rows < 400:
        f = int(rng.integers(6))
        j, i = (int(v) for v in rng.integers(-h, N + h, size=2))
        if (0 <= j < N and 0 <= i < N) or ocs.is_corner(j, i, N):
            continue
        got = out[(f * W + (j + h)) * W + (i + h)].cpu().numpy().astype(np.float64)
        ents = oq.quad_entries(f, j, i, N, 2)
        src = [(gg * W + (jj + h)) * W + (ii + h) for (gg, jj, ii), _ in ents]
        w = np.array([wv for _, wv in ents])
        X = full[torch.tensor(src, device="cuda")].cpu().numpy().astype(np.float64)  # inputs as the GPU holds them
        y = w @ X
        R = ocs.rside(f, ocs.side_of(j, i, N))
        ref = y.copy()
        ref[u_sl] = R[0, 0] * y[u_sl] + R[0, 1] * y[v_sl]
        ref[v_sl] = R[1, 0] * y[u_sl] + R[1, 1] * y[v_sl]
        # weights agree with the host's to 1e-13 per entry (pinned host-side);
        # rounding of the weights to the plan's type and of <= 25 terms' sum
        pat = np.abs(X).sum(axis=0)
        mag = np.abs(w) @ np.abs(X)
        bnd = 1e-13 * pat + 64 * eps * mag
        bnd_rot = bnd.copy()
        bnd_rot[u_sl] = np.maximum(bnd[u_sl], bnd[v_sl])
        bnd_rot[v_sl] = bnd_rot[u_sl]
        assert (np.abs(got - ref) <= bnd_rot).all(), (f, j, i)
        rows += 1


def test_batch_64_grids_full_size(tmp_path):
    """The batch of 64 cubed-sphere grids (C48..C768, halo 2..4, 1..128
    levels, FP32) in the autotuned, graph-captured launch: bit-identical to
    64 plain applies, and sampled rows of three grids against the oracle's
    rows (FP32 weights and accumulation: 8 roundings of sum |w x|)."""
    draws = synthinputs.batch_draw()
    plans, inputs = [], []
    for k, (N, h, L) in enumerate(draws):
        grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE)
        plans.append(hb.Plan(prog, inner=L, dtype=hb.F32))
        W = N + 2 * h
        full = torch.full((6, W, W, L), float("nan"), dtype=torch.float32, device="cuda")
        full[:, h:h + N, h:h + N, :] = synthinputs.cs_sh_field_torch(N, 1, L, seed=4000 + k, dtype=torch.float32)
        inputs.append(full.reshape(-1))
    want = []
    for plan, x in zip(plans, inputs):
        y = x.clone()
        hb.apply(plan, y)
        want.append(y)
    batch = hb.Batch(plans)
    fields = [x.clone() for x in inputs]
    batch.bind(fields)
    batch.autotune(str(tmp_path / "batch_tune.jsonl"))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        batch.graph_capture(s.cuda_stream)
        for rep in range(2):
            for f, x in zip(fields, inputs):
                f.copy_(x)
            torch.cuda.synchronize()
            batch.graph_launch(s.cuda_stream)
            torch.cuda.synchronize()
            for k, (f, w) in enumerate(zip(fields, want)):
                assert torch.equal(f, w), (rep, k, draws[k])
    del want
    rng = np.random.default_rng(8)
    sizes = [N for N, _, _ in draws]
    for k in {int(np.argmin(sizes)), int(np.argmax(sizes)), 17}:
        N, h, L = draws[k]
        W = N + 2 * h
        x = inputs[k].reshape(-1, L)
        out = fields[k].reshape(-1, L)
        checked = 0
        while checked < 60:
            f = int(rng.integers(6))
            j, i = (int(v) for v in rng.integers(-h, N + h, size=2))
            if (0 <= j < N and 0 <= i < N) or ocs.is_corner(j, i, N):
                continue
            ents = ocs.lagrange_entries(f, j, i, N)
            src = [(g * W + (jj + h)) * W + (ii + h) for (g, jj, ii), _ in ents]
            w = np.array([wv for _, wv in ents])
            X = x[torch.tensor(src, device="cuda")].cpu().numpy().astype(np.float64)
            ref = w @ X
            got = out[(f * W + (j + h)) * W + (i + h)].cpu().numpy().astype(np.float64)
            assert (np.abs(got - ref) <= 8 * 2.0 ** -24 * (np.abs(w) @ np.abs(X))).all(), (k, f, j, i)
            checked += 1


def test_c384_cross_consumer_sampled():
    """The cross consumer (weights -4, 1, 1, 1, 1, the line walk) on the full
    C384 x 256 FP64 field ((u, v) rotated), with the oracle's own columns and
    weights in the BC program so that the plain arithmetic bound applies:
    every sampled cell within 1e-13 of sum_o |w_o| T[c + o], T = |u| on data
    cells and sum |A| |u| on ghosts, fused (composed boundary rows) and
    unfused (stored ghosts)."""
    from helpers import cs_full_field
    N, h, nf, nl = 384, 3, 4, 64
    I = nf * nl
    vec = (2 * nl, nl, nl)
    W = N + 2 * h
    cross = [(0, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    wts = [-4.0, 1.0, 1.0, 1.0, 1.0]
    grid, prog = oracle_weights_program(hb, N, h, True)
    prog.set_consumer(cross)
    plan = hb.Plan(prog, inner=I, vec=vec, dtype=hb.F64)
    cons = hb.Consumer(plan, cross, wts)
    assert cons.stats()["boundary_rows"] > 0
    full = cs_full_field(N, h, nf, nl, seed=2, noise=1e-3)
    ndata = 6 * N * N
    ys = {}
    for fused in (True, False):
        x = torch.from_numpy(full).cuda()
        if not fused:
            hb.apply(plan, x)
        y = torch.full((ndata * I,), float("nan"), dtype=torch.float64, device="cuda")
        cons.apply(x, y, fused=fused)
        torch.cuda.synchronize()
        ys[fused] = y.view(ndata, I).cpu().numpy()
        del x, y
    og = ocs.grid(N, h)
    op = assemble(og, ocs.subs(N, h, "lagrange", vector=True))
    up = o_apply(op, full, vec).reshape(6, W, W, I)
    T = o_apply(magnitude_operator(op), np.abs(full), vec).reshape(6, W, W, I)
    # every cell along the edges of faces 0 and 4 (j = 0, N - 1) and faces 2
    # and 5 (i = 0, N - 1), then random interior cells
    ii = np.arange(N)
    f_, i_, j_ = [], [], []
    for f in (0, 4):
        for j in (0, N - 1):
            f_.append(np.full(N, f)), i_.append(ii), j_.append(np.full(N, j))
    for f in (2, 5):
        for i in (0, N - 1):
            f_.append(np.full(N, f)), i_.append(np.full(N, i)), j_.append(ii)
    rng = np.random.default_rng(7)
    f_.append(rng.integers(0, 6, 1000)), i_.append(rng.integers(1, N - 1, 1000)), j_.append(rng.integers(1, N - 1, 1000))
    f, i, j = (np.concatenate(a) for a in (f_, i_, j_))
    ref = np.zeros((len(f), I))
    bound = np.zeros((len(f), I))
    for (_, di, dj), w in zip(cross, wts):
        ref += w * up[f, h + i + di, h + j + dj]
        bound += abs(w) * T[f, h + i + di, h + j + dj]
    rows = f * N * N + i * N + j
    for fused, y in ys.items():
        got = y[rows]
        assert np.isfinite(got).all(), fused
        ratio = np.abs(got - ref) / np.maximum(1e-13 * bound, 1e-300)
        assert ratio.max() <= 1.0, (fused, float(ratio.max()))


def test_c384_field_beyond_4_gib():
    """A field of more than 4 GiB (C384, halo 3, 768 FP64 values per cell:
    5.6 GB), so that cell offsets need 64 bits: the window kernel and the row
    kernel (a plan built without windows) on the program carrying the
    oracle's own weights; 3000 sampled ghost rows, all 768 values, within
    the plain bound 1e-13 * max(|ref|, sum |w x|) of the oracle's rows; and
    the adjoint on the same field, 3000 sampled data cells that some ghost
    reads against ybar + A^T ybar from the oracle's columns (bound: (entries
    + 2) roundings of |ybar| + |A|^T |ybar|)."""
    N, h, I = 384, 3, 768
    grid, prog = oracle_weights_program(hb, N, h, False)
    og = ocs.grid(N, h)
    assert og.ncells * I * 8 > 4 * 2 ** 30
    rng = np.random.default_rng(11)
    full = rng.standard_normal((og.ncells, I))
    op = assemble(og, ocs.subs(N, h, "lagrange"))
    A = sum(op.parts.values()).tocsr()
    G = og.ghost_cells
    pick = rng.choice(np.nonzero(op.covered)[0], 3000, replace=False)
    ref = np.zeros((len(pick), I))
    mag = np.zeros((len(pick), I))
    for k, r in enumerate(pick):
        cols = og.data_cells[A.indices[A.indptr[r]:A.indptr[r + 1]]]
        w = A.data[A.indptr[r]:A.indptr[r + 1]]
        ref[k] = w @ full[cols]
        mag[k] = np.abs(w) @ np.abs(full[cols])
    cells = torch.from_numpy(G[pick]).cuda()
    src = torch.from_numpy(full).cuda()
    del full
    for windows in (True, False):
        plan = hb.Plan(prog, inner=I, dtype=hb.F64, windows=windows)
        st = plan.stats()
        assert (st["rows_window"] > 0) == windows
        x = src.clone()
        hb.apply(plan, x)
        torch.cuda.synchronize()
        got = x[cells].cpu().numpy()
        del x
        bound = 1e-13 * np.maximum(np.abs(ref), mag)
        assert (np.abs(got - ref) <= bound).all(), (windows, float((np.abs(got - ref) / bound).max()))
    # the adjoint: src as ybar (random, so every covered ghost carries a value)
    yb = src.cpu().numpy()
    Acsc = A.tocsc()
    read = np.nonzero(np.diff(Acsc.indptr))[0]  # data columns some ghost reads
    dpick = rng.choice(read, 3000, replace=False)
    aref = np.zeros((len(dpick), I))
    amag = np.zeros((len(dpick), I))
    cnt = np.diff(Acsc.indptr)[dpick]
    for k, j in enumerate(dpick):
        rows = Acsc.indices[Acsc.indptr[j]:Acsc.indptr[j + 1]]
        w = Acsc.data[Acsc.indptr[j]:Acsc.indptr[j + 1]]
        c = og.data_cells[j]
        aref[k] = yb[c] + w @ yb[G[rows]]
        amag[k] = np.abs(yb[c]) + np.abs(w) @ np.abs(yb[G[rows]])
    del yb
    dcells = torch.from_numpy(og.data_cells[dpick]).cuda()
    for windows in (True, False):
        plan = hb.Plan(prog, inner=I, dtype=hb.F64, windows=windows)
        y = src.clone()
        hb.apply_adjoint(plan, y)
        torch.cuda.synchronize()
        assert (y[cells] == 0).all()
        got = y[dcells].cpu().numpy()
        del y
        bound = (cnt[:, None] + 2) * U64 * amag
        assert (np.abs(got - aref) <= bound).all(), (windows, float((np.abs(got - aref) / bound).max()))
