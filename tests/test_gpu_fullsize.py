"""Full-size GPU checks in the launch configurations the bench times.

* C384, halo 3, 256 inner values (4 fields x 64 levels, (u, v) rotated),
  FP64, after the autotuner has picked the launch shape: sampled ghost rows
  (all 256 values of each; edge strips and corners) against the rows the
  oracle evaluates one by one from the geometry;
* C768, halo 3, 32 levels, with a sub-vector b on every side: the adjoint
  against the forward through the dot-product identity;
* C384 wide interpolation rows (16..25 entries, LDS-staged kernel): sampled
  rows against the oracle's;
* the 64-grid FP32 batch in its autotuned graph launch: bit identity with
  plain applies and sampled rows against the oracle's.
"""
import numpy as np
import pytest

import synthinputs
from helpers import gpu_available
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
        # arithmetic: 1e-13 of sum |w x|; position: the fractional index is
        # known to ~8 N eps and the weights' slopes stay below 4
        ax = np.abs(X).sum(axis=0)
        wx = np.abs(w) @ np.abs(X)
        bnd = 1e-13 * np.maximum(wx, 1e-300) + 8 * N * U64 * 4 * ax
        if dt == hb.F32:  # weight rounding (1 ulp each) and four FP32 roundings of the sum
            bnd = bnd + 8 * 2.0 ** -24 * wx
        bnd_rot = bnd.copy()
        bnd_rot[u_sl] = np.maximum(bnd[u_sl], bnd[v_sl])
        bnd_rot[v_sl] = bnd_rot[u_sl]
        assert (np.abs(got - ref) <= bnd_rot).all(), (f, j, i)
        rows += 1
    assert corners > 0


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
