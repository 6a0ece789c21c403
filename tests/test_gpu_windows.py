"""Sliding-window kernel (4-point Lagrange rows of face-edge strips, each
wavefront walking a run of rows along the neighbour's grid line).

Its sum is the general row path's, so the bar is bit identity with a plan of
the same program built with windows=False (the general row kernel), for FP64
and FP32, with and without the component rotation and b, for run lengths from
1 to 64 rows, both orders of loads and stores, and rows of 256 bytes to 2 KiB; the general row path itself is
checked against the oracle elsewhere.  Also: a graph captured before a change
of the launch shape is refused, not replayed over freed tables.
"""
import numpy as np
import pytest

import synthinputs
from helpers import gpu_available
from oracle import cubed_sphere as ocs

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_2605_14780_amd as hb


def cs_pair(N, h, nf, nl, dtype, vector, with_b):
    I = nf * nl
    vec = (2 * nl, nl, nl) if vector else None
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE, vector=vector)
    if with_b:
        rng = np.random.default_rng(N + I)
        for f in (0, 3):
            for side in (ocs.LEFT, ocs.TOP):
                prog.add_vector(ocs.side_box(f, side, N, h), rng.standard_normal((N * h, I)), ninner=I)
        prog.add_vector(ocs.side_box(5, ocs.RIGHT, N, h), rng.standard_normal((N * h, 1)), ninner=1)
    pw = hb.Plan(prog, inner=I, vec=vec, dtype=dtype)
    pr = hb.Plan(prog, inner=I, vec=vec, dtype=dtype, windows=False)
    return grid, pw, pr


def field(N, h, nf, nl, tdt, seed):
    W = N + 2 * h
    I = nf * nl
    full = torch.full((6, W, W, I), float("nan"), dtype=tdt, device="cuda")
    full[:, h:h + N, h:h + N] = synthinputs.cs_sh_field_torch(N, nf, nl, seed=seed, device="cuda").to(tdt)
    return full.reshape(-1)


@pytest.mark.parametrize("N,h,nf,nl,dtype,vector,with_b", [
    (48, 3, 1, 32, "f64", False, False),   # 256-byte rows, the shortest that take windows (without b)
    (40, 3, 4, 16, "f32", True, False),    # 256-byte FP32 rows
    (48, 3, 4, 16, "f64", True, False),    # 512-byte rows
    (48, 3, 4, 16, "f64", True, True),
    (48, 2, 1, 128, "f32", False, True),   # 512-byte FP32 rows
    (96, 3, 4, 32, "f32", True, False),
    (64, 4, 4, 64, "f64", True, True),     # 2 KiB rows, two slices per row
    (37, 3, 4, 24, "f64", True, False),    # odd N, rows of 1.5 slices
    (384, 3, 4, 64, "f64", True, False),   # the C384 workload
    (384, 3, 4, 64, "f32", True, False),
])
def test_window_kernel_bitwise_general_path(N, h, nf, nl, dtype, vector, with_b):
    dt, tdt = (hb.F64, torch.float64) if dtype == "f64" else (hb.F32, torch.float32)
    grid, pw, pr = cs_pair(N, h, nf, nl, dt, vector, with_b)
    st = pw.stats()
    assert st["rows_window"] == st["rows_ell"] > 0 and st["window_runs"] > 0
    assert pr.stats()["rows_window"] == 0
    x = field(N, h, nf, nl, tdt, seed=N)
    want = x.clone()
    hb.apply(pr, want)
    for R in (1, 5, 16, 64):
        for order in (0, 1):  # pipelined and ordered loads and stores
            pw.tune = dict(pw.tune, rows_per_tile=R, window_order=order)
            got = x.clone()
            hb.apply(pw, got)
            torch.cuda.synchronize()
            assert torch.isfinite(got).all(), (R, order)
            assert torch.equal(got, want), (R, order)


def test_window_rows_with_b_from_512_bytes():
    """Segments with b take windows from 512-byte rows, the others from 256:
    at 256 bytes a plan with b on some strips windows only the others, and
    still gives the general path's bits."""
    N, h, nf, nl = 48, 3, 1, 32
    grid, pw, pr = cs_pair(N, h, nf, nl, hb.F64, False, True)
    st = pw.stats()
    assert 0 < st["rows_window"] < st["rows_ell"]
    x = field(N, h, nf, nl, torch.float64, seed=3)
    want, got = x.clone(), x.clone()
    hb.apply(pr, want)
    hb.apply(pw, got)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    grid, pw2, _ = cs_pair(N, h, 4, 16, hb.F64, True, True)  # 512-byte rows: every strip
    st2 = pw2.stats()
    assert st2["rows_window"] == st2["rows_ell"] > 0


def test_window_adjoint_and_graph_after_tuning():
    """The adjoint of a window plan equals the general plan's (same tables);
    a graph captured before set_tune is refused, a new capture runs."""
    N, h, nf, nl = 48, 3, 4, 16
    grid, pw, pr = cs_pair(N, h, nf, nl, hb.F64, True, True)
    gen = torch.Generator(device="cuda").manual_seed(5)
    y = torch.randn(grid.cells * nf * nl, dtype=torch.float64, device="cuda", generator=gen)
    a, b = y.clone(), y.clone()
    hb.apply_adjoint(pw, a)
    hb.apply_adjoint(pr, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    x = field(N, h, nf, nl, torch.float64, seed=9)
    want = x.clone()
    hb.apply(pr, want)
    f = x.clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = hb.ApplyGraph(pw, [f], 2, stream=s.cuda_stream)
        g.launch(s.cuda_stream)
        s.synchronize()
        assert torch.equal(f, want)
        pw.tune = dict(pw.tune, rows_per_tile=7)
        with pytest.raises(hb.HbcError):
            g.launch(s.cuda_stream)
        g2 = hb.ApplyGraph(pw, [f], 2, stream=s.cuda_stream)
        f.copy_(x)
        g2.launch(s.cuda_stream)
        s.synchronize()
        assert torch.equal(f, want)
