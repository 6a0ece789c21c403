"""The allocation-free adjoint (hbc_apply_adjoint_noalloc) against the
adjoint that owns its counters (hbc_apply_adjoint): the same kernels, so the
bar is bit identity, on consecutive calls over plans of different sizes (the
static counter array keeps the last call's contents), FP64 and FP32; the call
is refused before the plan's transposed tables exist, and repeated calls
leave the device's free memory unchanged."""
import numpy as np
import pytest

from helpers import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_2605_14780_amd as hb


def cs_plan(N, h, nf, nl, dtype):
    I = nf * nl
    vec = (2 * nl, nl, nl) if nf >= 4 else None
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE, vector=vec is not None)
    return grid, hb.Plan(prog, inner=I, vec=vec, dtype=dtype)


def grads(grid, I, tdt, seed):
    gen = torch.Generator(device="cuda").manual_seed(seed)
    return torch.randn(grid.cells * I, dtype=tdt, device="cuda", generator=gen)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_adjoint_matches_adjoint(dtype):
    dt, tdt = (hb.F64, torch.float64) if dtype == "f64" else (hb.F32, torch.float32)
    big = cs_plan(48, 3, 4, 8, dt)      # 32 values per cell
    small = cs_plan(24, 2, 1, 16, dt)   # a smaller grid and field
    for (grid, plan), I in ((big, 32), (small, 16)):
        y = grads(grid, I, tdt, seed=I)
        with pytest.raises(hb.HbcError) as e:       # transposed tables not built yet
            hb.apply_adjoint_noalloc(plan, y.clone())
        assert e.value.code == hb.EINVAL
    # build the tables with the allocating adjoint, keep its results
    want = {}
    for (grid, plan), I, seed in ((big, 32, 1), (small, 16, 2)):
        y = grads(grid, I, tdt, seed)
        ref = y.clone()
        hb.apply_adjoint(plan, ref)
        want[id(plan)] = (y, ref)
    torch.cuda.synchronize()
    # consecutive calls: the larger plan, then the smaller, then the larger again
    for k, (grid, plan) in enumerate((big, small, big, small)):
        y, ref = want[id(plan)]
        got = y.clone()
        hb.apply_adjoint_noalloc(plan, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), k
    # the counter arrays used: the LDS path with shared ghost rows
    assert big[1].stats()["rows_ell"] > 0


def test_noalloc_adjoint_allocates_nothing():
    grid, plan = cs_plan(48, 3, 4, 8, hb.F64)
    y = grads(grid, 32, torch.float64, seed=3)
    ref = y.clone()
    hb.apply_adjoint(plan, ref)
    got = y.clone()
    hb.apply_adjoint_noalloc(plan, got)   # first call on this GPU takes the array's address
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        got.copy_(y)
        hb.apply_adjoint_noalloc(plan, got)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert torch.equal(got, ref)
    # captured in a graph, replayed with eager work in between
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = torch.cuda.CUDAGraph()
        got.copy_(y)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            hb.apply_adjoint_noalloc(plan, got, stream=s.cuda_stream)
        for rep in range(3):
            got.copy_(y)
            hb.apply_adjoint(plan, y.clone())     # eager work on the plan's own counters
            s.synchronize()
            g.replay()
            s.synchronize()
            assert torch.equal(got, ref), rep
