"""New values for a sub-vector of a compiled plan (Sec. III-B: the affine part
b of F, e.g. a Dirichlet value that changes every step): the apply equals,
bit for bit, that of a plan compiled with the new values, in eager launches
and in a graph captured before the update."""
import numpy as np
import pytest

from helpers import cs_full_field, gpu_available, lagrange_tolerance
from oracle import apply as o_apply, assemble
from oracle import cubed_sphere as ocs
from oracle import VectorSub

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_2605_14780_amd as hb


def _program(N, h, I, b):
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE)
    sid = prog.add_vector(ocs.side_box(2, ocs.BOTTOM, N, h), b, ninner=I)
    return grid, prog, sid


@pytest.mark.parametrize("dtype,order,I", [("f64", "pm", 8), ("f32", "pm", 12), ("f64", "plane", 4),
                                           ("f32", "pm", 7)])
def test_set_vector_equals_a_plan_built_with_the_new_values(dtype, order, I):
    N, h = 16, 3
    dt, npdt = (hb.F64, np.float64) if dtype == "f64" else (hb.F32, np.float32)
    lay = hb.POINT_MAJOR if order == "pm" else hb.PLANE_MAJOR
    rng = np.random.default_rng(I)
    b_old, b_new = rng.standard_normal((N * h, I)), rng.standard_normal((N * h, I))
    grid, prog, sid = _program(N, h, I, b_old)
    plan = hb.Plan(prog, inner=I, order=lay, dtype=dt)
    _, prog_new, _ = _program(N, h, I, b_new)
    fresh = hb.Plan(prog_new, inner=I, order=lay, dtype=dt)
    full = cs_full_field(N, h, 1, I, seed=3).astype(npdt)
    x = full if lay == hb.POINT_MAJOR else np.ascontiguousarray(full.T)
    src = torch.from_numpy(x).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        fields = [src.clone()]
        g = hb.ApplyGraph(plan, fields, 1, stream=s.cuda_stream)  # captured with the old values
        plan.set_vector(sid, b_new, stream=s.cuda_stream)
        a, want = src.clone(), src.clone()
        hb.apply(plan, a, stream=s.cuda_stream)
        hb.apply(fresh, want, stream=s.cuda_stream)
        fields[0].copy_(src)
        g.launch(s.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(a, want)
    assert torch.equal(fields[0], want)
    # and the updated plan agrees with the oracle's operator with the new b
    if dt == hb.F64 and lay == hb.POINT_MAJOR:
        og = ocs.grid(N, h)
        op = assemble(og, ocs.subs(N, h, "lagrange") + [VectorSub(ocs.side_box(2, ocs.BOTTOM, N, h), b_new)])
        ref = o_apply(op, full)
        G = og.ghost_cells
        got = a.cpu().numpy()
        tol = lagrange_tolerance(N, h, full, ref, None)
        assert (np.abs(got[G] - ref[G]) <= tol).all()


def test_set_vector_reaches_a_batch_and_its_graph():
    """A batch holding the plan (and the batch's captured graph) reads the new
    values from its next launch, as a plan compiled with them would give."""
    N, h, I = 12, 2, 5
    rng = np.random.default_rng(11)
    b_old, b_new = rng.standard_normal((N * h, I)), rng.standard_normal((N * h, I))
    grid, prog, sid = _program(N, h, I, b_old)
    plan = hb.Plan(prog, inner=I, dtype=hb.F32)
    other_grid, other_prog = hb.cs_program(16, 3, hb.CS_LAGRANGE)
    other = hb.Plan(other_prog, inner=3, dtype=hb.F32)
    _, prog_new, _ = _program(N, h, I, b_new)
    fresh = hb.Plan(prog_new, inner=I, dtype=hb.F32)
    x = torch.from_numpy(cs_full_field(N, h, 1, I, seed=9).astype(np.float32)).cuda()
    y = torch.from_numpy(cs_full_field(16, 3, 1, 3, seed=10).astype(np.float32)).cuda()
    want = x.clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        hb.apply(fresh, want, stream=s.cuda_stream)
        batch = hb.Batch([plan, other])
        fx, fy = x.clone(), y.clone()
        batch.bind([fx, fy])
        batch.graph_capture(s.cuda_stream)  # captured with the old values
        plan.set_vector(sid, b_new, stream=s.cuda_stream)
        batch.apply(s.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(fx, want)
    with torch.cuda.stream(s):
        fx.copy_(x)
        batch.graph_launch(s.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(fx, want)
