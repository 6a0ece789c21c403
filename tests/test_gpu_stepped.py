"""GPU applies on grids of stepped slices (Sec. IV-A-1: staggered variables,
multigrid levels) against the oracle: copies and scaled copies bit-exact,
two-entry interpolation rows within two roundings of sum |w x|."""
import numpy as np
import pytest

from helpers import gpu_available
from oracle import apply as o_apply, assemble
from test_abi_host import _stepped_programs

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_2605_14780_amd as hb


@pytest.mark.parametrize("I,order,dtype", [(1, 0, "f64"), (16, 0, "f64"), (8, 1, "f64"), (32, 0, "f32")])
def test_stepped_grid_apply(I, order, dtype):
    g, p, og, subs = _stepped_programs(nx=9, ny=7)
    dt, npdt, eps = (hb.F64, np.float64, 2.0 ** -53) if dtype == "f64" else (hb.F32, np.float32, 2.0 ** -24)
    plan = hb.Plan(p, inner=I, order=order, dtype=dt)
    rng = np.random.default_rng(I)
    full = rng.standard_normal((og.ncells, I)).astype(npdt)
    op = assemble(og, subs)
    ref = o_apply(op, full.astype(np.float64))
    arr = full if order == 0 else np.ascontiguousarray(full.T)
    t = torch.from_numpy(arr.copy()).cuda()
    hb.apply(plan, t)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    got = (got if order == 0 else np.ascontiguousarray(got.T)).astype(np.float64)
    G, D = og.ghost_cells, og.data_cells
    assert np.array_equal(got[D], full[D].astype(np.float64))
    A = op.dense()
    mag = np.abs(A) @ np.abs(full[D].astype(np.float64)) + (np.abs(op.b) if op.b is not None else 0)
    assert (np.abs(got[G] - ref[G]) <= 2 * eps * mag).all()
    one_entry = (np.abs(A) > 0).sum(axis=1) <= 1
    # copies, copies scaled by -0.5, zeros and uncovered rows are exact in both precisions
    assert np.array_equal(got[G][one_entry & ~op.has_b], ref[G][one_entry & ~op.has_b])
