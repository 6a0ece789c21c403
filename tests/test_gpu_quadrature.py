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
