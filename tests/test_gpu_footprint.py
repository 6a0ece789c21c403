"""GPU checks of the consumer footprint (Sec. IV-C): with the consumer's read
offsets declared, the apply writes exactly the live ghosts (equal to the
oracle's restricted operator), leaves the others untouched, and the
consumer's output (a cross sum over the field) is unchanged."""
import numpy as np
import pytest

from helpers import cs_full_field, gpu_available, lagrange_tolerance
from oracle import apply as o_apply, assemble
from oracle import cubed_sphere as ocs
from oracle import footprint as ofp

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_2605_14780_amd as hb


def cross(r):
    out = [(0, 0, 0)]
    for k in range(1, r + 1):
        out += [(0, k, 0), (0, -k, 0), (0, 0, k), (0, 0, -k)]
    return out


def cross_sum(t, N, h, r, I):
    W = N + 2 * h
    v = t.view(6, W, W, I)
    s = slice(h, h + N)
    out = v[:, s, s].clone()
    for k in range(1, r + 1):
        out += v[:, h + k:h + k + N, s] + v[:, h - k:h - k + N, s]
        out += v[:, s, h + k:h + k + N] + v[:, s, h - k:h - k + N]
    return out


@pytest.mark.parametrize("mode,N,h,r,nl", [("sync", 12, 3, 1, 3), ("lagrange", 16, 3, 2, 2)])
def test_footprint_apply(mode, N, h, r, nl):
    nf = 4
    I = nf * nl
    vec = (2 * nl, nl, nl)
    grid, prog = hb.cs_program(N, h, hb.CS_LAGRANGE if mode == "lagrange" else hb.CS_SYNC, vector=True)
    prog.set_consumer(cross(r))
    plan = hb.Plan(prog, inner=I, vec=vec)
    grid_f, prog_f = hb.cs_program(N, h, hb.CS_LAGRANGE if mode == "lagrange" else hb.CS_SYNC, vector=True)
    plan_f = hb.Plan(prog_f, inner=I, vec=vec)
    full = cs_full_field(N, h, nf, nl, seed=8)
    t = torch.from_numpy(full.copy()).cuda()
    tf = torch.from_numpy(full.copy()).cuda()
    hb.apply(plan, t)
    hb.apply(plan_f, tf)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    og = ocs.grid(N, h)
    live = ofp.live_ghost_mask(og, cross(r))
    G = og.ghost_cells
    assert np.isnan(got[G][~live]).all(), "dead ghosts must not be written"
    # live ghosts: the same bits as the plan without a footprint
    assert np.array_equal(got[G][live], tf.cpu().numpy()[G][live])
    op = ofp.restrict(assemble(og, ocs.subs(N, h, mode, vector=True)), live)
    ref = o_apply(op, full, vec)
    if mode == "sync":
        assert np.array_equal(got[G][live], ref[G][live])
    else:
        tol = lagrange_tolerance(N, h, full, o_apply(assemble(og, ocs.subs(N, h, mode, vector=True)), full, vec), vec)
        assert (np.abs(got[G][live] - ref[G][live]) <= tol[live]).all()
    # the consumer sees the same values
    assert torch.equal(cross_sum(t, N, h, r, I), cross_sum(tf, N, h, r, I))
