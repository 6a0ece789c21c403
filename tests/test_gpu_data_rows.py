"""GPU checks of data rows (block-edge averaging, Sec. III-B) against the oracle.

A vertex-centred cubed sphere carries a ghost program (rotated copies) and
the averaging rows together; every row of one apply reads the input field, so
the ghosts copy the *un-averaged* source values.  Pairs (weights 1/2) are
exact; triples (weights 1/3) agree within a few units of rounding.
"""
import numpy as np
import pytest

from helpers import gpu_available
from oracle import assemble
from oracle import averaging as oav
from oracle import cubed_sphere as ocs

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_2605_14780_amd as hb


def build(Np, h, I, dtype):
    g = hb.Grid.cubed_sphere(Np, h)
    p = hb.Program(g)
    p.cs_add(Np, h, hb.CS_SYNC)
    p.cs_add_edge_average(Np)
    plan = hb.Plan(p, inner=I, dtype=dtype)
    og = ocs.grid(Np, h)
    op = assemble(og, ocs.subs(Np, h, "sync"))
    dop = oav.assemble_data(og, oav.edge_average_subs(Np))
    return g, plan, og, op, dop


def field(og, I, seed):
    rng = np.random.default_rng(seed)
    u = np.full((og.ncells, I), np.nan)
    u[og.data_cells] = rng.standard_normal((og.ndata, I))
    return u


def bound(dop, og, u, ulps):
    """Per data row: ulps * 2^-53 * sum |w x| (FP64 rounding of the averages)."""
    X = np.abs(u[og.data_cells])
    return ulps * 2.0 ** -53 * (abs(dop.S) @ X)


@pytest.mark.parametrize("Np,h,I", [(9, 2, 5), (16, 3, 8), (4, 1, 1)])
def test_edge_average_with_ghosts_fp64(Np, h, I):
    g, plan, og, op, dop = build(Np, h, I, hb.F64)
    u = field(og, I, Np)
    t = torch.from_numpy(u.copy()).cuda()
    hb.apply(plan, t)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    ref = oav.apply_with_data_rows(op, dop, u)
    G = og.ghost_cells
    # ghosts are copies of the input values: bit-exact
    assert np.array_equal(got[G], ref[G])
    rows = og.data_cells[dop.rows]
    b = bound(dop, og, u, 4)[dop.rows]
    assert (np.abs(got[rows] - ref[rows]) <= b).all()
    pair = np.asarray(dop.S.getnnz(axis=1))[dop.rows] == 2
    assert np.array_equal(got[rows][pair], ref[rows][pair])
    # interior points untouched
    keep = og.data_cells[~dop.rows]
    assert np.array_equal(got[keep], u[keep])


def test_edge_average_fp32_and_graph_replays():
    Np, h, I = 12, 2, 4
    g, plan, og, op, dop = build(Np, h, I, hb.F32)
    u = field(og, I, 7).astype(np.float32)
    src = torch.from_numpy(u.copy()).cuda()
    want = src.clone()
    hb.apply(plan, want)
    torch.cuda.synchronize()
    ref = oav.apply_with_data_rows(op, dop, u.astype(np.float64))
    rows = og.data_cells[dop.rows]
    got = want.cpu().numpy().astype(np.float64)
    assert np.array_equal(got[og.ghost_cells], ref[og.ghost_cells])
    assert np.abs(got[rows] - ref[rows]).max() <= 4 * 2.0 ** -24 * np.nanmax(np.abs(u))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        bufs = [src.clone() for _ in range(2)]
        graph = hb.ApplyGraph(plan, bufs, 2, stream=s.cuda_stream)  # one apply per field
        for rep in range(3):
            for b in bufs:
                b.copy_(src)
            torch.cuda.synchronize()
            graph.launch(s.cuda_stream)
            torch.cuda.synchronize()
            for b in bufs:
                assert torch.equal(b, want), rep


def test_data_rows_refuse_adjoint_and_batch():
    g, plan, og, op, dop = build(6, 1, 2, hb.F64)
    t = torch.zeros(g.cells * 2, dtype=torch.float64, device="cuda")
    with pytest.raises(hb.HbcError) as e:
        hb.apply_adjoint(plan, t)
    assert e.value.code == hb.EUNSUPPORTED
    with pytest.raises(hb.HbcError) as e:
        hb.Batch([plan])
    assert e.value.code == hb.EUNSUPPORTED


@pytest.mark.parametrize("length", [5, 12])
def test_custom_data_rows_chain(length):
    """A cyclic chain of rows (each the mean of itself and its right
    neighbour) forms one component: registers for <= 8 rows, scratch above."""
    Np, h, I = 16, 2, 3
    W = Np + 2 * h
    g = hb.Grid.cubed_sphere(Np, h)
    p = hb.Program(g)
    p.cs_add(Np, h, hb.CS_SYNC)

    def lin(f, j, i):
        return (f * W + (j + h)) * W + (i + h)

    f, j = 2, 5
    cols, ptr, subs_rows, subs_ents = [], [0], [], []
    for i in range(length):
        nxt = (i + 1) % length
        cols += [lin(f, j, 1 + i), lin(f, j, 1 + nxt)]
        ptr.append(len(cols))
        subs_rows.append((f, j, 1 + i))
        subs_ents.append([((f, j, 1 + i), 0.5), ((f, j, 1 + nxt), 0.5)])
    p.add_data_csr([(f, f + 1), (j, j + 1), (1, 1 + length)], ptr, cols, [0.5] * len(cols))
    # a row that reads only cells no data row writes
    p.add_data_csr([(f, f + 1), (j + 2, j + 3), (3, 4)], [0, 2], [lin(f, 0, 0), lin(f, 9, 9)], [0.25, 0.5])
    subs_rows.append((f, j + 2, 3))
    subs_ents.append([((f, 0, 0), 0.25), ((f, 9, 9), 0.5)])
    plan = hb.Plan(p, inner=I)
    og = ocs.grid(Np, h)
    op = assemble(og, ocs.subs(Np, h, "sync"))
    dop = oav.assemble_data(og, [oav.DataRowsSub(subs_rows, subs_ents)])
    u = field(og, I, 21)
    t = torch.from_numpy(u.copy()).cuda()
    hb.apply(plan, t)
    torch.cuda.synchronize()
    ref = oav.apply_with_data_rows(op, dop, u)
    assert np.array_equal(t.cpu().numpy(), ref, equal_nan=True)
