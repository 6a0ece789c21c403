"""Seeded random BC programs on small multi-block grids, every cell against
the oracle: forward, adjoint, new b values on the compiled plans, random
consumer stencils read after them, and a batch of them; and HIP-graph
replays of their forward and adjoint against the eager calls.

Each case draws a grid of 1-3 blocks (a leading block coordinate and a 2-D
box with a halo of 1-3 cells), fills every ghost strip and corner of every
block with one randomly chosen basic sub-matrix (Sec. IV-A-3, Tables II/III):

* a periodic copy or a mirror from the block's own data region, or a copy
  from another block's data region, with a random weight and, for vector
  layouts, a random component rotation;
* zero rows;
* ELL rows of width 1-6 or CSR rows of 0-12 entries reading random data
  cells of any block, with random weights (and rotation);
* nothing (the ghosts stay as they are),

adds a sub-vector b (one value per row, or one per inner slot, the same
width throughout a program) to some of the boxes, and compiles the program
for a random layout: inner extent, point- or plane-major, FP64 or FP32,
sliding windows allowed or not.  The oracle assembles the same sub-matrices and sub-vectors from their
definitions.  Data cells and uncovered ghosts must come back unchanged, and
every covered ghost value must lie within 32 roundings of
sum |A| |x| + |b| (taken through the row's component rotation) of the
oracle's value.
"""
import numpy as np
import pytest

from helpers import gpu_available, magnitude_operator
from oracle import MapSub, RowsSub, VectorSub, ZeroSub, apply as o_apply, assemble
from oracle.grid import Grid as OGrid

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    import paper_2605_14780_amd as hb

ROTS = [(1, 0, 0, 1), (0, 1, 1, 0), (-1, 0, 0, 1), (1, 0, 0, -1), (-1, 0, 0, -1), (0, -1, 1, 0), (0, 1, -1, 0),
        (0, -1, -1, 0)]
KINDS = ["periodic", "mirror", "other", "zero", "ell", "csr", "none"]


def draw_case(seed, force_dtype=None, force_order=None, force_shape=None):
    """One random case; force_shape = (halo, n0, n1) fixes the block shape."""
    rng = np.random.default_rng(seed)
    nb = int(rng.integers(1, 4))
    h = int(rng.integers(1, 4))
    n = [int(rng.integers(max(h, 4), 20)), int(rng.integers(max(h, 4), 24))]
    if force_shape is not None:
        h, n = force_shape[0], list(force_shape[1:])
    lo, hi = [0, -h, -h], [nb, n[0] + h, n[1] + h]
    g = hb.Grid(lo, hi)
    og = OGrid(lo, hi)
    for k in range(nb):
        full = [(k, k + 1), (-h, n[0] + h), (-h, n[1] + h)]
        data = [(k, k + 1), (0, n[0]), (0, n[1])]
        g.add_block(full, data)
        og.add_block(full, data)
    I = int(rng.choice([1, 2, 3, 4, 5, 8, 12, 16, 31, 32, 64, 96]))
    vec = (0, I // 2, I // 2) if I % 2 == 0 and rng.random() < 0.5 else None
    order = int(rng.integers(0, 2))
    dtype = "f64" if rng.random() < 0.5 else "f32"
    order = order if force_order is None else force_order
    dtype = dtype if force_dtype is None else force_dtype
    windows = bool(rng.random() < 0.7)
    nin = 1 if rng.random() < 0.5 else I  # b values per row (one width for the whole program)
    W0, W1 = n[0] + 2 * h, n[1] + 2 * h

    def cell(k, x, y):  # the library's linear cell index (blocks in order, full boxes row-major)
        return (k * W0 + (x + h)) * W1 + (y + h)

    prog = hb.Program(g)
    subs = []
    vectors = []  # (sub-vector id, index in subs, values shape)
    # the ghost region of a block: 4 strips and 4 corners
    spans = [[(-h, 0), (0, n[d]), (n[d], n[d] + h)] for d in range(2)]
    for k in range(nb):
        for sx in range(3):
            for sy in range(3):
                if sx == 1 and sy == 1:
                    continue
                rows = [(k, k + 1), spans[0][sx], spans[1][sy]]
                box_cells = [(k, x, y) for x in range(*rows[1]) for y in range(*rows[2])]
                kind = str(rng.choice(KINDS))
                if kind == "other" and nb == 1:
                    kind = "periodic"
                rot = ROTS[int(rng.integers(0, 8))] if vec is not None and rng.random() < 0.4 else None
                if kind in ("periodic", "mirror", "other"):
                    M = np.eye(3, dtype=np.int64)
                    off = np.zeros(3, dtype=np.int64)
                    if kind == "other":
                        off[0] = int(rng.choice([j for j in range(nb) if j != k])) - k
                    for d, s in ((1, sx), (2, sy)):
                        nd = n[d - 1]
                        if s == 1:
                            continue
                        if kind == "mirror":  # reflect about the block's face
                            M[d, d] = -1
                            off[d] = -1 if s == 0 else 2 * nd - 1
                        else:  # wrap into the data region
                            off[d] = nd if s == 0 else -nd
                    w = float(rng.choice([1.0, rng.standard_normal()]))
                    prog.add_map(rows, M, off, weight=w, rot=rot)
                    subs.append(MapSub(rows, lambda c, M=M, off=off: tuple(int(v) for v in M @ np.array(c) + off),
                                       w, rot))
                elif kind == "zero":
                    prog.add_zero(rows)
                    subs.append(ZeroSub(rows))
                elif kind in ("ell", "csr"):
                    width = int(rng.integers(1, 7))
                    ents, cols, vals, ptr = {}, [], [], [0]
                    for c in box_cells:
                        m = width if kind == "ell" else int(rng.integers(0, 13))
                        e = []
                        for _ in range(m):
                            kk = int(rng.integers(0, nb))
                            x, y = int(rng.integers(0, n[0])), int(rng.integers(0, n[1]))
                            wv = float(rng.standard_normal())
                            e.append(((kk, x, y), wv))
                            cols.append(cell(kk, x, y))
                            vals.append(wv)
                        ptr.append(len(cols))
                        ents[c] = e
                    if kind == "ell":
                        prog.add_ell(rows, width, cols, vals, rot=rot)
                    else:
                        prog.add_csr(rows, ptr, cols, vals, rot=rot)
                    subs.append(RowsSub(rows, lambda c, ents=ents: ents[tuple(c)], rot))
                if rng.random() < 0.4:
                    b = rng.standard_normal((len(box_cells), nin))
                    sid = prog.add_vector(rows, b, ninner=nin)
                    subs.append(VectorSub(rows, b if nin > 1 else b[:, 0]))
                    vectors.append((sid, len(subs) - 1, b.shape))
    return g, og, prog, subs, I, vec, order, dtype, windows, rng, vectors


@pytest.mark.parametrize("seed", range(24))
def test_random_program_matches_oracle(seed):
    g, og, prog, subs, I, vec, order, dtype, windows, rng, vectors = draw_case(seed)
    dt, npdt, eps = (hb.F64, np.float64, 2.0 ** -53) if dtype == "f64" else (hb.F32, np.float32, 2.0 ** -24)
    plan = hb.Plan(prog, inner=I, order=order, vec=vec, dtype=dt, windows=windows)
    op = assemble(og, subs)
    u = rng.standard_normal((og.ncells, I)).astype(npdt).astype(np.float64)  # inputs as the GPU holds them
    arr = u if order == 0 else np.ascontiguousarray(u.T)
    t = torch.from_numpy(np.ascontiguousarray(arr.astype(npdt))).cuda()
    hb.apply(plan, t)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.float64)
    got = got if order == 0 else np.ascontiguousarray(got.T)
    ref = o_apply(op, u, vec)
    D, G = og.data_cells, og.ghost_cells
    assert np.array_equal(got[D], u[D])
    cov = G[op.covered]
    assert np.array_equal(got[G[~op.covered]], u[G[~op.covered]])
    mag = o_apply(magnitude_operator(op), np.abs(u), vec)[cov]  # sum |A| |x| + |b| per value
    err = np.abs(got[cov] - ref[cov])
    bad = np.argwhere(err > 32 * eps * mag)
    assert bad.size == 0, (seed, I, vec, order, dtype, windows, bad[:3].tolist(),
                           [og.coord_of_cell(int(cov[r])) for r, _ in bad[:3]])


@pytest.mark.parametrize("seed", range(24))
def test_random_program_adjoint_matches_oracle(seed):
    """The adjoint of the same random programs against the oracle's VJP
    (data cells gain A^T of the covered ghosts' values, covered ghosts
    become 0, uncovered ghosts keep theirs): every value within
    (entries of its column + 4) roundings of |ybar| + |A|^T |ybar| (through
    the rotations' permutations)."""
    from oracle import vjp
    g, og, prog, subs, I, vec, order, dtype, windows, rng, vectors = draw_case(seed)
    dt, npdt, eps = (hb.F64, np.float64, 2.0 ** -53) if dtype == "f64" else (hb.F32, np.float32, 2.0 ** -24)
    plan = hb.Plan(prog, inner=I, order=order, vec=vec, dtype=dt, windows=windows)
    op = assemble(og, subs)
    yb = rng.standard_normal((og.ncells, I)).astype(npdt).astype(np.float64)
    arr = yb if order == 0 else np.ascontiguousarray(yb.T)
    t = torch.from_numpy(np.ascontiguousarray(arr.astype(npdt))).cuda()
    hb.apply_adjoint(plan, t)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.float64)
    got = got if order == 0 else np.ascontiguousarray(got.T)
    ref = vjp(op, yb, vec)
    D, G = og.data_cells, og.ghost_cells
    assert (got[G[op.covered]] == 0).all()
    assert np.array_equal(got[G[~op.covered]], yb[G[~op.covered]])
    mag = vjp(magnitude_operator(op), np.abs(yb), vec)[D]
    cnt = 0
    for A in op.parts.values():
        cnt = cnt + np.diff(A.tocsc().indptr)  # entries per source (column)
    err = np.abs(got[D] - ref[D])
    bad = np.argwhere(err > (np.asarray(cnt)[:, None] + 4) * eps * mag)
    assert bad.size == 0, (seed, I, vec, order, dtype, bad[:3].tolist())


@pytest.mark.parametrize("seed", range(16))
def test_random_consumer_matches_oracle(seed):
    """A random stencil (1-9 offsets within the halo, repeats allowed, random
    weights) read after the same random programs (point-major), fused and
    unfused, against the oracle's stencil over its BC: every value within 64
    roundings of sum_o |w_o| T[c + o] (T = |u| on data cells and uncovered
    ghosts, sum |A| |x| + |b| on covered ones).  Uncovered ghosts are read as
    stored by both."""
    from oracle.consumer import stencil_after_bc
    g, og, prog, subs, I, vec, _, dtype, windows, rng, _ = draw_case(1000 + seed)
    h = -og.blocks[0].full[1][0]
    noff = int(rng.integers(1, 10))
    offs = [(0, int(rng.integers(-h, h + 1)), int(rng.integers(-h, h + 1))) for _ in range(noff)]
    if rng.random() < 0.5:  # a stencil on lines of the last dimension (the line walk)
        offs = [(0, o[1], max(-1, min(1, o[2]))) for o in offs]
    wts = [float(v) for v in rng.standard_normal(noff)]
    dt, npdt, tdt, eps = ((hb.F64, np.float64, torch.float64, 2.0 ** -53) if dtype == "f64"
                          else (hb.F32, np.float32, torch.float32, 2.0 ** -24))
    plan = hb.Plan(prog, inner=I, vec=vec, dtype=dt, windows=windows)
    cons = hb.Consumer(plan, offs, wts)
    op = assemble(og, subs)
    u = rng.standard_normal((og.ncells, I)).astype(npdt).astype(np.float64)
    ndata = len(og.data_cells)
    ref = stencil_after_bc(op, u, offs, wts, vec)
    T = o_apply(magnitude_operator(op), np.abs(u), vec)
    bound = 64 * eps * stencil_after_bc(assemble(og, []), T, offs, [abs(v) for v in wts])
    for fused in (False, True):
        x = torch.from_numpy(u.astype(npdt)).cuda()
        if not fused:
            hb.apply(plan, x)
        y = torch.full((ndata * I,), float("nan"), dtype=tdt, device="cuda")
        cons.apply(x, y, fused=fused)
        torch.cuda.synchronize()
        got = y.view(ndata, I).cpu().numpy().astype(np.float64)
        assert np.isfinite(got).all(), fused
        bad = np.argwhere(np.abs(got - ref) > bound)
        assert bad.size == 0, (seed, fused, offs, I, vec, dtype, bad[:3].tolist())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_random_programs_in_one_batch(dtype):
    """Six random programs (point-major, one dtype) applied as one batch: the
    general-row instance of the batch kernel (ELL of other widths, CSR rows,
    maps, zero rows, b).  Every launch shape gives the same bits; they equal
    the plan's plain apply (except where the plain apply sends CSR rows of
    >= 8 entries and < 32 bytes to the entry-splitting kernel, whose sum is
    ordered differently), and the oracle within the forward test's bound."""
    dt, npdt, tdt, eps = ((hb.F64, np.float64, torch.float64, 2.0 ** -53) if dtype == "f64"
                          else (hb.F32, np.float32, torch.float32, 2.0 ** -24))
    cases = [draw_case(3000 + k, force_dtype=dtype, force_order=0) for k in range(6)]
    plans, inputs, ops, vecs = [], [], [], []
    for (g, og, prog, subs, I, vec, _, _, windows, rng, _) in cases:
        plans.append(hb.Plan(prog, inner=I, vec=vec, dtype=dt, windows=windows))
        u = rng.standard_normal((og.ncells, I)).astype(npdt)
        inputs.append(torch.from_numpy(u).cuda())
        ops.append((og, assemble(og, subs), u.astype(np.float64)))
        vecs.append(vec)
    want = []
    for plan, x in zip(plans, inputs):
        y = x.clone()
        hb.apply(plan, y)
        want.append(y)
    same_order = [p.stats()["rows_narrow"] == 0 for p in plans]
    assert any(same_order) and not all(same_order)
    batch = hb.Batch(plans)
    fields = [x.clone() for x in inputs]
    batch.bind(fields)
    first = None
    for tune in [None, dict(block=128, lanes_per_row=32, rows_per_tile=0, persistent=0),
                 dict(block=256, lanes_per_row=0, rows_per_tile=4096, persistent=300),
                 dict(block=64, lanes_per_row=0, rows_per_tile=64, persistent=0)]:
        if tune is not None:
            batch.tune = tune
        for f, x in zip(fields, inputs):
            f.copy_(x)
        batch.apply()
        torch.cuda.synchronize()
        if first is None:
            first = [f.clone() for f in fields]
        for k, (f, w, f0) in enumerate(zip(fields, want, first)):
            assert torch.equal(f, f0), (k, tune)
            if same_order[k]:
                assert torch.equal(f, w), (k, tune)
    for f, (og, op, u), vec in zip(fields, ops, vecs):
        got = f.cpu().numpy().astype(np.float64)
        ref = o_apply(op, u, vec)
        cov = og.ghost_cells[op.covered]
        mag = o_apply(magnitude_operator(op), np.abs(u), vec)[cov]
        assert (np.abs(got[cov] - ref[cov]) <= 32 * eps * mag).all()


@pytest.mark.parametrize("seed", range(12))
def test_random_program_new_b_values(seed):
    """New values for every sub-vector of a compiled random program
    (set_vector, Sec. III-B's affine part changing between applies): the next
    apply equals the oracle's operator assembled with the new values, within
    the forward test's bound."""
    g, og, prog, subs, I, vec, order, dtype, windows, rng, vectors = draw_case(seed)
    if not vectors:
        pytest.skip("this draw has no sub-vector")
    dt, npdt, eps = (hb.F64, np.float64, 2.0 ** -53) if dtype == "f64" else (hb.F32, np.float32, 2.0 ** -24)
    plan = hb.Plan(prog, inner=I, order=order, vec=vec, dtype=dt, windows=windows)
    subs = list(subs)
    for sid, k, shape in vectors:
        nb = rng.standard_normal(shape)
        plan.set_vector(sid, nb)
        subs[k] = VectorSub(subs[k].rows, nb if shape[1] > 1 else nb[:, 0])
    op = assemble(og, subs)
    u = rng.standard_normal((og.ncells, I)).astype(npdt).astype(np.float64)
    arr = u if order == 0 else np.ascontiguousarray(u.T)
    t = torch.from_numpy(np.ascontiguousarray(arr.astype(npdt))).cuda()
    hb.apply(plan, t)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.float64)
    got = got if order == 0 else np.ascontiguousarray(got.T)
    ref = o_apply(op, u, vec)
    cov = og.ghost_cells[op.covered]
    mag = o_apply(magnitude_operator(op), np.abs(u), vec)[cov]
    assert (np.abs(got[cov] - ref[cov]) <= 32 * eps * mag).all()


@pytest.mark.parametrize("seed", range(8))
def test_random_program_graph_replays(seed):
    """Forward and adjoint of random programs captured in HIP graphs: three
    replays, with eager copies and synchronisations between them, each equal
    bit for bit to the eager call (the adjoint's reader counters are
    restored by every call, so a replay starts from the same state)."""
    g, og, prog, subs, I, vec, order, dtype, windows, rng, _ = draw_case(5000 + seed)
    dt, npdt = (hb.F64, np.float64) if dtype == "f64" else (hb.F32, np.float32)
    plan = hb.Plan(prog, inner=I, order=order, vec=vec, dtype=dt, windows=windows)
    u = rng.standard_normal((og.ncells, I)).astype(npdt)
    arr = u if order == 0 else np.ascontiguousarray(u.T)
    src = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for op_kind, eager in ((hb.OP_APPLY, hb.apply), (hb.OP_ADJOINT, hb.apply_adjoint)):
            want = src.clone()
            eager(plan, want, stream=s.cuda_stream)
            x = src.clone()
            graph = hb.ApplyGraph(plan, [x], 1, stream=s.cuda_stream, op=op_kind)
            for rep in range(3):
                x.copy_(src)
                torch.cuda.synchronize()
                graph.launch(stream=s.cuda_stream)
                torch.cuda.synchronize()
                assert torch.equal(x, want), (op_kind, rep)
            del graph


@pytest.mark.parametrize("shape", [(1, 5, 1), (1, 3, 2), (2, 2, 3), (1, 1, 1)])
def test_random_consumer_on_thin_blocks(shape):
    """Blocks of 1-3 data cells along a dimension (runs of one or two cells,
    every stencil reaching the halo): random programs and the cross and
    9-point box (the line walk) and a stencil with a repeated offset (the
    general walk), fused and unfused, against the oracle."""
    from oracle.consumer import stencil_after_bc
    h = shape[0]
    stencils = [[(0, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)],
                [(0, a, b) for a in (-1, 0, 1) for b in (-1, 0, 1)],
                [(0, h, -h), (0, 0, 0), (0, -h, h), (0, 0, 0)]]  # a repeated offset: the general walk
    for k, offs in enumerate(stencils):
        g, og, prog, subs, I, vec, _, dtype, windows, rng, _ = draw_case(7000 + 10 * k + sum(shape), force_order=0,
                                                                         force_shape=shape)
        wts = [float(v) for v in rng.standard_normal(len(offs))]
        dt, npdt, tdt, eps = ((hb.F64, np.float64, torch.float64, 2.0 ** -53) if dtype == "f64"
                              else (hb.F32, np.float32, torch.float32, 2.0 ** -24))
        plan = hb.Plan(prog, inner=I, vec=vec, dtype=dt, windows=windows)
        cons = hb.Consumer(plan, offs, wts)
        op = assemble(og, subs)
        u = rng.standard_normal((og.ncells, I)).astype(npdt).astype(np.float64)
        ndata = len(og.data_cells)
        ref = stencil_after_bc(op, u, offs, wts, vec)
        T = o_apply(magnitude_operator(op), np.abs(u), vec)
        bound = 64 * eps * stencil_after_bc(assemble(og, []), T, offs, [abs(v) for v in wts])
        for fused in (False, True):
            x = torch.from_numpy(u.astype(npdt)).cuda()
            if not fused:
                hb.apply(plan, x)
            y = torch.full((ndata * I,), float("nan"), dtype=tdt, device="cuda")
            cons.apply(x, y, fused=fused)
            torch.cuda.synchronize()
            got = y.view(ndata, I).cpu().numpy().astype(np.float64)
            assert np.isfinite(got).all(), (shape, k, fused)
            assert (np.abs(got - ref) <= bound).all(), (shape, k, fused)


@pytest.mark.parametrize("shape", [(1, 5, 1), (1, 3, 2), (2, 2, 3), (1, 1, 1), (3, 3, 3)])
@pytest.mark.parametrize("k", range(3))
def test_random_program_thin_blocks(shape, k):
    """Random programs on blocks of 1-3 data cells along a dimension (strips
    of one or two rows, runs of one row), random layouts: forward and
    adjoint against the oracle, every cell."""
    from oracle import vjp
    g, og, prog, subs, I, vec, order, dtype, windows, rng, _ = draw_case(8000 + 7 * k + sum(shape),
                                                                         force_shape=shape)
    dt, npdt, eps = (hb.F64, np.float64, 2.0 ** -53) if dtype == "f64" else (hb.F32, np.float32, 2.0 ** -24)
    plan = hb.Plan(prog, inner=I, order=order, vec=vec, dtype=dt, windows=windows)
    op = assemble(og, subs)
    u = rng.standard_normal((og.ncells, I)).astype(npdt).astype(np.float64)
    D, G = og.data_cells, og.ghost_cells
    cov = G[op.covered]
    for adjoint in (False, True):
        arr = u if order == 0 else np.ascontiguousarray(u.T)
        t = torch.from_numpy(np.ascontiguousarray(arr.astype(npdt))).cuda()
        (hb.apply_adjoint if adjoint else hb.apply)(plan, t)
        torch.cuda.synchronize()
        got = t.cpu().numpy().astype(np.float64)
        got = got if order == 0 else np.ascontiguousarray(got.T)
        if not adjoint:
            ref = o_apply(op, u, vec)
            mag = o_apply(magnitude_operator(op), np.abs(u), vec)
            assert np.array_equal(got[D], u[D])
            assert (np.abs(got[cov] - ref[cov]) <= 32 * eps * mag[cov]).all(), (shape, k)
        else:
            ref = vjp(op, u, vec)
            mag = vjp(magnitude_operator(op), np.abs(u), vec)
            cnt = 0
            for A in op.parts.values():
                cnt = cnt + np.diff(A.tocsc().indptr)
            assert (got[cov] == 0).all()
            assert (np.abs(got[D] - ref[D]) <= (np.asarray(cnt)[:, None] + 4) * eps * mag[D]).all(), (shape, k)
        assert np.array_equal(got[G[~op.covered]], u[G[~op.covered]])
