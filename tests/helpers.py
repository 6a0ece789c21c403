"""Shared helpers of the GPU parity tests (build inputs, run both sides, compare)."""
from __future__ import annotations

import dataclasses

import math

import numpy as np

import synthinputs


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def cs_full_field(N, h, nfields, nlevels, seed, noise=0.0, fill=np.nan):
    """Full cubed-sphere field (cells, I), ghosts = fill, data = seeded SH sums."""
    I = nfields * nlevels
    W = N + 2 * h
    full = np.full((6, W, W, I), fill)
    full[:, h:h + N, h:h + N, :] = synthinputs.cs_sh_field(N, nfields, nlevels, seed=seed, noise=noise)
    return full.reshape(-1, I)


def closed_form_weights(N, h):
    """Lagrange bases / weights per (layer, tangential index), written out here
    from the equiangular geometry (used only to feed host-only plan tests)."""
    base = np.zeros(h * N, dtype=np.int32)
    w = np.zeros((h * N, 4))
    D = math.pi / (2 * N)
    for k in range(h):
        ta = math.tan(math.pi / 4 + (k + 0.5) * D)
        for t in range(N):
            tb = math.tan(-math.pi / 4 + (t + 0.5) * D)
            s = (math.atan(tb / ta) + math.pi / 4) / D - 0.5
            if abs(s - round(s)) <= 1e-9:
                s = float(round(s))
            b0 = min(max(math.floor(s) - 1, 0), N - 4)
            d = [s - (b0 + n) for n in range(4)]
            base[k * N + t] = b0
            w[k * N + t] = [-d[1] * d[2] * d[3] / 6, d[0] * d[2] * d[3] / 2, -d[0] * d[1] * d[3] / 2,
                            d[0] * d[1] * d[2] / 6]
    return base, w


def interp_tolerance(ref_op, X_data, key_rows, scale_floor=0.0):
    """Per-row bound 1e-13 * max(|ref|, sum_m |w_m x_m|) (per inner slot)."""
    acc = None
    for A in ref_op.parts.values():
        t = abs(A) @ np.abs(X_data)
        acc = t if acc is None else acc + t
    return acc


def max_rel(got, ref, bound):
    diff = np.abs(got - ref)
    return float(np.max(diff / np.maximum(bound, 1e-300)))


U64 = 2.0 ** -53


def _lagrange_abs_rows(N, h, which):
    """Cubed-sphere Lagrange sub-matrices whose entries are |w_m(s)| ('w') or
    |dw_m/ds| ('dw') at the oracle's own s (component rotations kept)."""
    from oracle import RowsSub, ZeroSub
    from oracle import cubed_sphere as ocs

    def entries(f, j, i):
        g, axis, L, s = ocs.neighbour_line(f, j, i, N)
        base, w, s = ocs.lagrange_weights(s, N)
        d = [s - (base + n) for n in range(4)]
        if which == "w":
            vals = [abs(v) for v in w]
        else:
            vals = [abs((d[1] * d[2] + d[1] * d[3] + d[2] * d[3]) / 6.0),
                    abs((d[0] * d[2] + d[0] * d[3] + d[2] * d[3]) / 2.0),
                    abs((d[0] * d[1] + d[0] * d[3] + d[1] * d[3]) / 2.0),
                    abs((d[0] * d[1] + d[0] * d[2] + d[1] * d[2]) / 6.0)]
        node = (lambda k: (g, k, L)) if axis == "i" else (lambda k: (g, L, k))
        return [(node(base + m), vals[m]) for m in range(4)]

    out = []
    for f in range(6):
        for side in range(4):
            rot = tuple(int(v) for v in ocs.rside(f, side).reshape(-1))
            out.append(RowsSub(ocs.side_box(f, side, N, h), lambda c, f=f: entries(f, c[1], c[2]), rot=rot))
        for box in ocs.corner_boxes(f, N, h):
            out.append(ZeroSub(box))
    return out


def ulp_n(N):
    """Spacing of FP64 numbers in [2^e, 2^(e+1)) holding N: the resolution of a
    fractional index s in [0, N)."""
    return 2.0 ** (math.floor(math.log2(N)) - 52)


# The ghost's position s in the neighbour's index space is a result of FP64
# geometry: the oracle projects the ghost's 3-D point onto the neighbour face
# and takes atan; the library evaluates a closed form with device atan / tan.
# The oracle's own s for one (layer, tangential index) differs across the 24
# face sides by up to 3 ulp(N) (N = 13 ... 768), and the closed form differs
# from the oracle by at most 3 ulp(N): the positions are held to DS_ULPS ulp(N).
DS_ULPS = 4


def lagrange_dw(s, base):
    """d w_m / d s of the 4-node Lagrange basis on nodes base .. base + 3."""
    d = [s - (base + n) for n in range(4)]
    return [-(d[1] * d[2] + d[1] * d[3] + d[2] * d[3]) / 6.0,
            (d[0] * d[2] + d[0] * d[3] + d[2] * d[3]) / 2.0,
            -(d[0] * d[1] + d[0] * d[3] + d[1] * d[3]) / 2.0,
            (d[0] * d[1] + d[0] * d[2] + d[1] * d[2]) / 6.0]


def lagrange_tolerance(N, h, full, ref, vec, rel=1e-13, ds=None):
    """Per-value bound for FP64 interpolated ghosts (ghost rows of the grid).

    rel * max(|ref|, sum_m |w_m x_m|) covers the arithmetic (the plain bound,
    ds=0); the ghost's position s is known to ds (default DS_ULPS ulp(N)),
    which moves the value by ds * sum_m |dw_m/ds| |x_m|.
    """
    from oracle import apply as o_apply, assemble
    from oracle import cubed_sphere as ocs

    ds = DS_ULPS * ulp_n(N) if ds is None else ds
    og = ocs.grid(N, h)
    ax = np.abs(full)
    S = np.abs(o_apply(assemble(og, _lagrange_abs_rows(N, h, "w")), ax, vec))
    G = og.ghost_cells
    tol = rel * np.maximum(np.abs(ref[G]), S[G])
    if ds > 0:
        Dd = np.abs(o_apply(assemble(og, _lagrange_abs_rows(N, h, "dw")), ax, vec))
        tol = tol + ds * Dd[G]
    return tol


def oracle_lagrange_rows(N, h):
    """The oracle's rows of every face side: {(f, side): (box, [entries of each
    row, row-major over the box])}, entries ((g, j, i), w) as the oracle gives them."""
    from oracle import cubed_sphere as ocs
    out = {}
    for f in range(6):
        for side in (ocs.LEFT, ocs.RIGHT, ocs.BOTTOM, ocs.TOP):
            box = ocs.side_box(f, side, N, h)
            out[(f, side)] = (box, [ocs.lagrange_entries(f, j, i, N) for j in range(*box[1])
                                    for i in range(*box[2])])
    return out


def oracle_weights_program(hb, N, h, vector, rows=None, b=None):
    """The cubed-sphere Lagrange BC as a program of basic sub-matrices built
    from the oracle's own columns and weights: one 4-wide ELL sub-matrix per
    face side (with its component rotation when ``vector``), zero corners.
    The library then applies exactly the oracle's A, so its result differs from
    the oracle's only by the arithmetic.  ``b``: optional {box: values} sub-vectors."""
    from oracle import cubed_sphere as ocs
    W = N + 2 * h
    rows = rows if rows is not None else oracle_lagrange_rows(N, h)
    g = hb.Grid.cubed_sphere(N, h)
    p = hb.Program(g)
    for (f, side), (box, ents) in rows.items():
        cols = [(gg * W + (jj + h)) * W + (ii + h) for e in ents for (gg, jj, ii), _ in e]
        vals = [w for e in ents for _, w in e]
        p.add_ell(box, 4, cols, vals, rot=ocs.rside(f, side) if vector else None)
    for f in range(6):
        for box in ocs.corner_boxes(f, N, h):
            p.add_zero(box)
    for box, vals in (b or []):
        p.add_vector(box, vals, ninner=vals.shape[1] if vals.ndim == 2 else 1)
    return g, p


def normwise_error(got_g, ref_g, data):
    """max over inner slots of max|got - ref| / max|data| (per slot)."""
    scale = np.abs(data).max(axis=0)
    return float((np.abs(got_g - ref_g).max(axis=0) / np.where(scale > 0, scale, 1.0)).max())


def magnitude_operator(op):
    """The oracle operator with |A|, |b| and every component rotation's signs
    dropped (a plain permutation of the two components), so that applying it
    to |u| gives sum |a| |x| + |b| for every ghost value, read through the
    same permutation as the value itself.  (Applying |A| with the signed
    rotation would give a negative partial sum for a negated component,
    which |b| then partly cancels.)"""
    parts, rows = {}, {}
    for k, A in op.parts.items():
        ak = None if k is None else tuple(abs(int(v)) for v in k)
        parts[ak] = parts[ak] + abs(A) if ak in parts else abs(A)
        rows[ak] = rows[ak] | op.part_rows[k] if ak in rows else op.part_rows[k].copy()
    return dataclasses.replace(op, parts=parts, part_rows=rows, b=None if op.b is None else np.abs(op.b))
