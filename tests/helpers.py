"""Shared helpers of the GPU parity tests (build inputs, run both sides, compare)."""
from __future__ import annotations

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


def lagrange_tolerance(N, h, full, ref, vec, rel=1e-13):
    """Per-value bound for FP64 interpolated ghosts (ghost rows of the grid).

    rel * max(|ref|, sum_m |w_m x_m|) covers the arithmetic; the ghost's
    position s in the neighbour's index space is itself only known to a few
    N*eps in FP64 (independent atan / tan evaluations), which moves the value by
    ds * sum_m |dw_m/ds| |x_m|; ds = 8 N eps is allowed for that.
    """
    from oracle import apply as o_apply, assemble
    from oracle import cubed_sphere as ocs

    og = ocs.grid(N, h)
    ax = np.abs(full)
    S = np.abs(o_apply(assemble(og, _lagrange_abs_rows(N, h, "w")), ax, vec))
    Dd = np.abs(o_apply(assemble(og, _lagrange_abs_rows(N, h, "dw")), ax, vec))
    G = og.ghost_cells
    return rel * np.maximum(np.abs(ref[G]), S[G]) + 8 * N * U64 * Dd[G]


def normwise_error(got_g, ref_g, data):
    """max over inner slots of max|got - ref| / max|data| (per slot)."""
    scale = np.abs(data).max(axis=0)
    return float((np.abs(got_g - ref_g).max(axis=0) / np.where(scale > 0, scale, 1.0)).max())
