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
