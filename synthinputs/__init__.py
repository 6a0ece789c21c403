"""Seeded synthetic inputs shared by the CPU reference and the GPU tests.

This module only draws numbers and samples test fields on grid points. It
holds none of the boundary-condition arithmetic (no ghost maps, no
interpolation weights, no operator assembly): both the CPU reference and the
GPU path receive the arrays produced here as plain inputs.

Recipes (each seeded with ``numpy.random.default_rng(seed)``):

* ``cs_sh_field``: on the equiangular gnomonic cubed sphere, every
  (field, level) slot is an independent sum of 4 real orthonormal spherical
  harmonics.  Per term: degree ``l ~ U{1..8}``, order ``m ~ U{-l..l}``,
  coefficient ``~ N(0, 1)``; evaluated as point values at the normalised
  cell-centre positions.  Optional additive ``N(0, noise)`` per value.
  Inner slot order is ``[field][level]`` (level fastest).
* ``uniform``: ``U(-1, 1)``.
* ``batch_draw``: per grid ``N ~ U{48, 96, 192, 384, 768}``, halo
  ``h ~ U{2, 3, 4}``, levels ``L ~ U{1..128}``.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import sph_harm_y

# Face frames (centre, first tangent axis, second tangent axis) of the cube,
# each right-handed (centre x first = second).  Defines where the test field
# is sampled.
_FRAMES = np.array(
    [
        [[1, 0, 0], [0, 1, 0], [0, 0, 1]],
        [[0, 1, 0], [-1, 0, 0], [0, 0, 1]],
        [[-1, 0, 0], [0, -1, 0], [0, 0, 1]],
        [[0, -1, 0], [1, 0, 0], [0, 0, 1]],
        [[0, 0, 1], [0, 1, 0], [-1, 0, 0]],
        [[0, 0, -1], [0, 1, 0], [1, 0, 0]],
    ],
    dtype=np.float64,
)


def cs_cell_centres(N: int) -> np.ndarray:
    """Unit vectors of the data-cell centres, shape (6, N, N, 3), index (face, j, i).

    ``i`` runs along the first tangent axis (angle alpha), ``j`` along the
    second (angle beta); centre angles are ``-pi/4 + (k + 1/2) * pi / (2N)``.
    """
    ang = -np.pi / 4 + (np.arange(N) + 0.5) * (np.pi / (2 * N))
    ta = np.tan(ang)
    out = np.empty((6, N, N, 3))
    for f in range(6):
        c, e1, e2 = _FRAMES[f]
        p = c[None, None, :] + ta[None, :, None] * e1[None, None, :] + ta[:, None, None] * e2[None, None, :]
        out[f] = p / np.linalg.norm(p, axis=-1, keepdims=True)
    return out


def real_sh(l: int, m: int, pts: np.ndarray) -> np.ndarray:
    """Real orthonormal spherical harmonic Y_lm at unit vectors ``pts`` (..., 3)."""
    polar = np.arccos(np.clip(pts[..., 2], -1.0, 1.0))
    azim = np.arctan2(pts[..., 1], pts[..., 0])
    y = sph_harm_y(l, abs(m), polar, azim)
    if m > 0:
        return np.sqrt(2.0) * y.real
    if m < 0:
        return np.sqrt(2.0) * y.imag
    return y.real


def sh_terms(rng: np.random.Generator, nterms: int = 4, lmax: int = 8):
    """Draw ``nterms`` (l, m, coefficient) triples."""
    out = []
    for _ in range(nterms):
        l = int(rng.integers(1, lmax + 1))
        m = int(rng.integers(-l, l + 1))
        c = float(rng.standard_normal())
        out.append((l, m, c))
    return out


def cs_sh_field(N: int, nfields: int = 1, nlevels: int = 1, seed: int = 1,
                noise: float = 0.0, dtype=np.float64) -> np.ndarray:
    """Data values on the cubed sphere, shape (6, N, N, nfields * nlevels).

    Slot ``k = field * nlevels + level`` is an independent 4-term real SH sum
    plus optional ``N(0, noise)`` noise, drawn in slot order from one
    generator.
    """
    rng = np.random.default_rng(seed)
    pts = cs_cell_centres(N)
    nslot = nfields * nlevels
    out = np.empty((6, N, N, nslot), dtype=dtype)
    cache: dict = {}
    for k in range(nslot):
        acc = np.zeros((6, N, N))
        for (l, m, c) in sh_terms(rng):
            key = (l, m)
            if key not in cache:
                cache[key] = real_sh(l, m, pts)
            acc += c * cache[key]
        if noise > 0.0:
            acc += rng.normal(0.0, noise, size=acc.shape)
        out[..., k] = acc
    return out


def uniform(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def normal(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).normal(0.0, scale, size=shape)


def batch_draw(n: int = 64, seed: int = 4):
    """(N, halo, levels) for ``n`` independent cubed-sphere grids."""
    rng = np.random.default_rng(seed)
    sizes = [48, 96, 192, 384, 768]
    out = []
    for _ in range(n):
        N = int(rng.choice(sizes))
        h = int(rng.integers(2, 5))
        L = int(rng.integers(1, 129))
        out.append((N, h, L))
    return out


def _legendre_table(x, lmax):
    """P[l][m] (Condon-Shortley phase) for 0 <= m <= l <= lmax, as torch tensors."""
    import torch
    P = {}
    s = torch.sqrt(torch.clamp(1 - x * x, min=0.0))
    pmm = torch.ones_like(x)
    for m in range(lmax + 1):
        if m > 0:
            pmm = -pmm * (2 * m - 1) * s
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = x * (2 * m + 1) * pmm
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * x * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def cs_cell_centres_torch(N, device, dtype=None):
    """Same points as ``cs_cell_centres``, computed with torch on ``device``."""
    import torch
    dtype = dtype or torch.float64
    fr = torch.tensor(_FRAMES, dtype=dtype, device=device)
    ang = -math.pi / 4 + (torch.arange(N, dtype=dtype, device=device) + 0.5) * (math.pi / (2 * N))
    ta = torch.tan(ang)
    p = (fr[:, 0][:, None, None, :] + ta[None, None, :, None] * fr[:, 1][:, None, None, :]
         + ta[None, :, None, None] * fr[:, 2][:, None, None, :])
    return p / torch.linalg.norm(p, dim=-1, keepdim=True)


def cs_sh_field_torch(N, nfields=1, nlevels=1, seed=1, noise=0.0, device="cuda", dtype=None):
    """``cs_sh_field`` evaluated with torch on ``device`` (same draws, same
    functions; values agree with the numpy version to rounding).  Noise, if
    any, comes from torch's generator seeded with ``seed`` and so differs
    from the numpy version's noise."""
    import torch
    dtype = dtype or torch.float64
    rng = np.random.default_rng(seed)
    pts = cs_cell_centres_torch(N, device)
    x = pts[..., 2].clamp(-1.0, 1.0)
    phi = torch.atan2(pts[..., 1], pts[..., 0])
    P = _legendre_table(x, 8)
    cache = {}

    def Y(l, m):
        key = (l, m)
        if key not in cache:
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            base = norm * P[(l, am)]
            if m > 0:
                cache[key] = math.sqrt(2.0) * base * torch.cos(am * phi)
            elif m < 0:
                cache[key] = math.sqrt(2.0) * base * torch.sin(am * phi)
            else:
                cache[key] = base
        return cache[key]

    nslot = nfields * nlevels
    out = torch.empty((6, N, N, nslot), dtype=dtype, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    for k in range(nslot):
        acc = torch.zeros((6, N, N), dtype=torch.float64, device=device)
        for (l, m, c) in sh_terms(rng):
            acc += c * Y(l, m)
        if noise > 0.0:
            acc += noise * torch.randn(acc.shape, dtype=torch.float64, device=device, generator=gen)
        out[..., k] = acc.to(dtype)
    return out
