"""The torch evaluation of the seeded spherical-harmonic inputs equals the
numpy / scipy one (same draws, same functions)."""
import numpy as np
import torch

import synthinputs


def test_torch_sh_field_equals_numpy():
    a = synthinputs.cs_sh_field(7, 2, 3, seed=9)
    b = synthinputs.cs_sh_field_torch(7, 2, 3, seed=9, device="cpu").numpy()
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_batch_draw_ranges():
    d = synthinputs.batch_draw()
    assert len(d) == 64
    assert all(N in (48, 96, 192, 384, 768) and 2 <= h <= 4 and 1 <= L <= 128 for N, h, L in d)
