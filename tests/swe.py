"""Linearised shallow-water step on the cubed sphere (test harness only).

Used only to check gradients through the BC: per face, (alpha, beta) is
treated as a Cartesian grid of spacing dx; metric terms are omitted.
    h_t = -H (d_alpha u + d_beta v),  u_t = -g d_alpha h,  v_t = -g d_beta h
with second-order centred differences (a cross stencil: corner ghosts are
never read) and classic RK4, the BC applied to the full field before every
stage.  Fields are stored point-major, inner slots [h levels | u levels |
v levels], so (u, v) form the layout's vector pair.
"""
from __future__ import annotations


def make_step(bc, N, halo, levels, H=1.0, g=1.0, dx=1.0, dt=0.1):
    import torch

    W = N + 2 * halo
    L = levels
    s = slice(halo, halo + N)

    def tendency(full):
        v = full.view(6, W, W, 3 * L)
        hh, uu, vv = v[..., :L], v[..., L:2 * L], v[..., 2 * L:]

        def d_alpha(x):
            return (x[:, s, halo + 1:halo + N + 1] - x[:, s, halo - 1:halo + N - 1]) / (2 * dx)

        def d_beta(x):
            return (x[:, halo + 1:halo + N + 1, s] - x[:, halo - 1:halo + N - 1, s]) / (2 * dx)

        dh = -H * (d_alpha(uu) + d_beta(vv))
        du = -g * d_alpha(hh)
        dv = -g * d_beta(hh)
        return torch.cat([dh, du, dv], dim=-1)  # (6, N, N, 3L) on data cells

    def add_data(full, k, c):
        v = full.view(6, W, W, 3 * L)
        out = v.clone()
        out[:, s, s, :] = v[:, s, s, :] + c * k
        return out.view(-1, 3 * L)

    def step(u0):
        u1 = bc(u0)
        k1 = tendency(u1)
        u2 = bc(add_data(u1, k1, dt / 2))
        k2 = tendency(u2)
        u3 = bc(add_data(u1, k2, dt / 2))
        k3 = tendency(u3)
        u4 = bc(add_data(u1, k3, dt))
        k4 = tendency(u4)
        return add_data(u1, (k1 + 2 * k2 + 2 * k3 + k4) / 6.0, dt)

    return step
