"""Analytic velocity fields of the paper's tests (oracle; test infrastructure only).

v(x, t) = A v0(x) g(t):
  uniform        v0 = u0, g = 1
  rotation       v0 = (c_y - y, x - c_x) about c = (u0[0], u0[1]), g = 1
                 (§4.1: Zalesak c = (0.5, 0.5), Rudman c = (2, 2))
  single vortex  v0 = (-sin^2(pi x) sin(2 pi y), sin(2 pi x) sin^2(pi y)),
                 g = cos(pi t / T)                                    (§4.2, Rider-Kothe)
  LeVeque 3D     v0 = (2 sin^2(pi x) sin(2 pi y) sin(2 pi z),
                       -sin(2 pi x) sin^2(pi y) sin(2 pi z),
                       -sin(2 pi x) sin(2 pi y) sin^2(pi z)),
                 g = cos(pi t / T)                                    (§4.3)
"""
from __future__ import annotations

import math

import torch

UNIFORM, ROTATION, SINGLE_VORTEX, LEVEQUE3D = 0, 1, 2, 3


def time_factor(kind: int, t: float, period: float) -> float:
    if kind in (SINGLE_VORTEX, LEVEQUE3D):
        return math.cos(math.pi * t / period)
    return 1.0


def spatial(kind: int, x: torch.Tensor, u0=(0.0, 0.0, 0.0)) -> torch.Tensor:
    """v0(x) for coordinates x[..., d]."""
    d = x.shape[-1]
    pi = math.pi
    if kind == UNIFORM:
        return torch.stack([torch.full_like(x[..., k], float(u0[k])) for k in range(d)], -1)
    if kind == ROTATION:
        if d != 2:
            raise ValueError("rotation field is 2D")
        return torch.stack([float(u0[1]) - x[..., 1], x[..., 0] - float(u0[0])], -1)
    if kind == SINGLE_VORTEX:
        if d != 2:
            raise ValueError("single vortex is 2D")
        X, Y = x[..., 0], x[..., 1]
        return torch.stack([-torch.sin(pi * X) ** 2 * torch.sin(2 * pi * Y),
                            torch.sin(2 * pi * X) * torch.sin(pi * Y) ** 2], -1)
    if kind == LEVEQUE3D:
        if d != 3:
            raise ValueError("LeVeque field is 3D")
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        return torch.stack([2 * torch.sin(pi * X) ** 2 * torch.sin(2 * pi * Y) * torch.sin(2 * pi * Z),
                            -torch.sin(2 * pi * X) * torch.sin(pi * Y) ** 2 * torch.sin(2 * pi * Z),
                            -torch.sin(2 * pi * X) * torch.sin(2 * pi * Y) * torch.sin(pi * Z) ** 2], -1)
    raise ValueError(f"unknown velocity kind {kind}")


def velocity(kind, x, t, amp, period, u0=(0.0, 0.0, 0.0)):
    """A v0(x) g(t); ``amp`` may be a float or a 0-d tensor (for gradients in A)."""
    return amp * spatial(kind, x, u0) * time_factor(kind, t, period)
