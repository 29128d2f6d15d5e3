"""Pins of the oracle's localized multiplier and of the analytic velocity fields.

Multiplier (§2, Eq. altconservativephasefieldeq: the diffusion and sharpening fluxes are
scaled by max(gamma, |v|) instead of a global velocity bound). For a uniform field v and a
zero jump penalty the phi residual splits exactly into an inviscid part, which is the psi
residual of the same data (psi := phi), and a viscous part that is linear in the
multiplier. Hence

    R_phi(phi, psi; v) - R_psi(phi; v) = max(gamma, |v|) / gamma * R_phi(phi, psi; 0),

where R_psi(phi; v) is the psi row evaluated with psi = phi, and the v = 0 residual has
multiplier max(gamma, 0) = gamma. The identity is checked in both branches of the max
(|v| < gamma and |v| > gamma) on perturbed 2D and 3D meshes.

Velocity fields (§4.2 Rider-Kothe vortex, §4.3 LeVeque deformation): properties the
printed fields have and that a transposed argument, a wrong sign or a wrong factor
breaks: zero divergence, the 2D vortex as the rotated gradient of its stream function
sin^2(pi x) sin^2(pi y) / pi, no flow through the walls of the unit square / cube, the
time reversal v(x, T - t) = -v(x, t), and the peak speed (1 and 2) that sets the time
step.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import Oracle
from oracle import velocity as vel


def T(a):
    return torch.as_tensor(a, dtype=torch.float64)


def _state(o, rng):
    """Smooth interface data: phi a tanh profile of a perturbed distance, psi another
    smooth field (so that the normal from psi differs from grad phi's)."""
    x = o.coords()
    d = x.shape[-1]
    c = np.full(d, 0.5)
    r = np.sqrt(np.sum((x - c) ** 2, axis=-1))
    wob = 0.03 * np.sin(2 * np.pi * x[..., 0]) * np.cos(2 * np.pi * x[..., 1])
    phi = 0.5 * (1.0 + np.tanh((0.3 - r + wob) / 0.05))
    psi = 0.3 - r + 0.05 * np.cos(2 * np.pi * x[..., 1]) + 0.01 * rng.standard_normal(r.shape)
    return T(phi), T(psi)


@pytest.mark.parametrize("d,p,shape", [(2, 3, (5, 4)), (3, 2, (3, 3, 2))])
@pytest.mark.parametrize("speed", [0.05, 0.7])
def test_multiplier_identity(d, p, shape, speed):
    rng = np.random.default_rng(11)
    theta = 0.6
    if d == 2:
        u0 = (speed * math.cos(theta), speed * math.sin(theta), 0.0)
    else:
        u0 = tuple(speed * np.array([math.cos(theta), 0.6 * math.sin(theta), 0.8 * math.sin(theta)]))
    mesh, prm = W.small_case(d, p, shape, perturb=0.2, seed=5, vel_kind=W.VEL_UNIFORM,
                             vel_u0=u0, tau=0.0)
    still = W.small_case(d, p, shape, perturb=0.2, seed=5, vel_kind=W.VEL_UNIFORM,
                         vel_u0=(0.0, 0.0, 0.0), tau=0.0)[1]
    o = Oracle(d, p, mesh, prm)
    o0 = Oracle(d, p, mesh, still)
    phi, psi = _state(o, rng)
    Rphi_v, _ = o.residual(phi, psi, 0.0)
    _, Rinv = o.residual(phi, phi, 0.0)          # the psi row with psi := phi
    Rphi_0, _ = o0.residual(phi, psi, 0.0)
    m = max(prm.gamma, speed)
    lhs = Rphi_v - Rinv
    rhs = (m / prm.gamma) * Rphi_0
    scale = float(rhs.abs().max())
    assert scale > 1e-2                         # the viscous part is not trivially zero
    err = float((lhs - rhs).abs().max()) / scale
    assert err < 1e-12, err


def test_multiplier_is_pointwise_speed():
    """The multiplier is max(gamma, |v|) at each solution and flux point, not one value per
    mesh or per element. Under the rotation field about the centre of an element, |v| is
    the distance to the centre. The viscous part of the phi residual (R_phi minus the psi
    row with psi := phi, tau = 0) is linear in the multiplier, so doubling the amplitude
    doubles it exactly on elements where |v| > gamma at every point (and on every face
    point) and leaves it unchanged on elements where 2|v| < gamma everywhere. A constant
    multiplier fails the first, a global max(gamma, max|v|) the second."""
    d, p, n = 2, 3, 25
    mesh, prm = W.small_case(d, p, (n, n), vel_kind=W.VEL_ROTATION, vel_u0=(0.5, 0.5, 0.0),
                             tau=0.0)
    o = Oracle(d, p, mesh, prm)
    # an interface through the rotation centre, so the slow core carries a viscous flux
    x = o.coords()
    s = (x[..., 0] - 0.5) + 0.3 * (x[..., 1] - 0.5) + 0.02 * np.sin(6 * x[..., 1])
    phi = T(0.5 * (1.0 + np.tanh(s / 0.04)))
    psi = T(s + 0.2 * (x[..., 1] - 0.5) ** 2)

    def visc(A):
        a, _ = o.residual(phi, psi, 0.0, amp=A)
        _, b = o.residual(phi, phi, 0.0, amp=A)
        return a - b

    v1, v2 = visc(1.0), visc(2.0)
    # distance range of each element's box to the centre (a box's farthest point is a
    # corner; its nearest is the projection of the centre)
    lo = mesh.x0
    hi = mesh.x0 + 2.0 * np.einsum("eii->ei", mesh.jac)
    c = np.array([0.5, 0.5])
    far_d = np.sqrt(np.sum(np.maximum(np.abs(lo - c), np.abs(hi - c)) ** 2, axis=1))
    near_d = np.sqrt(np.sum(np.maximum(np.maximum(lo - c, c - hi), 0.0) ** 2, axis=1))
    fast = torch.as_tensor(near_d > prm.gamma)
    slow = torch.as_tensor(2.0 * far_d < prm.gamma)
    assert int(fast.sum()) > 100 and int(slow.sum()) >= 1
    scale = float(v1.abs().max())
    e_fast = float((v2[fast] - 2.0 * v1[fast]).abs().max()) / scale
    slow_scale = float(v1[slow].abs().max())
    assert slow_scale > 1e-4 * scale                       # the slow core is not trivial
    e_slow = float((v2[slow] - v1[slow]).abs().max()) / slow_scale
    assert e_fast < 1e-12, e_fast
    assert e_slow < 1e-12, e_slow


# ----------------------------------------------------------------------------------------
# velocity fields
# ----------------------------------------------------------------------------------------
def _divergence(kind, x):
    x = x.clone().requires_grad_(True)
    v = vel.spatial(kind, x)
    div = torch.zeros(x.shape[0], dtype=torch.float64)
    for k in range(x.shape[1]):
        g, = torch.autograd.grad(v[:, k].sum(), x, retain_graph=True)
        div = div + g[:, k]
    return div.detach(), v.detach()


@pytest.mark.parametrize("kind,d", [(vel.SINGLE_VORTEX, 2), (vel.LEVEQUE3D, 3)])
def test_field_is_divergence_free(kind, d):
    x = T(np.random.default_rng(4).uniform(0.0, 1.0, (4000, d)))
    div, v = _divergence(kind, x)
    assert float(v.abs().max()) > 0.5
    assert float(div.abs().max()) < 1e-12


def test_vortex_is_rotated_stream_function_gradient():
    """u = -ds/dy, v = ds/dx with s = sin^2(pi x) sin^2(pi y) / pi."""
    x = T(np.random.default_rng(5).uniform(0.0, 1.0, (3000, 2))).requires_grad_(True)
    s = torch.sin(math.pi * x[:, 0]) ** 2 * torch.sin(math.pi * x[:, 1]) ** 2 / math.pi
    g, = torch.autograd.grad(s.sum(), x)
    v = vel.spatial(vel.SINGLE_VORTEX, x.detach())
    assert float((v[:, 0] + g[:, 1]).abs().max()) < 1e-14
    assert float((v[:, 1] - g[:, 0]).abs().max()) < 1e-14


@pytest.mark.parametrize("kind,d", [(vel.SINGLE_VORTEX, 2), (vel.LEVEQUE3D, 3)])
def test_no_flow_through_the_walls(kind, d):
    rng = np.random.default_rng(6)
    for k in range(d):
        for side in (0.0, 1.0):
            x = rng.uniform(0.0, 1.0, (500, d))
            x[:, k] = side
            v = vel.spatial(kind, T(x))
            assert float(v[:, k].abs().max()) < 1e-14


@pytest.mark.parametrize("kind,d,period", [(vel.SINGLE_VORTEX, 2, 8.0), (vel.LEVEQUE3D, 3, 3.0)])
def test_time_reversal(kind, d, period):
    x = T(np.random.default_rng(7).uniform(0.0, 1.0, (500, d)))
    for t in (0.0, 0.3, 1.1, 0.5 * period):
        a = vel.velocity(kind, x, t, 1.0, period)
        b = vel.velocity(kind, x, period - t, 1.0, period)
        assert float((a + b).abs().max()) < 1e-14
    # and the field stops at half period
    assert float(vel.velocity(kind, x, 0.5 * period, 1.0, period).abs().max()) < 1e-15


@pytest.mark.parametrize("kind,d,vmax", [(vel.SINGLE_VORTEX, 2, 1.0), (vel.LEVEQUE3D, 3, 2.0)])
def test_peak_speed(kind, d, vmax):
    """The peak |v| the time step is set with (workloads.VMAX) is the field's maximum."""
    assert W.VMAX[kind] == vmax
    g = np.linspace(0.0, 1.0, 41 if d == 3 else 201)
    x = np.stack(np.meshgrid(*([g] * d), indexing="ij"), -1).reshape(-1, d)
    sp = torch.linalg.vector_norm(vel.spatial(kind, T(x)), dim=-1)
    assert float(sp.max()) <= vmax + 1e-12
    assert float(sp.max()) >= vmax - 1e-12       # attained on the grid (x = 1/2, y = 1/4, ...)
