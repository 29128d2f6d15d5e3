"""P15 (oracle half): the oracle's discrete adjoint (reverse-mode autograd through reset,
pseudo-time preconditioning and the physical RK4 steps) agrees with central finite
differences of the same discrete map, for the initial phi field and for the velocity
amplitude A."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import Oracle


def T(a):
    return torch.as_tensor(a, dtype=torch.float64)


def _setup(d=2, p=3, shape=(4, 4), kind=W.VEL_SINGLE_VORTEX):
    mesh, prm = W.small_case(d, p, shape, vel_kind=kind, vel_period=4.0, precond_iters=3)
    o = Oracle(d, p, mesh, prm)
    x = o.coords()
    centre = (0.5, 0.6) if d == 2 else (0.45, 0.5, 0.55)
    phi0 = T(W.ic_phi(x, centre, 0.3, 0.06))
    target = T(W.ic_phi(x, np.array(centre) + 0.03, 0.3, 0.06))
    return o, prm, phi0, target


def _loss(o, phi0, amp, target, dt, nsteps):
    phi, psi, t = o.run(phi0, None, 0.0, dt, nsteps, amp=amp)
    return 0.5 * o.integral((phi - target) ** 2)


@pytest.mark.parametrize("d", [2, 3])
def test_oracle_adjoint_matches_central_differences(d):
    shape = (4, 4) if d == 2 else (3, 3, 3)
    o, prm, phi0, target = _setup(d, 3 if d == 2 else 2, shape,
                                  W.VEL_SINGLE_VORTEX if d == 2 else W.VEL_LEVEQUE3D)
    dt, nsteps = 0.01, 4
    p0 = phi0.clone().requires_grad_(True)
    A = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    L = _loss(o, p0, A, target, dt, nsteps)
    gphi, gA = torch.autograd.grad(L, (p0, A))
    rng = np.random.default_rng(2)
    v = T(rng.standard_normal(phi0.shape))
    h = 1e-5
    with torch.no_grad():
        Lp = _loss(o, phi0 + h * v, 1.0, target, dt, nsteps)
        Lm = _loss(o, phi0 - h * v, 1.0, target, dt, nsteps)
        fd = float((Lp - Lm) / (2 * h))
        ad = float(torch.sum(gphi * v))
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
        LpA = _loss(o, phi0, 1.0 + h, target, dt, nsteps)
        LmA = _loss(o, phi0, 1.0 - h, target, dt, nsteps)
        fdA = float((LpA - LmA) / (2 * h))
        assert abs(fdA - float(gA)) <= 1e-6 * abs(float(gA)), (fdA, float(gA))
