"""Pins of the oracle's time integration and whole-run invariants.

P7  mass conservation over a full run (the 16x16, p=3 advection workload, 200 steps).
P10 return of a rotated disk after one revolution (§4.1 velocity field).
P11 classic RK4: the amplification factor of u' = lambda u; P11b its stage times (fourth order
    on a time-dependent field).
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import Oracle
from oracle.solver import rk4


def T(a):
    return torch.as_tensor(a, dtype=torch.float64)


def test_rk4_amplification():
    for lam in (-1.0, -2.3 + 1.1j, 0.5j, 1.7):
        h = 0.37
        z = lam * h
        y = rk4(lambda y: lam * y, 1.0 + 0j, h)
        g = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
        assert abs(y - g) < 1e-15


def test_mass_conserved_over_advection_run():
    cfg = W.config("C1")
    mesh = cfg.mesh()
    o = Oracle(2, 3, mesh, cfg.params)
    phi0 = T(W.ic_phi(o.coords(), cfg.centre, cfg.radius, cfg.params.eps_w))
    phi, psi, t = o.run(phi0, None, 0.0, cfg.dt(mesh), cfg.steps)
    em = float(o.mass_error(phi, phi0, phi0))
    assert abs(em) < 1e-12
    # the translated disk returns to its start after a shift of (1, 0.5)*t: compare
    xs = o.coords()
    exact = T(W.ic_phi(np.mod(xs - np.array([1.0, 0.5]) * t, 1.0), cfg.centre, cfg.radius,
                       cfg.params.eps_w))
    assert float(o.rel_error(phi, exact)) < 0.05


@pytest.mark.slow
def test_rotated_disk_returns():
    """Disk r = 0.15 at (0.5, 0.75) in v = (0.5 - y, x - 0.5), one revolution (t = 2 pi),
    periodic 16x16 mesh, p = 3 (the interface stays far from the boundary; the copy-BC
    ghost state of §3.3 is not stable at inflow boundaries with a central flux). E_m at round-off; E_r of the same order as the paper's
    slotted-disk errors on finer meshes (context, not parity)."""
    N, p = 16, 3
    mesh, prm = W.small_case(2, p, (N, N), periodic=True, vel_kind=W.VEL_ROTATION)
    o = Oracle(2, p, mesh, prm)
    phi0 = T(W.ic_phi(o.coords(), (0.5, 0.75), 0.15, prm.eps_w))
    vmax = math.sqrt(0.5)
    nst = int(math.ceil(2 * math.pi / (0.1 * (1.0 / N) / vmax)))
    dt = 2 * math.pi / nst
    phi, psi, t = o.run(phi0, None, 0.0, dt, nst)
    assert abs(float(o.mass_error(phi, phi0, phi0))) < 1e-12
    er = float(o.rel_error(phi, phi0))
    assert er < 0.2, er


def test_rk4_stage_times_fourth_order_on_time_dependent_field():
    """P11b: classic RK4 evaluates the velocity at the stage times t, t + dt/2, t + dt/2,
    t + dt (§3.1 Step 6 with the time factor cos(pi t / T) of §4.2). On the single vortex,
    whose amplitude changes over the run, the step error of the semi-discrete system must
    fall 16x per halving of dt (fourth order); a stage evaluated at a wrong time breaks the
    condition sum b_i c_i = 1/2 and leaves first order (ratio 2). Same mesh for every dt, so
    the spatial error cancels. gamma = 0 keeps the right-hand side smooth in time (the kink
    of max(gamma, |v|) where |v| crosses gamma costs RK4 its order: ratios 3-5 with the
    paper's gamma), and no reset falls inside the runs."""
    mesh, prm = W.small_case(2, 2, (6, 6), vel_kind=W.VEL_SINGLE_VORTEX, vel_period=0.5,
                             reset_every=10 ** 9, gamma=0.0)
    o = Oracle(2, 2, mesh, prm)
    phi0 = T(W.ic_phi(o.coords(), (0.5, 0.6), 0.25, prm.eps_w * 4))
    psi0, _ = o.precondition(phi0)
    t0, span = 0.05, 0.15                     # g = cos(pi t / 0.5) falls from 0.95 to 0.59

    def run(n):
        phi, psi, t = o.run(phi0, psi0, t0, span / n, n, step0=1)
        assert abs(t - (t0 + span)) < 1e-14
        return phi

    ref = run(256)
    e = [float(torch.max(torch.abs(run(n) - ref))) for n in (16, 32)]
    assert e[1] > 0 and 14.0 < e[0] / e[1] < 19.0, e
