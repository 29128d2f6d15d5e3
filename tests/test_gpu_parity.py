"""GPU parity of the FP64 HIP path against the FP64 CPU oracle (called through the C ABI).

Bar (FP64): L_inf relative difference max|R_gpu - R_oracle| / max|R_oracle| <= 1e-12 for
every residual; trajectories <= 1e-10 relative after 200 steps. Inputs come from the
seeded generators in ``workloads`` or from the oracle itself, never from the GPU path.
"""
import math
import zlib

import numpy as np
import pytest
import torch

import workloads as W
from oracle import Oracle
from oracle import residual as ores

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _solver(mesh, p, prm, precision="fp64"):
    from paper_2006_10967_amd import Solver
    return Solver.from_box(mesh, p, prm, precision=precision)


def _rel(a, b):
    a = a.detach().double().cpu() if torch.is_tensor(a) else torch.as_tensor(a)
    b = b.detach().double().cpu() if torch.is_tensor(b) else torch.as_tensor(b)
    den = float(b.abs().max())
    return float((a - b).abs().max()) / (den if den > 0 else 1.0)


def _states(o, rng, kind):
    x = o.coords()
    d = x.shape[-1]
    E, Nu = x.shape[:2]
    if kind == "random":
        return (torch.tensor(rng.uniform(0, 1, (E, Nu))), torch.tensor(rng.standard_normal((E, Nu))))
    c = 0.5 + rng.uniform(-0.1, 0.1, d)
    phi = torch.tensor(W.ic_phi(x, c, 0.27, 0.04))
    psi = torch.tensor(W.signed_distance_ball(x, c, 0.27) + 1e-3 * rng.standard_normal((E, Nu)))
    return phi, psi


CASES = [
    # (id, d, p, shape, small_case kwargs)
    ("2d_p3_uniform", 2, 3, (16, 16), dict(vel_u0=(1.0, 0.5))),
    ("2d_p4_vortex_ragged", 2, 4, (11, 13), dict(vel_kind=W.VEL_SINGLE_VORTEX)),
    ("2d_p2_sheared", 2, 2, (8, 8), dict(shear=0.25, vel_u0=(0.3, -0.7))),
    ("2d_p3_copybc_rotation", 2, 3, (7, 9), dict(periodic=False, vel_kind=W.VEL_ROTATION)),
    ("2d_p1", 2, 1, (9, 7), dict(vel_u0=(0.2, 0.9))),
    ("2d_p5_perturbed", 2, 5, (6, 5), dict(perturb=0.2, vel_kind=W.VEL_SINGLE_VORTEX)),
    ("2d_p6", 2, 6, (4, 5), dict(vel_u0=(-0.4, 0.3))),
    ("2d_single_element", 2, 3, (1, 1), dict(vel_u0=(1.0, 0.25))),
    ("3d_p3_leveque_ragged", 3, 3, (5, 6, 7), dict(vel_kind=W.VEL_LEVEQUE3D, vel_period=3.0)),
    ("3d_p4_perturbed", 3, 4, (4, 5, 3), dict(perturb=0.2, vel_kind=W.VEL_LEVEQUE3D, vel_period=3.0)),
    ("3d_p2_copybc", 3, 2, (3, 4, 5), dict(periodic=False, vel_u0=(0.3, 0.2, -0.5))),
    ("3d_p1", 3, 1, (6, 5, 4), dict(vel_u0=(0.3, 0.2, -0.5))),
    ("3d_p5", 3, 5, (3, 2, 3), dict(vel_kind=W.VEL_LEVEQUE3D, vel_period=3.0)),
    # walls in some directions only: most - faces have a neighbour, some lie on a wall
    ("2d_p4_mixed_bc", 2, 4, (9, 7), dict(periodic=(True, False), vel_u0=(0.7, -0.3))),
    ("3d_p3_mixed_bc", 3, 3, (4, 5, 3), dict(periodic=(False, True, False),
                                             vel_u0=(0.3, -0.4, 0.2))),
    # skewed hexes (full, non-diagonal J; non-axis face normals), periodic with shifted
    # wraps, and with walls
    ("3d_p3_skew", 3, 3, (4, 5, 3), dict(shear=(0.25, 0.05, 0.2), vel_u0=(0.3, 0.2, -0.5))),
    ("3d_p2_skew_leveque", 3, 2, (4, 5, 6), dict(shear=(0.25, 0.05, 0.2),
                                                 vel_kind=W.VEL_LEVEQUE3D, vel_period=3.0)),
    ("3d_p4_skew_copybc", 3, 4, (3, 3, 2), dict(shear=(0.3, -0.2, 0.1), periodic=False,
                                                vel_u0=(-0.2, 0.5, 0.3))),
]


@pytest.mark.parametrize("cid,d,p,shape,kw", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("kind", ["smooth", "random"])
def test_physical_residual_parity(cid, d, p, shape, kw, kind):
    mesh, prm = W.small_case(d, p, shape, **kw)
    o = Oracle(d, p, mesh, prm)
    s = _solver(mesh, p, prm)
    rng = np.random.default_rng(zlib.crc32(f"{cid}:{kind}".encode()))
    phi, psi = _states(o, rng, kind)
    t = 0.37
    Rp, Rs = o.residual(phi, psi, t)
    gp, gs = s.residual(phi, psi, t)
    assert _rel(gp, Rp) <= TOL, (cid, kind, _rel(gp, Rp))
    assert _rel(gs, Rs) <= TOL, (cid, kind, _rel(gs, Rs))


PC_CASES = [c for c in CASES if c[0] in ("2d_p3_uniform", "2d_p4_vortex_ragged",
                                         "2d_p3_copybc_rotation", "3d_p3_leveque_ragged",
                                         "3d_p4_perturbed", "3d_p2_copybc", "2d_single_element",
                                         "3d_p3_mixed_bc", "3d_p3_skew",
                                         "3d_p4_skew_copybc")]


@pytest.mark.parametrize("cid,d,p,shape,kw", PC_CASES, ids=[c[0] for c in PC_CASES])
def test_reset_sign_sensor_and_precond_residual_parity(cid, d, p, shape, kw):
    mesh, prm = W.small_case(d, p, shape, **kw)
    o = Oracle(d, p, mesh, prm)
    s = _solver(mesh, p, prm)
    rng = np.random.default_rng(7)
    phi, psi = _states(o, rng, "smooth")
    # a1: reset + smeared sign
    s.set_state(phi)
    s.precondition(0)
    psi0 = o.reset_psi(phi)
    sgn = ores.smeared_sign(o.disc, prm, psi0)
    assert _rel(s.sign(), sgn) <= TOL
    _, gpsi0, _, _ = s.get_state()
    assert float((gpsi0.cpu() - psi0).abs().max()) == 0.0
    # sensor on fields with a spread of top-mode energies (ramp, clipped and zero regions)
    for amp in (0.0, 1e-4, 1e-2, 1.0):
        field = psi + amp * torch.tensor(rng.standard_normal(psi.shape))
        nu_o = o.sensor(field)
        nu_g = s.sensor(field)
        assert float((nu_g.cpu() - nu_o).abs().max()) <= TOL * prm.nu_max
    # a2: preconditioning residual with the stored sign
    for amp in (1e-3, 1e-1):
        field = psi + amp * torch.tensor(rng.standard_normal(psi.shape))
        R = o.precond_residual(field, sgn)
        _, gR = s.residual(None, field, 0.0, mode=1)
        assert _rel(gR, R) <= TOL, (cid, amp, _rel(gR, R))


@pytest.mark.parametrize("cfg_name", ["C1"])
def test_precondition_parity(cfg_name):
    cfg = W.config(cfg_name)
    mesh = cfg.mesh()
    o = Oracle(cfg.ndims, cfg.order, mesh, cfg.params)
    s = _solver(mesh, cfg.order, cfg.params)
    phi = torch.tensor(W.ic_phi(o.coords(), cfg.centre, cfg.radius, cfg.params.eps_w))
    psi_o, _ = o.precondition(phi)
    s.set_state(phi)
    s.precondition()
    _, psi_g, _, _ = s.get_state()
    assert _rel(psi_g, psi_o) <= 1e-12


def test_trajectory_parity_advection_200_steps():
    """The 16x16, p=3 advection workload: reset + 10 pseudo iterations, then 200 RK4 steps;
    phi and psi match the oracle to 1e-10 and the GPU conserves mass to 1e-12."""
    cfg = W.config("C1")
    mesh = cfg.mesh()
    o = Oracle(2, 3, mesh, cfg.params)
    s = _solver(mesh, 3, cfg.params)
    phi0 = torch.tensor(W.ic_phi(o.coords(), cfg.centre, cfg.radius, cfg.params.eps_w))
    dt = cfg.dt(mesh)
    phi_o, psi_o, _ = o.run(phi0, None, 0.0, dt, cfg.steps)
    s.set_state(phi0)
    s.step(dt, cfg.steps)
    phi_g, psi_g, t, n = s.get_state()
    assert n == cfg.steps and abs(t - cfg.steps * dt) < 1e-12
    assert _rel(phi_g, phi_o) <= 1e-10
    assert _rel(psi_g, psi_o) <= 1e-10
    m0 = s.mass(phi0)
    assert abs(s.mass() - m0) / m0 <= 1e-12
    assert abs(m0 - float(o.mass(phi0))) <= 1e-14 * abs(m0)
    assert abs(s.l1(phi0) - float(o.l1(phi_g.cpu(), phi0))) <= 1e-13


def test_trajectory_parity_mixed_walls():
    """Periodic in x, walls in y (9x7 quads, p=4): reset + 3 pseudo iterations, then 30 RK4
    steps with a reset at step 20; phi and psi match the oracle to 1e-10."""
    mesh, prm = W.small_case(2, 4, (9, 7), periodic=(True, False), vel_u0=(0.7, -0.3),
                             precond_iters=3, reset_every=20)
    o = Oracle(2, 4, mesh, prm)
    s = _solver(mesh, 4, prm)
    x = o.coords()
    phi0 = torch.tensor(W.ic_phi(x, np.array([0.45, 0.5]), 0.25, 0.05))
    dt = 0.005          # dt |v| / h = 0.034, half the RK4 limit at p = 4
    phi_o, psi_o, _ = o.run(phi0, None, 0.0, dt, 30)
    s.set_state(phi0)
    s.step(dt, 30)
    phi_g, psi_g, _, _ = s.get_state()
    assert _rel(phi_g, phi_o) <= 1e-10
    assert _rel(psi_g, psi_o) <= 1e-10


def test_trajectory_parity_skewed_hexes():
    """Skewed periodic hexes (4x5x3, p=3, full J) under the LeVeque field: reset + 3
    pseudo iterations, 20 RK4 steps with a reset at step 12; phi and psi match the oracle
    to 1e-10 and mass is conserved to round-off."""
    mesh, prm = W.small_case(3, 3, (4, 5, 3), shear=(0.25, 0.05, 0.2),
                             vel_kind=W.VEL_LEVEQUE3D, vel_period=3.0, precond_iters=3,
                             reset_every=12)
    o = Oracle(3, 3, mesh, prm)
    s = _solver(mesh, 3, prm)
    x = o.coords()
    phi0 = torch.tensor(W.ic_phi(x, np.array([0.45, 0.5, 0.55]), 0.3, 0.08))
    dt = 0.004
    phi_o, psi_o, _ = o.run(phi0, None, 0.0, dt, 20)
    s.set_state(phi0)
    s.step(dt, 20)
    phi_g, psi_g, _, _ = s.get_state()
    assert _rel(phi_g, phi_o) <= 1e-10
    assert _rel(psi_g, psi_o) <= 1e-10
    m0 = s.mass(phi0)
    assert abs(s.mass() - m0) / m0 <= 1e-12


def test_full_size_vortex_residual():
    """The 128x128, p=4 vortex mesh at full size (the benchmarked launch shape)."""
    cfg = W.config("C2")
    mesh = cfg.mesh()
    o = Oracle(2, 4, mesh, cfg.params)
    s = _solver(mesh, 4, cfg.params)
    x = o.coords()
    phi = torch.tensor(W.ic_phi(x, cfg.centre, cfg.radius, cfg.params.eps_w))
    psi = torch.tensor(W.signed_distance_ball(x, cfg.centre, cfg.radius))
    for t in (0.0, 2.3):
        Rp, Rs = o.residual(phi, psi, t)
        gp, gs = s.residual(phi, psi, t)
        assert _rel(gp, Rp) <= TOL and _rel(gs, Rs) <= TOL


def test_step_is_deterministic():
    cfg = W.config("C1")
    mesh = cfg.mesh()
    s = _solver(mesh, 3, cfg.params)
    x = s.solution_coords()
    phi0 = torch.tensor(W.ic_phi(x, cfg.centre, cfg.radius, cfg.params.eps_w))
    outs = []
    for _ in range(2):
        s.set_state(phi0)
        s.step(cfg.dt(mesh), 20)
        outs.append(s.get_state()[0].cpu())
    assert torch.equal(outs[0], outs[1])


def test_nonfinite_is_reported():
    from paper_2006_10967_amd import PcpfError
    cfg = W.config("C1")
    mesh = cfg.mesh()
    s = _solver(mesh, 3, cfg.params)
    x = s.solution_coords()
    phi0 = torch.tensor(W.ic_phi(x, cfg.centre, cfg.radius, cfg.params.eps_w))
    s.set_state(phi0)
    with pytest.raises(PcpfError) as ei:
        s.step(100 * cfg.dt(mesh), 40)
    assert ei.value.status == 5


NPHI_CASES = [c for c in CASES if c[0] in ("2d_p4_vortex_ragged", "2d_p3_copybc_rotation",
                                           "2d_p2_sheared", "3d_p3_leveque_ragged",
                                           "3d_p4_perturbed", "3d_p3_skew",
                                           "3d_p4_skew_copybc")]


@pytest.mark.parametrize("cid,d,p,shape,kw", NPHI_CASES, ids=[c[0] for c in NPHI_CASES])
def test_unpreconditioned_residual_parity(cid, d, p, shape, kw):
    """The unpreconditioned form (interface normal from phi, §2): the residual against the
    oracle in the same mode, on smooth and random states."""
    import dataclasses
    mesh, prm = W.small_case(d, p, shape, **kw)
    prm = dataclasses.replace(prm, normal_mode=W.NORMAL_PHI)
    o = Oracle(d, p, mesh, prm)
    s = _solver(mesh, p, prm)
    for kind in ("smooth", "random"):
        rng = np.random.default_rng(zlib.crc32(f"nphi:{cid}:{kind}".encode()))
        phi, psi = _states(o, rng, kind)
        Rp, Rs = o.residual(phi, psi, 0.3)
        gp, gs = s.residual(phi, psi, 0.3)
        assert _rel(gp, Rp) <= TOL, (cid, kind, _rel(gp, Rp))
        assert _rel(gs, Rs) <= TOL, (cid, kind, _rel(gs, Rs))


def test_unpreconditioned_trajectory():
    import dataclasses
    cfg = W.config("C1")
    mesh = cfg.mesh()
    prm = dataclasses.replace(cfg.params, normal_mode=W.NORMAL_PHI, reset_every=0)
    o = Oracle(2, 3, mesh, prm)
    s = _solver(mesh, 3, prm)
    x = o.coords()
    phi0 = torch.tensor(W.ic_phi(x, cfg.centre, cfg.radius, cfg.params.eps_w))
    psi0 = phi0 - 0.5
    dt = cfg.dt(mesh)
    with torch.no_grad():
        phi_o, _, _ = o.run(phi0, psi0, 0.0, dt, 100)
    s.set_state(phi0, psi0, 0.0, 0)
    s.step(dt, 100)
    phi_g = s.get_state(want_psi=False)[0]
    assert _rel(phi_g, phi_o) <= 1e-10
