"""The FP32 precision form against the FP64 CPU oracle (called through the C ABI).

FP32 state, FP32 pointwise math and FP32 line operators; FP64 only in the mass/L1
reductions and the logit reset. Bars, stated from the arithmetic:

* residual: R = -div f / |J| is a difference of line products whose terms are each of size
  ~ p^2 |f| / h, so the absolute FP32 error is ~ (ops per point ~ 30) * u * p^2 |f| / h with
  u = 6e-8, and relative to max|R| it is that times the cancellation factor
  p^2 max|f| / (h max|R|), 10-100 on these states (largest for psi v with div v = 0, where
  R is only v . grad psi). Hence a few 1e-5; the bar is RES_TOL = 2e-4 (measured 4e-6 to
  8e-5).
* trajectory (200 RK4 steps of the 16x16 p=3 advection workload with its reset): the
  interface L1 difference int|phi_32 - phi_64| relative to int phi is a random walk of one
  FP32 rounding per stage update, ~ 3 u sqrt(200 * 4) = 5e-6 = TRAJ_TOL; the FP32 mass
  drift stays within MASS_TOL = 2e-6 (the scheme conserves mass exactly up to rounding).
"""
import zlib

import numpy as np
import pytest
import torch

import workloads as W
from oracle import Oracle
from oracle import residual as ores

pytestmark = pytest.mark.gpu

RES_TOL = 2e-4
TRAJ_TOL = 5e-6
MASS_TOL = 2e-6


def _solver(mesh, p, prm, precision):
    from paper_2006_10967_amd import Solver
    return Solver.from_box(mesh, p, prm, precision=precision)


def _rel(a, b):
    a = a.detach().double().cpu()
    b = b.detach().double().cpu()
    return float((a - b).abs().max()) / float(b.abs().max())


CASES = [
    ("2d_p4_vortex", 2, 4, (11, 13), dict(vel_kind=W.VEL_SINGLE_VORTEX)),
    ("2d_p3_sheared", 2, 3, (8, 8), dict(shear=0.25, vel_u0=(0.3, -0.7))),
    ("2d_p3_copybc_rotation", 2, 3, (7, 9), dict(periodic=False, vel_kind=W.VEL_ROTATION)),
    ("3d_p3_leveque", 3, 3, (5, 6, 7), dict(vel_kind=W.VEL_LEVEQUE3D, vel_period=3.0)),
    ("3d_p4_perturbed", 3, 4, (4, 5, 3), dict(perturb=0.2, vel_kind=W.VEL_LEVEQUE3D,
                                              vel_period=3.0)),
    ("3d_p3_skew", 3, 3, (4, 5, 3), dict(shear=(0.25, 0.05, 0.2), vel_kind=W.VEL_LEVEQUE3D,
                                         vel_period=3.0)),
    # odd element counts: the last block of the 3D FP32 line kernel holds one element, and
    # at p = 5 its 216 points take two passes of the 192-thread block
    ("3d_p4_ragged", 3, 4, (3, 3, 3), dict(vel_kind=W.VEL_LEVEQUE3D, vel_period=3.0)),
    ("3d_p5_copybc", 3, 5, (3, 2, 3), dict(periodic=False)),
]


def _smooth_state(o, cid):
    rng = np.random.default_rng(zlib.crc32(cid.encode()))
    x = o.coords()
    d = x.shape[-1]
    c = 0.5 + rng.uniform(-0.1, 0.1, d)
    phi = torch.tensor(W.ic_phi(x, c, 0.27, 0.04))
    psi = torch.tensor(W.signed_distance_ball(x, c, 0.27))
    return phi, psi


@pytest.mark.parametrize("cid,d,p,shape,kw", CASES, ids=[c[0] for c in CASES])
def test_fp32_residual_within_stated_tolerance(cid, d, p, shape, kw):
    mesh, prm = W.small_case(d, p, shape, **kw)
    o = Oracle(d, p, mesh, prm)
    s = _solver(mesh, p, prm, "fp32")
    phi, psi = _smooth_state(o, cid)
    Rp, Rs = o.residual(phi, psi, 0.37)
    gp, gs = s.residual(phi, psi, 0.37)
    ep, es = _rel(gp, Rp), _rel(gs, Rs)
    print(f"[fp32] {cid}: residual rel L_inf phi {ep:.2e} psi {es:.2e}")
    assert ep <= RES_TOL and es <= RES_TOL, (cid, ep, es)


NPHI_CASES = [c for c in CASES if c[0] in ("2d_p4_vortex", "2d_p3_sheared", "3d_p3_skew")]


@pytest.mark.parametrize("cid,d,p,shape,kw", NPHI_CASES, ids=[c[0] for c in NPHI_CASES])
def test_fp32_unpreconditioned_residual(cid, d, p, shape, kw):
    """The unpreconditioned form (normal from phi) in FP32, against the oracle in the same
    mode: the FP32 residual bar (2D: the line kernel of the FP32 form; 3D skewed hexes:
    the general-J line kernel)."""
    import dataclasses
    mesh, prm = W.small_case(d, p, shape, **kw)
    prm = dataclasses.replace(prm, normal_mode=W.NORMAL_PHI)
    o = Oracle(d, p, mesh, prm)
    s = _solver(mesh, p, prm, "fp32")
    phi, psi = _smooth_state(o, "nphi:" + cid)
    Rp, Rs = o.residual(phi, psi, 0.37)
    gp, gs = s.residual(phi, psi, 0.37)
    ep, es = _rel(gp, Rp), _rel(gs, Rs)
    assert ep <= RES_TOL and es <= RES_TOL, (cid, ep, es)


@pytest.mark.parametrize("cid,d,p,shape,kw", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_fp32_precond_residual_within_stated_tolerance(cid, d, p, shape, kw):
    mesh, prm = W.small_case(d, p, shape, **kw)
    o = Oracle(d, p, mesh, prm)
    s = _solver(mesh, p, prm, "fp32")
    phi, psi = _smooth_state(o, cid)
    s.set_state(phi, None, 0.0, 0)
    s.precondition(0)            # reset only: the smeared sign of psi0 = phi - 1/2
    psi0 = phi - 0.5
    osgn = ores.smeared_sign(o.disc, prm, psi0)
    e_sgn = _rel(s.sign(), osgn)
    R = o.precond_residual(psi, osgn)
    _, g = s.residual(None, psi, 0.0, mode=1)
    e = _rel(g, R)
    print(f"[fp32] {cid}: sign rel {e_sgn:.2e}, precond residual rel {e:.2e}")
    assert e_sgn <= RES_TOL and e <= RES_TOL, (cid, e_sgn, e)


def test_fp32_trajectory_interface_l1_and_mass():
    cfg = W.config("C1")
    mesh = cfg.mesh()
    o = Oracle(cfg.ndims, cfg.order, mesh, cfg.params)
    x = o.coords()
    phi0 = torch.tensor(W.ic_phi(x, cfg.centre, cfg.radius, cfg.params.eps_w))
    dt = cfg.dt(mesh)
    with torch.no_grad():
        phi_o, _, _ = o.run(phi0, None, 0.0, dt, cfg.steps)
    s = _solver(mesh, cfg.order, cfg.params, "fp32")
    s.set_state(phi0, None, 0.0, 0)
    s.step(dt, cfg.steps)
    phi32 = s.get_state(want_psi=False)[0].double().cpu()
    l1 = float(o.l1(phi32, phi_o)) / float(o.mass(phi_o))
    drift = abs(float(o.mass(phi32)) - float(o.mass(phi0))) / float(o.mass(phi0))
    print(f"[fp32] C1 200 steps: int|phi32 - phi64| / int phi = {l1:.2e}, mass drift {drift:.2e}")
    assert l1 <= TRAJ_TOL, l1
    assert drift <= MASS_TOL, drift
