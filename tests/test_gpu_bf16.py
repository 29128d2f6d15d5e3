"""The BF16 precision form (line operators of the gradient and the divergence on the
matrix cores, bf16 operands, fp32 accumulation; fp32 state and pointwise math) against
the FP64 CPU oracle, through the C ABI.

Each line product takes the line's values as deviations from their mean (the mean's part
added in fp32 through the operator's row sums, so constants are exact) and splits both
operands into bf16 pairs x_hi + x_lo (three MFMAs: A_hi d_hi + A_hi d_lo + A_lo d_hi), so
an operand carries a relative error of about 2^-17 instead of the 2^-9 of a single bf16.

Bars, from that arithmetic. The line products DT u and DH f~ see the data as if rounded to
U_R = 2^-17 relative before every product, and on the sharp profiles of the method the
divergence of such data amplifies it by the cancellation factor of the derivative (up to
O(1) of max|R|). The residual bar is therefore stated against the FP64 method's own
sensitivity to U_R-sized data errors: with delta = max|R(u (1 + xi)) - R(u)| over relative
perturbations xi of size U_R (evaluated by the oracle), the BF16 residual is within
RES_FACTOR = 8 delta of the oracle's (8 covers the rounding of the data, of the
intermediate flux and of the operator coefficients). Over 200 steps of the 16x16 p=3
advection workload the interface L1 difference int|phi_bf16 - phi_64| / int phi is a
random walk of about one U_R-sized error per stage update, 3 U_R sqrt(200 * 4) = 6e-4, so
TRAJ_TOL = 1e-3; the split coefficients keep the summation-by-parts identity of DH to
about U_R, so the mass drift stays within MASS_TOL = 1e-5 (200 steps of U_R-sized
per-stage defects, with margin).
"""
import zlib

import numpy as np
import pytest
import torch

import workloads as W
from oracle import Oracle
from oracle import residual as ores

pytestmark = pytest.mark.gpu

U_R = 2.0 ** -17
RES_FACTOR = 8.0
TRAJ_TOL = 1e-3
MASS_TOL = 1e-5


def _solver(mesh, p, prm, precision="bf16"):
    from paper_2006_10967_amd import Solver
    return Solver.from_box(mesh, p, prm, precision=precision)


def _rel(a, b):
    a = a.detach().double().cpu()
    b = b.detach().double().cpu()
    return float((a - b).abs().max()) / float(b.abs().max())


CASES = [
    ("2d_p4_vortex", 2, 4, (11, 13), dict(vel_kind=W.VEL_SINGLE_VORTEX)),
    ("2d_p3_copybc_rotation", 2, 3, (7, 9), dict(periodic=False, vel_kind=W.VEL_ROTATION)),
    ("2d_p6", 2, 6, (4, 5), dict(vel_u0=(-0.4, 0.3))),
    ("3d_p3_leveque", 3, 3, (5, 6, 7), dict(vel_kind=W.VEL_LEVEQUE3D, vel_period=3.0)),
    ("3d_p4_perturbed", 3, 4, (4, 5, 3), dict(perturb=0.2, vel_kind=W.VEL_LEVEQUE3D,
                                              vel_period=3.0)),
    ("3d_p2_copybc", 3, 2, (3, 4, 5), dict(periodic=False, vel_u0=(0.3, 0.2, -0.5))),
    ("3d_p3_skew", 3, 3, (4, 5, 3), dict(shear=(0.25, 0.05, 0.2), vel_kind=W.VEL_LEVEQUE3D,
                                         vel_period=3.0)),
]


@pytest.mark.parametrize("cid,d,p,shape,kw", CASES, ids=[c[0] for c in CASES])
def test_bf16_residuals_within_stated_tolerance(cid, d, p, shape, kw):
    mesh, prm = W.small_case(d, p, shape, **kw)
    o = Oracle(d, p, mesh, prm)
    s = _solver(mesh, p, prm)
    rng = np.random.default_rng(zlib.crc32(cid.encode()))
    x = o.coords()
    c = 0.5 + rng.uniform(-0.1, 0.1, d)
    phi = torch.tensor(W.ic_phi(x, c, 0.27, 0.04))
    psi = torch.tensor(W.signed_distance_ball(x, c, 0.27))
    Rp, Rs = o.residual(phi, psi, 0.37)
    gp, gs = s.residual(phi, psi, 0.37)
    s.set_state(phi, None, 0.0, 0)
    s.precondition(0)
    osgn = ores.smeared_sign(o.disc, prm, phi - 0.5)
    Rpc = o.precond_residual(phi - 0.5, osgn)
    _, gpc = s.residual(None, phi - 0.5, 0.0, mode=1)
    got = [gp, gs, s.sign(), gpc]
    ref = [Rp, Rs, osgn, Rpc]
    # the FP64 method's sensitivity to relative data errors of size U_R
    delta = [torch.zeros(()) for _ in ref]
    for seed in (1, 2, 3):
        g = np.random.default_rng(seed)
        xi1 = torch.tensor(g.uniform(-1, 1, phi.shape)) * U_R
        xi2 = torch.tensor(g.uniform(-1, 1, phi.shape)) * U_R
        ph, ps = phi * (1 + xi1), psi * (1 + xi2)
        qp, qs = o.residual(ph, ps, 0.37)
        qsgn = ores.smeared_sign(o.disc, prm, (phi - 0.5) * (1 + xi1))
        qpc = o.precond_residual((phi - 0.5) * (1 + xi1), qsgn)
        for i, (a_, b_) in enumerate(zip((qp, qs, qsgn, qpc), ref)):
            delta[i] = torch.maximum(delta[i], (a_ - b_).abs().max())
    names = ("R_phi", "R_psi", "sign", "R_pc")
    for n_, g_, r_, d_ in zip(names, got, ref, delta):
        err = float((g_.detach().double().cpu() - r_).abs().max())
        print(f"[bf16] {cid} {n_}: max err {err:.2e} = {err / float(d_):.2f} x the U_R "
              f"data sensitivity ({float(d_):.2e}; {err / float(r_.abs().max()):.2e} of max|R|)")
        assert err <= RES_FACTOR * float(d_), (cid, n_, err, float(d_))
    # and the matrix-core form really differs from the fp32 one (bf16 rounding is visible)
    s32 = _solver(mesh, p, prm, "fp32")
    g32, _ = s32.residual(phi, psi, 0.37)
    assert _rel(gp, g32) > 1e-6


def test_bf16_trajectory_interface_l1_and_mass():
    cfg = W.config("C1")
    mesh = cfg.mesh()
    o = Oracle(cfg.ndims, cfg.order, mesh, cfg.params)
    x = o.coords()
    phi0 = torch.tensor(W.ic_phi(x, cfg.centre, cfg.radius, cfg.params.eps_w))
    dt = cfg.dt(mesh)
    with torch.no_grad():
        phi_o, _, _ = o.run(phi0, None, 0.0, dt, cfg.steps)
    s = _solver(mesh, cfg.order, cfg.params)
    s.set_state(phi0, None, 0.0, 0)
    s.step(dt, cfg.steps)
    phib = s.get_state(want_psi=False)[0].double().cpu()
    l1 = float(o.l1(phib, phi_o)) / float(o.mass(phi_o))
    drift = abs(float(o.mass(phib)) - float(o.mass(phi0))) / float(o.mass(phi0))
    print(f"[bf16] C1 200 steps: int|phi_bf16 - phi64| / int phi = {l1:.2e}, mass drift {drift:.2e}")
    assert l1 <= TRAJ_TOL, l1
    assert drift <= MASS_TOL, drift


def test_bf16_form_has_no_adjoint():
    from paper_2006_10967_amd import PcpfError
    mesh, prm = W.small_case(2, 3, (4, 4), vel_kind=W.VEL_SINGLE_VORTEX)
    s = _solver(mesh, 3, prm)
    x = s.solution_coords()
    s.set_state(torch.tensor(W.ic_phi(x, (0.5, 0.5), 0.3, 0.05)))
    with pytest.raises(PcpfError) as ei:
        s.forward_ckpt(1e-3, 2, 1)
    assert ei.value.status == 3


POLY_CASES = [("2d_p4", 2, 4, (6, 7)), ("3d_p4_perturbed", 3, 4, (3, 4, 3))]


@pytest.mark.parametrize("cid,d,p,shape", POLY_CASES, ids=[c[0] for c in POLY_CASES])
def test_polynomial_exactness_loss(cid, d, p, shape):
    """How far the reduced-precision line operators are from exact on polynomials.

    psi is a global polynomial of degree p in each coordinate (exact in every element and
    continuous across faces), phi = 0 and v uniform, so the exact residual is
    R_psi = -v . grad psi (FP64 reaches it to round-off). A relative data or coefficient
    error u_r in a line product sum_b D_ab psi_b moves it by up to u_r ||D||_inf max|psi|
    with ||D||_inf the row-sum norm of the physical derivative (2/h ||D1||_inf on the
    reference line). The bar is 4 d u_r |v| ||D||_inf max|psi| / max|R| with
    u_r = 2^-24 (FP32) or 2 U_R (the split bf16 data and coefficients, BF16). A derivative
    on these meshes cancels about 9 bits (||D||_inf max|psi| / max|R| ~ 500), all that a
    single bf16 carries; the split operands keep about 17."""
    from oracle.basis import Basis1D
    mesh, prm = W.small_case(d, p, shape, periodic=False, perturb=0.15 if d == 3 else 0.0,
                             vel_u0=(0.6, -0.35, 0.25))
    o = Oracle(d, p, mesh, prm)
    x = o.coords()
    a = np.array([0.31, 0.62, 0.45])[:d]
    psi_np = np.prod([(x[..., k] - a[k]) ** (p - k) for k in range(d)], axis=0) + x[..., 0]
    grad = np.stack([(np.prod([(x[..., m] - a[m]) ** (p - m) if m != k else
                               (p - k) * (x[..., m] - a[m]) ** (p - k - 1)
                               for m in range(d)], axis=0) + (1.0 if k == 0 else 0.0))
                     for k in range(d)], -1)
    v = np.array(prm.vel_u0[:d])
    R = torch.tensor(-(grad @ v))
    b = Basis1D(p)
    D1 = b.dlagrange(b.xi)
    hmin = min(float(np.min(np.diff(pl))) for pl in mesh.planes)
    dnorm = 2.0 / hmin * float(np.max(np.abs(D1).sum(1)))
    scale = d * float(np.abs(v).max()) * dnorm * float(np.abs(psi_np).max()) / float(R.abs().max())
    phi = torch.zeros_like(R)
    psi = torch.tensor(psi_np)
    # FP64 oracle: exact to round-off on this data
    assert _rel(o.residual(phi, psi, 0.0)[1], R) < 1e-11
    for prec, u_r in (("fp32", 2.0 ** -24), ("bf16", 2 * U_R)):
        s = _solver(mesh, p, prm, precision=prec)
        g = s.residual(phi, psi, 0.0)[1]
        loss = _rel(g, R)
        bar = min(4 * u_r * scale, 1.0)
        print(f"[bf16] {cid} {prec}: polynomial-exactness loss max|R - R_exact| / max|R_exact| "
              f"= {loss:.2e} (bar {bar:.2e})")
        assert loss <= bar, (prec, loss, bar)
