"""GPU parity of the triangle element (dense per-element operators, called through
pcpf_create_dense) against the FP64 CPU oracle's triangle discretisation.

Meshes are split-Cartesian triangle meshes from ``workloads`` (periodic, wall-bounded,
mixed, with perturbed grid lines: general affine triangles); the dense description is the
library's own triangle operators with geometry from the element maps and owners by the LDG
switch vector. Bars as for the tensor elements: FP64 residuals <= 1e-12 relative (L_inf
over max|R_oracle|), trajectories <= 1e-10 relative, mass conserved to 1e-12; FP32
residuals <= 2e-4 relative (the FP32 bar of the tensor elements, same arithmetic per point).
"""
import zlib

import numpy as np
import pytest
import torch

import workloads as W
from oracle import Oracle
from oracle import residual as ores
from tri_dense import tri_dense

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _rel(a, b):
    a = a.detach().double().cpu() if torch.is_tensor(a) else torch.as_tensor(a)
    b = b.detach().double().cpu() if torch.is_tensor(b) else torch.as_tensor(b)
    den = float(b.abs().max())
    return float((a - b).abs().max()) / (den if den > 0 else 1.0)


CASES = [
    # (id, p, n cells per side, split_tri_mesh kwargs, velocity parameters)
    ("tri_p1_uniform", 1, 7, dict(), dict(vel_u0=(0.6, 0.3))),
    ("tri_p2_perturbed_vortex", 2, 6, dict(perturb=0.2), dict(vel_kind=W.VEL_SINGLE_VORTEX)),
    ("tri_p3_copybc_rotation", 3, 5, dict(periodic=False), dict(vel_kind=W.VEL_ROTATION,
                                                                 vel_u0=(0.5, 0.5, 0.0))),
    ("tri_p3_mixed_bc", 3, 4, dict(periodic=(True, False)), dict(vel_u0=(0.7, -0.3))),
    ("tri_p4_perturbed", 4, 4, dict(perturb=0.15, seed=5), dict(vel_u0=(-0.4, 0.8))),
    ("tri_p4_copybc_vortex", 4, 3, dict(periodic=False, perturb=0.1),
     dict(vel_kind=W.VEL_SINGLE_VORTEX)),
    ("tri_p5", 5, 3, dict(), dict(vel_u0=(0.3, -0.9))),
    ("tri_single_cell", 2, 1, dict(), dict(vel_u0=(1.0, 0.25))),
]


def _case(p, n, mkw, vkw, **over):
    mesh = W.split_tri_mesh(n, **mkw)
    prm = W.default_params(2, p, 1.0 / n, **vkw, **over)
    return mesh, prm


def _solver(p, mesh, prm, precision="fp64"):
    from paper_2006_10967_amd import Solver
    dm, _ = tri_dense(p, mesh)
    return Solver.from_dense(dm, prm, precision=precision)


def _states(o, rng, kind):
    x = o.coords()
    E, Nu = x.shape[:2]
    if kind == "random":
        return (torch.tensor(rng.uniform(0, 1, (E, Nu))), torch.tensor(rng.standard_normal((E, Nu))))
    c = 0.5 + rng.uniform(-0.1, 0.1, 2)
    phi = torch.tensor(W.ic_phi(x, c, 0.27, 0.05))
    psi = torch.tensor(W.signed_distance_ball(x, c, 0.27) + 1e-3 * rng.standard_normal((E, Nu)))
    return phi, psi


@pytest.mark.parametrize("cid,p,n,mkw,vkw", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("kind", ["smooth", "random"])
def test_triangle_physical_residual_parity(cid, p, n, mkw, vkw, kind):
    mesh, prm = _case(p, n, mkw, vkw)
    o = Oracle(2, p, mesh, prm)
    s = _solver(p, mesh, prm)
    rng = np.random.default_rng(zlib.crc32(f"{cid}:{kind}".encode()))
    phi, psi = _states(o, rng, kind)
    for t in (0.0, 0.37):
        Rp, Rs = o.residual(phi, psi, t)
        gp, gs = s.residual(phi, psi, t)
        assert _rel(gp, Rp) <= TOL, (cid, kind, t, _rel(gp, Rp))
        assert _rel(gs, Rs) <= TOL, (cid, kind, t, _rel(gs, Rs))


NPHI = [c for c in CASES if c[0] in ("tri_p2_perturbed_vortex", "tri_p4_copybc_vortex")]


@pytest.mark.parametrize("cid,p,n,mkw,vkw", NPHI, ids=[c[0] for c in NPHI])
def test_triangle_unpreconditioned_residual_parity(cid, p, n, mkw, vkw):
    mesh, prm = _case(p, n, mkw, vkw, normal_mode=W.NORMAL_PHI)
    o = Oracle(2, p, mesh, prm)
    s = _solver(p, mesh, prm)
    for kind in ("smooth", "random"):
        rng = np.random.default_rng(zlib.crc32(f"nphi:{cid}:{kind}".encode()))
        phi, psi = _states(o, rng, kind)
        Rp, Rs = o.residual(phi, psi, 0.3)
        gp, gs = s.residual(phi, psi, 0.3)
        assert _rel(gp, Rp) <= TOL, (cid, kind, _rel(gp, Rp))
        assert _rel(gs, Rs) <= TOL, (cid, kind, _rel(gs, Rs))


PC = [c for c in CASES if c[0] in ("tri_p2_perturbed_vortex", "tri_p3_copybc_rotation",
                                   "tri_p3_mixed_bc", "tri_p4_perturbed", "tri_p5",
                                   "tri_single_cell")]


@pytest.mark.parametrize("cid,p,n,mkw,vkw", PC, ids=[c[0] for c in PC])
def test_triangle_reset_sign_sensor_and_precond_residual_parity(cid, p, n, mkw, vkw):
    mesh, prm = _case(p, n, mkw, vkw)
    o = Oracle(2, p, mesh, prm)
    s = _solver(p, mesh, prm)
    rng = np.random.default_rng(zlib.crc32(f"pc:{cid}".encode()))
    phi, psi = _states(o, rng, "smooth")
    s.set_state(phi)
    s.precondition(0)
    psi0 = o.reset_psi(phi)
    sgn = ores.smeared_sign(o.disc, prm, psi0)
    assert _rel(s.sign(), sgn) <= TOL
    _, gpsi0, _, _ = s.get_state()
    assert float((gpsi0.cpu() - psi0).abs().max()) == 0.0
    for amp in (0.0, 1e-4, 1e-2, 1.0):
        field = psi + amp * torch.tensor(rng.standard_normal(psi.shape))
        nu_o = o.sensor(field)
        nu_g = s.sensor(field)
        assert float((nu_g.cpu() - nu_o).abs().max()) <= TOL * prm.nu_max, (cid, amp)
    for amp in (1e-3, 1e-1):
        field = psi + amp * torch.tensor(rng.standard_normal(psi.shape))
        R = o.precond_residual(field, sgn)
        _, gR = s.residual(None, field, 0.0, mode=1)
        assert _rel(gR, R) <= TOL, (cid, amp, _rel(gR, R))


def test_triangle_preconditioning_parity():
    """Reset + 10 pseudo-time RK4 iterations on a perturbed periodic p=3 mesh."""
    mesh, prm = _case(3, 6, dict(perturb=0.2, seed=2), dict(vel_u0=(0.5, 0.5)))
    o = Oracle(2, 3, mesh, prm)
    s = _solver(3, mesh, prm)
    phi = torch.tensor(W.ic_phi(o.coords(), np.array([0.47, 0.52]), 0.3, prm.eps_w))
    psi_o, _ = o.precondition(phi)
    s.set_state(phi)
    s.precondition()
    _, psi_g, _, _ = s.get_state()
    assert _rel(psi_g, psi_o) <= 1e-12


@pytest.mark.parametrize("p,n,mkw,vkw", [
    (3, 6, dict(perturb=0.2, seed=4), dict(vel_kind=W.VEL_SINGLE_VORTEX)),
    (2, 5, dict(periodic=False), dict(vel_kind=W.VEL_ROTATION, vel_u0=(0.5, 0.5, 0.0))),
    (4, 4, dict(periodic=(False, True), perturb=0.1), dict(vel_u0=(0.4, -0.6))),
], ids=["p3_perturbed_vortex", "p2_walls_rotation", "p4_mixed_bc"])
def test_triangle_trajectory_parity(p, n, mkw, vkw):
    """Reset + 3 pseudo iterations, 20 RK4 steps with a reset at step 12: phi and psi match
    the oracle to 1e-10; the GPU's quadrature equals the oracle's, and it conserves mass
    to round-off where no flux crosses the boundary (periodic, or the single vortex, whose
    velocity is tangential on the walls)."""
    mesh, prm = _case(p, n, mkw, vkw, precond_iters=3, reset_every=12)
    o = Oracle(2, p, mesh, prm)
    s = _solver(p, mesh, prm)
    phi0 = torch.tensor(W.ic_phi(o.coords(), np.array([0.45, 0.5]), 0.25, 0.06))
    dt = 0.05 / (n * (2 * p + 1))
    phi_o, psi_o, _ = o.run(phi0, None, 0.0, dt, 20)
    s.set_state(phi0)
    s.step(dt, 20)
    phi_g, psi_g, t, nst = s.get_state()
    assert nst == 20 and abs(t - 20 * dt) < 1e-12
    assert _rel(phi_g, phi_o) <= 1e-10
    assert _rel(psi_g, psi_o) <= 1e-10
    m0 = s.mass(phi0)
    assert abs(m0 - float(o.mass(phi0))) <= 1e-14 * abs(m0)
    if mkw.get("periodic", True) is True or vkw.get("vel_kind") == W.VEL_SINGLE_VORTEX:
        assert abs(s.mass() - m0) / m0 <= 1e-12
    assert abs(s.l1(phi0) - float(o.l1(phi_g.cpu(), phi0))) <= 1e-13


FP32 = [c for c in CASES if c[0] in ("tri_p2_perturbed_vortex", "tri_p3_copybc_rotation",
                                     "tri_p4_perturbed")]


@pytest.mark.parametrize("cid,p,n,mkw,vkw", FP32, ids=[c[0] for c in FP32])
def test_triangle_fp32_residual(cid, p, n, mkw, vkw):
    mesh, prm = _case(p, n, mkw, vkw)
    o = Oracle(2, p, mesh, prm)
    s = _solver(p, mesh, prm, "fp32")
    rng = np.random.default_rng(zlib.crc32(f"fp32:{cid}".encode()))
    phi, psi = _states(o, rng, "smooth")
    Rp, Rs = o.residual(phi, psi, 0.2)
    gp, gs = s.residual(phi.float(), psi.float(), 0.2)
    assert _rel(gp, Rp) <= 2e-4, (cid, _rel(gp, Rp))
    assert _rel(gs, Rs) <= 2e-4, (cid, _rel(gs, Rs))


def test_triangle_adjoint_and_bf16_refused():
    from paper_2006_10967_amd import PcpfError, _lib
    mesh, prm = _case(2, 3, dict(), dict(vel_u0=(0.5, 0.5)))
    s = _solver(2, mesh, prm)
    o = Oracle(2, 2, mesh, prm)
    s.set_state(torch.tensor(W.ic_phi(o.coords(), np.array([0.5, 0.5]), 0.3, 0.1)))
    with pytest.raises(PcpfError) as ei:
        s.forward_ckpt(1e-3, 4)
    assert ei.value.status == _lib.PCPF_EUNSUPPORTED
    with pytest.raises(PcpfError) as ei:
        _solver(2, mesh, prm, "bf16")
    assert ei.value.status == _lib.PCPF_EUNSUPPORTED


def _tri_sub_block(mesh, lo, m):
    """The m x m cells from cell (lo) as a copy-boundary split mesh on the full mesh's own
    grid lines, the full-mesh index of each of its triangles, and which of them lie off its
    outer cell layer. A triangle's residual depends on its own state, its edge neighbours'
    traces and the common fluxes their owners compute from their own gradients, which need
    the owners' neighbours: every triangle within two edge hops, all inside the 3 x 3 cells
    around its own; so the inner triangles of the sub-block reproduce the full mesh."""
    n = mesh.shape[0]
    planes = [np.asarray(mesh.planes[k])[lo[k]:lo[k] + m + 1] for k in range(2)]
    sub = W.split_tri_mesh(m, periodic=False, planes=planes)
    e = np.arange(sub.nelem)
    cell = e // 2
    ci, cj = cell % m, cell // m
    full = 2 * ((ci + lo[0]) + n * (cj + lo[1])) + e % 2
    inner = (ci >= 1) & (ci <= m - 2) & (cj >= 1) & (cj <= m - 2)
    return sub, full, inner


def test_full_size_sampled_residuals_triangles():
    """The 1024^2-cell triangle mesh (2.1 M triangles, p = 4) in the launch configuration
    the benchmark times: residuals of two 8 x 8-cell sub-blocks (across the circle's
    interface, and at the high-index corner, where a second small circle gives an interface)
    against the oracle <= 1e-12, and mass conservation of the whole residual."""
    from paper_2006_10967_amd import Solver
    cfg = W.config("T2")
    mesh = cfg.mesh()
    p, prm = cfg.order, cfg.params
    s = Solver.from_triangles(mesh, p, prm)
    x = s.solution_coords()
    n = mesh.shape[0]
    h = 1.0 / n
    c2, r2 = np.array([1.0 - 4 * h, 1.0 - 4 * h]), 2.5 * h
    dist = np.maximum(W.signed_distance_ball(x, cfg.centre, cfg.radius),
                      W.signed_distance_ball(x, c2, r2))
    phi = torch.tensor(W.tanh_profile(dist, prm.eps_w))
    psi = torch.tensor(dist)
    del x
    gp, gs = s.residual(phi, psi, 0.3)
    gp, gs = gp.cpu(), gs.cpu()
    # the circle (0.5, 0.75), r = 0.15, crosses x = 0.35 at y = 0.75
    for lo in ((int(0.35 * n) - 4, int(0.75 * n) - 4), (n - 8, n - 8)):
        sub, full, inner = _tri_sub_block(mesh, lo, 8)
        o = Oracle(2, p, sub, prm)
        Rp, Rs = o.residual(phi[full], psi[full], 0.3)
        sel = torch.as_tensor(inner)
        assert float(phi[full][sel].min()) < 0.1 and float(phi[full][sel].max()) > 0.9, lo
        assert _rel(gp[full][sel], Rp[sel]) <= TOL, (lo, _rel(gp[full][sel], Rp[sel]))
        assert _rel(gs[full][sel], Rs[sel]) <= TOL, (lo, _rel(gs[full][sel], Rs[sel]))
    assert int(full.max()) == mesh.nelem - 1
    # sum |J| W R_phi = 0 on the periodic mesh (each common flux is shared by its two sides)
    dm = s.dense
    w = torch.as_tensor(dm.keep["detj"])[:, None] * torch.as_tensor(dm.keep["W"])[None, :]
    tot = float((w * gp).sum())
    scale = float((w * gp.abs()).sum())
    assert abs(tot) <= 1e-13 * scale, (tot, scale)


TRI_RMS_CASES = [
    # (id, p, n, eps_w of the IC, sign mode): the RMS stop rule ends after 5, 10, 13 and 18
    # iterations, every iteration's RMS at least 3.8e-3 from 1/2 (oracle), so rounding
    # cannot move the decision
    ("p2_psi0", 2, 6, 0.05, W.SGN_PSI0),
    ("p2_current", 2, 6, 0.04, W.SGN_CURRENT),
    ("p3_psi0", 3, 6, 0.04, W.SGN_PSI0),
    ("p2_current_18", 2, 8, 0.03, W.SGN_CURRENT),
]


@pytest.mark.parametrize("cid,p,n,ew,sgn", TRI_RMS_CASES, ids=[c[0] for c in TRI_RMS_CASES])
def test_triangle_rms_stop_rule_parity(cid, p, n, ew, sgn):
    """The printed stop rule (and, in two cases, the printed sign) on triangles: the same
    iteration count as the oracle, its last RMS to 1e-10, psi to 1e-12."""
    mesh, prm = _case(p, n, dict(), dict(vel_u0=(0.6, 0.3)), stop_mode=W.STOP_RMS,
                      precond_iters=20, sgn_mode=sgn)
    o = Oracle(2, p, mesh, prm)
    s = _solver(p, mesh, prm)
    phi = torch.tensor(W.ic_phi(o.coords(), (0.5, 0.5), 0.3, ew))
    psi_o, _ = o.precondition(phi)
    s.set_state(phi)
    s.precondition()
    k, rms = s.precond_info()
    _, psi_g, _, _ = s.get_state()
    assert 1 < o.last_iters < 20
    assert k == o.last_iters, (k, o.last_iters)
    assert abs(rms - o.last_rms) <= 1e-10 * o.last_rms
    assert _rel(psi_g, psi_o) <= TOL


@pytest.mark.parametrize("reset", [W.RESET_LINEAR, W.RESET_LOGIT], ids=["linear", "logit"])
def test_triangle_printed_forms_and_logit_trajectory(reset):
    """Printed sign and RMS stop rule, with the linear or the logit reset, over 40 steps
    with resets every 16 on a perturbed p = 3 mesh under the single vortex: phi and psi
    match the oracle to 1e-10 (the stop decisions at the three resets are at least 3.5e-3
    from the threshold in the oracle run)."""
    mesh, prm = _case(3, 5, dict(perturb=0.1, seed=3), dict(vel_kind=W.VEL_SINGLE_VORTEX),
                      stop_mode=W.STOP_RMS, precond_iters=20, sgn_mode=W.SGN_CURRENT,
                      reset_mode=reset, reset_every=16)
    o = Oracle(2, 3, mesh, prm)
    s = _solver(3, mesh, prm)
    phi0 = torch.tensor(W.ic_phi(o.coords(), np.array([0.45, 0.5]), 0.25, 0.06))
    dt = 0.05 / (5 * 7)
    phi_o, psi_o, _ = o.run(phi0, None, 0.0, dt, 40)
    s.set_state(phi0)
    s.step(dt, 40)
    phi_g, psi_g, _, _ = s.get_state()
    assert s.precond_info()[0] == o.last_iters
    assert _rel(phi_g, phi_o) <= 1e-10
    assert _rel(psi_g, psi_o) <= 1e-10
