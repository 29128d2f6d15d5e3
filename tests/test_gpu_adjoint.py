"""GPU parity of the hand-written adjoint (pcpf_forward_ckpt + pcpf_adjoint) against the
FP64 CPU oracle's reverse-mode autograd through the same discrete map (reset, smeared
sign, pseudo-time preconditioning with the sensor, physical RK4 steps), and against
central differences of the GPU forward run.

Bar (FP64): the vector-Jacobian products dL/dphi0, dL/dpsi0 (L_inf relative) and dL/dA
(relative) within 1e-10 of the oracle's; central differences (h = 1e-5) within 1e-6
relative of the adjoint's directional derivative. Seeds and inputs come from the seeded
generators in ``workloads`` or from the oracle, never from the GPU path.
"""
import zlib

import numpy as np
import pytest
import torch

import workloads as W
from oracle import Oracle

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _solver(mesh, p, prm, precision="fp64"):
    from paper_2006_10967_amd import Solver
    return Solver.from_box(mesh, p, prm, precision=precision)


def _rel(a, b):
    a = a.detach().double().cpu()
    b = b.detach().double().cpu()
    den = float(b.abs().max())
    return float((a - b).abs().max()) / (den if den > 0 else 1.0)


# (id, d, p, shape, small_case kwargs, nsteps, every, step0, psi given, psi seed)
CASES = [
    ("2d_p3_vortex_reset0", 2, 3, (5, 4), dict(vel_kind=W.VEL_SINGLE_VORTEX, vel_period=4.0,
                                                precond_iters=3), 4, 2, 0, False, False),
    ("2d_p4_midrun_resets", 2, 4, (6, 5), dict(vel_u0=(0.8, -0.4), precond_iters=2,
                                                reset_every=2), 5, 2, 1, True, True),
    ("2d_p2_sheared_psi", 2, 2, (8, 8), dict(shear=0.25, vel_u0=(0.3, -0.7), precond_iters=2,
                                             reset_every=3), 4, 3, 1, True, True),
    ("2d_p3_copybc_logit", 2, 3, (5, 6), dict(periodic=False, vel_u0=(0.6, 0.3),
                                              reset_mode=W.RESET_LOGIT, precond_iters=2),
     3, 3, 0, False, True),
    ("3d_p2_leveque", 3, 2, (3, 4, 3), dict(vel_kind=W.VEL_LEVEQUE3D, vel_period=3.0,
                                            precond_iters=2), 3, 3, 0, False, True),
    ("3d_p3_perturbed", 3, 3, (3, 2, 3), dict(perturb=0.2, vel_u0=(0.3, 0.2, -0.5),
                                              precond_iters=1, reset_every=2), 3, 1, 1, True,
     False),
    ("3d_p2_skew", 3, 2, (4, 5, 3), dict(shear=(0.25, 0.05, 0.2), vel_kind=W.VEL_LEVEQUE3D,
                                         vel_period=3.0, precond_iters=2, reset_every=2),
     3, 2, 0, False, True),
]


def _inputs(o, prm, d, seed, psi_given):
    rng = np.random.default_rng(seed)
    x = o.coords()
    c = np.full(d, 0.5) + rng.uniform(-0.08, 0.08, d)
    phi0 = torch.tensor(W.ic_phi(x, c, 0.28, 0.08))
    psi0 = None
    if psi_given:
        psi0 = torch.tensor(W.signed_distance_ball(x, c, 0.28)
                            + 1e-3 * rng.standard_normal(phi0.shape))
    gphi = torch.tensor(rng.standard_normal(phi0.shape))
    gpsi = torch.tensor(rng.standard_normal(phi0.shape))
    return phi0, psi0, gphi, gpsi


def _dt(mesh):
    return 0.05 * float(min(np.min(np.diff(p)) for p in mesh.planes))


def _oracle_vjp(o, phi0, psi0, amp, t0, dt, nsteps, step0, gphi, gpsi):
    p0 = phi0.clone().requires_grad_(True)
    s0 = psi0.clone().requires_grad_(True) if psi0 is not None else None
    A = torch.tensor(amp, dtype=torch.float64, requires_grad=True)
    phiT, psiT, _ = o.run(p0, s0, t0, dt, nsteps, step0=step0, amp=A)
    L = torch.sum(phiT * gphi) + (torch.sum(psiT * gpsi) if gpsi is not None else 0.0)
    wrt = [p0, A] + ([s0] if s0 is not None else [])
    g = torch.autograd.grad(L, wrt, allow_unused=True)
    gs0 = None
    if s0 is not None:
        gs0 = g[2] if g[2] is not None else torch.zeros_like(phi0)
    return g[0], gs0, float(g[1]), phiT.detach()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_adjoint_matches_oracle_autograd(case):
    cid, d, p, shape, kw, nsteps, every, step0, psi_given, psi_seed = case
    mesh, prm = W.small_case(d, p, shape, **kw)
    o = Oracle(d, p, mesh, prm)
    s = _solver(mesh, p, prm)
    phi0, psi0, gphi, gpsi = _inputs(o, prm, d, zlib.crc32(cid.encode()), psi_given)
    if not psi_seed:
        gpsi = None
    dt, t0, amp = _dt(mesh), 0.21, 0.9
    ogp, ogs, oga, ophiT = _oracle_vjp(o, phi0, psi0, amp, t0, dt, nsteps, step0, gphi, gpsi)

    s.set_velocity_amplitude(amp)
    s.set_state(phi0, psi0, t0, step0)
    s.forward_ckpt(dt, nsteps, every)
    phiT = s.get_state(want_psi=False)[0]
    assert _rel(phiT, ophiT) <= TOL, (cid, "forward", _rel(phiT, ophiT))
    gp, gs, ga = s.adjoint(gphi, gpsi)
    assert _rel(gp, ogp) <= TOL, (cid, "dphi0", _rel(gp, ogp))
    assert abs(ga - oga) <= TOL * max(abs(oga), 1e-300), (cid, "dA", ga, oga)
    if psi_given:
        assert _rel(gs, ogs) <= TOL, (cid, "dpsi0", _rel(gs, ogs))
    elif step0 % (prm.reset_every or 1) == 0:
        # the first step resets psi: psi(0) does not influence the result
        assert float(gs.abs().max()) == 0.0


def test_adjoint_checkpoint_interval_is_bitwise_invariant():
    """The reverse sweep recomputes each segment from its checkpoint in the same order
    as the forward run, so the interval changes nothing."""
    mesh, prm = W.small_case(2, 3, (6, 5), vel_kind=W.VEL_SINGLE_VORTEX, vel_period=4.0,
                             precond_iters=2, reset_every=3)
    o = Oracle(2, 3, mesh, prm)
    s = _solver(mesh, 3, prm)
    phi0, psi0, gphi, gpsi = _inputs(o, prm, 2, 11, True)
    dt = _dt(mesh)
    out = []
    for every in (1, 2, 3):
        s.set_state(phi0, psi0, 0.0, 1)
        s.forward_ckpt(dt, 6, every)
        out.append(s.adjoint(gphi, gpsi))
    for gp, gs, ga in out[1:]:
        assert torch.equal(gp, out[0][0]) and torch.equal(gs, out[0][1]) and ga == out[0][2]


def test_adjoint_matches_gpu_central_differences():
    """Directional derivative of L = 1/2 int (phi(T) - target)^2 in phi0 and in A: the
    adjoint against central differences of the GPU forward run."""
    mesh, prm = W.small_case(2, 3, (8, 8), vel_kind=W.VEL_SINGLE_VORTEX, vel_period=4.0,
                             precond_iters=3)
    o = Oracle(2, 3, mesh, prm)
    s = _solver(mesh, 3, prm)
    x = o.coords()
    phi0 = torch.tensor(W.ic_phi(x, (0.5, 0.6), 0.3, 0.06))
    target = torch.tensor(W.ic_phi(x, (0.53, 0.63), 0.3, 0.06)).cuda()
    wq = (o.disc.tdetJ[:, None] * o.disc.tW[None, :]).cuda()
    dt, nsteps = 0.01, 4

    def loss(phi_init, amp):
        s.set_velocity_amplitude(amp)
        s.set_state(phi_init, None, 0.0, 0)
        s.step(dt, nsteps)
        phi = s.get_state(want_psi=False)[0]
        return 0.5 * float(torch.sum(wq * (phi - target) ** 2))

    s.set_velocity_amplitude(1.0)
    s.set_state(phi0, None, 0.0, 0)
    s.forward_ckpt(dt, nsteps, 2)
    phiT = s.get_state(want_psi=False)[0]
    gp, _, ga = s.adjoint(wq * (phiT - target))
    v = torch.tensor(np.random.default_rng(5).standard_normal(phi0.shape))
    v /= torch.linalg.vector_norm(v)   # unit direction: O(h^2) truncation stays ~1e-10
    h = 1e-5
    fd = (loss(phi0 + h * v, 1.0) - loss(phi0 - h * v, 1.0)) / (2 * h)
    ad = float(torch.sum(gp.cpu() * v))
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    fdA = (loss(phi0, 1.0 + h) - loss(phi0, 1.0 - h)) / (2 * h)
    assert abs(fdA - ga) <= 1e-6 * abs(ga), (fdA, ga)


def test_autograd_function_runs_the_library_adjoint():
    from paper_2006_10967_amd.autograd import run
    mesh, prm = W.small_case(2, 2, (5, 5), vel_kind=W.VEL_SINGLE_VORTEX, vel_period=4.0,
                             precond_iters=2)
    o = Oracle(2, 2, mesh, prm)
    s = _solver(mesh, 2, prm)
    phi0, _, gphi, _ = _inputs(o, prm, 2, 3, False)
    dt = _dt(mesh)
    p0 = phi0.cuda().requires_grad_(True)
    A = torch.tensor(1.1, dtype=torch.float64, requires_grad=True)
    phiT, psiT = run(s, p0, A, dt, 3)
    torch.sum(phiT * gphi.cuda()).backward()
    ogp, _, oga, _ = _oracle_vjp(o, phi0, None, 1.1, 0.0, dt, 3, 0, gphi, None)
    assert _rel(p0.grad, ogp) <= TOL
    assert abs(float(A.grad) - oga) <= TOL * abs(oga)


def test_adjoint_fp32_form_tracks_fp64():
    mesh, prm = W.small_case(2, 3, (6, 6), vel_kind=W.VEL_SINGLE_VORTEX, vel_period=4.0,
                             precond_iters=2)
    o = Oracle(2, 3, mesh, prm)
    phi0, _, gphi, _ = _inputs(o, prm, 2, 8, False)
    dt = _dt(mesh)
    res = []
    for prec in ("fp64", "fp32"):
        s = _solver(mesh, 3, prm, prec)
        s.set_state(phi0, None, 0.0, 0)
        s.forward_ckpt(dt, 3, 3)
        res.append(s.adjoint(gphi))
    assert _rel(res[1][0], res[0][0]) <= 2e-4, _rel(res[1][0], res[0][0])
    assert abs(res[1][2] - res[0][2]) <= 2e-4 * abs(res[0][2])


def test_adjoint_at_full_size_matches_oracle():
    """The 64x64 p=3 single-vortex workload: two steps from a reset with the full ten
    preconditioning iterations, oracle VJP on the CPU.

    Away from the interface phi is 0 or 1 to the last bit, psi is constant, grad psi is
    rounding noise and the derivative grad psi / |grad psi| of the eikonal term takes its
    direction from that noise: there the discrete VJP is ill-conditioned (a 1e-16 relative
    perturbation of phi0 moves the oracle's own dL/dphi0 by ~2e-7 of its maximum, 1e-14 by
    ~5e-6). On the interface band phi0 (1 - phi0) > 1e-4, along interface-supported
    directions and for dL/dA it is well conditioned (1e-14 moves it by < 1e-11), so the
    1e-10 bar applies there; elsewhere the bound is the conditioning one, 1e-4."""
    cfg = W.config("C4")
    mesh = cfg.mesh()
    o = Oracle(cfg.ndims, cfg.order, mesh, cfg.params)
    s = _solver(mesh, cfg.order, cfg.params)
    x = o.coords()
    phi0 = torch.tensor(W.ic_phi(x, cfg.centre, cfg.radius, cfg.params.eps_w))
    tgt = torch.tensor(W.ic_phi(x, W.adjoint_target_centre(cfg), cfg.radius, cfg.params.eps_w))
    dt = cfg.dt(mesh)
    nsteps = 2
    wq = o.disc.tdetJ[:, None] * o.disc.tW[None, :]
    with torch.no_grad():
        phiT_o, _, _ = o.run(phi0, None, 0.0, dt, nsteps)
    seed = wq * (phiT_o - tgt)
    ogp, _, oga, _ = _oracle_vjp(o, phi0, None, cfg.params.vel_amp, 0.0, dt, nsteps, 0, seed,
                                 None)
    s.set_state(phi0, None, 0.0, 0)
    s.forward_ckpt(dt, nsteps, 32 if nsteps >= 32 else nsteps)
    gp, _, ga = s.adjoint(seed)
    gp = gp.cpu()
    scale = float(ogp.abs().max())
    band = (phi0 * (1 - phi0)) > 1e-4
    assert float(((gp - ogp) * band).abs().max()) <= TOL * scale
    v = phi0 * (1 - phi0)
    assert abs(float(torch.sum((gp - ogp) * v))) <= TOL * abs(float(torch.sum(ogp * v)))
    assert _rel(gp, ogp) <= 1e-4, _rel(gp, ogp)
    assert abs(ga - oga) <= TOL * abs(oga), (ga, oga)


def test_autograd_interleaved_runs_on_one_solver():
    """Two differentiable runs on one Solver, the second recorded before the first one's
    backward: each backward gives its own run's gradient (the binding records the stale
    run again from its saved inputs), checked against the oracle's VJP of each run."""
    from paper_2006_10967_amd.autograd import run
    mesh, prm = W.small_case(2, 2, (5, 5), vel_kind=W.VEL_SINGLE_VORTEX, vel_period=4.0,
                             precond_iters=2)
    o = Oracle(2, 2, mesh, prm)
    s = _solver(mesh, 2, prm)
    phi_a, _, g_a, _ = _inputs(o, prm, 2, 3, False)
    phi_b, _, g_b, _ = _inputs(o, prm, 2, 4, False)
    dt = _dt(mesh)
    pa = phi_a.cuda().requires_grad_(True)
    pb = phi_b.cuda().requires_grad_(True)
    Aa = torch.tensor(1.1, dtype=torch.float64, requires_grad=True)
    Ab = torch.tensor(0.8, dtype=torch.float64, requires_grad=True)
    phiT_a, _ = run(s, pa, Aa, dt, 3)
    phiT_b, _ = run(s, pb, Ab, dt, 4)           # records over run a
    torch.sum(phiT_a * g_a.cuda()).backward()   # run a's backward after run b's forward
    torch.sum(phiT_b * g_b.cuda()).backward()
    for p, A, phi0, g, amp, n in ((pa, Aa, phi_a, g_a, 1.1, 3), (pb, Ab, phi_b, g_b, 0.8, 4)):
        ogp, _, oga, _ = _oracle_vjp(o, phi0, None, amp, 0.0, dt, n, 0, g, None)
        assert _rel(p.grad, ogp) <= TOL, _rel(p.grad, ogp)
        assert abs(float(A.grad) - oga) <= TOL * abs(oga), (float(A.grad), oga)


def _c4_loss_setup(precision="fp64"):
    cfg = W.config("C4")
    mesh = cfg.mesh()
    s = _solver(mesh, cfg.order, cfg.params, precision)
    x = s.solution_coords()
    phi0 = torch.tensor(W.ic_phi(x, cfg.centre, cfg.radius, cfg.params.eps_w))
    tgt = torch.tensor(W.ic_phi(x, W.adjoint_target_centre(cfg), cfg.radius,
                                cfg.params.eps_w)).cuda()
    det = torch.as_tensor(mesh.jac).det()
    w1 = torch.as_tensor(s.mesh.ops["weights"])
    wq = (det[:, None] * torch.kron(w1, w1)[None, :]).cuda()
    return cfg, mesh, s, phi0, tgt, wq


def test_adjoint_full_horizon_central_differences():
    """The adjoint workload at its own horizon: 64x64 p=3 single vortex, 512 RK4 steps
    from a reset with ten preconditioning iterations, checkpoints every 32 steps, loss
    L = 1/2 int (phi(T) - target)^2. The adjoint's dL/dA and its derivative along an
    interface direction of phi0 agree with central differences of the GPU forward run to
    1e-6 relative.

    Step sizes: at this horizon L(A) carries structure on the scale 1e-5..1e-4 of A (a
    sweep of h from 1e-3 down to 1e-8 converges to the adjoint like h^2: 2e-3 at h = 1e-5,
    3.5e-6 at 1e-7, 3e-7 at 3e-8, 5e-8 at 1e-8), so dL/dA takes h = 1e-8, where the
    truncation (~4e-8) and the rounding of L (~7e-8) are both far below the bar. The phi0
    direction v = 4 phi0 (1 - phi0)(target - phi0) (at most 1 in magnitude, supported on the
    interface, where the map is well conditioned) takes h = 1e-6."""
    cfg, mesh, s, phi0, tgt, wq = _c4_loss_setup()
    dt, nsteps, every = cfg.dt(mesh), cfg.steps, 32

    def loss(phi_init, amp):
        s.set_velocity_amplitude(amp)
        s.set_state(phi_init, None, 0.0, 0)
        s.step(dt, nsteps)
        phi = s.get_state(want_psi=False)[0]
        return 0.5 * float(torch.sum(wq * (phi - tgt) ** 2))

    s.set_velocity_amplitude(1.0)
    s.set_state(phi0, None, 0.0, 0)
    s.forward_ckpt(dt, nsteps, every)
    phiT = s.get_state(want_psi=False)[0]
    gp, _, ga = s.adjoint(wq * (phiT - tgt))
    h = 1e-8
    fdA = (loss(phi0, 1.0 + h) - loss(phi0, 1.0 - h)) / (2 * h)
    print(f"[adjoint] 512 steps: dL/dA adjoint {ga:.10e}, central difference {fdA:.10e}, "
          f"rel {abs(fdA - ga) / abs(ga):.2e}")
    assert abs(fdA - ga) <= 1e-6 * abs(ga), (fdA, ga)
    v = 4.0 * phi0 * (1 - phi0) * (tgt.cpu() - phi0)
    h = 1e-6
    fd = (loss(phi0 + h * v, 1.0) - loss(phi0 - h * v, 1.0)) / (2 * h)
    ad = float(torch.sum(gp.cpu() * v))
    print(f"[adjoint] 512 steps: dL/dphi0 . v adjoint {ad:.10e}, central difference "
          f"{fd:.10e}, rel {abs(fd - ad) / abs(ad):.2e}")
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)


def test_adjoint_matches_oracle_over_checkpoints_and_a_reset():
    """The 64x64 p=3 workload over 40 steps with a reset at step 24 (ten preconditioning
    iterations at step 0 and at step 24) and checkpoints every 16 steps, so the reverse
    sweep crosses two checkpoint boundaries and a reset: GPU VJP against the oracle's
    autograd. dL/dA and the interface-band / interface-direction parts of dL/dphi0 to
    1e-10 (well conditioned there; elsewhere dL/dphi0 takes its direction from rounding
    noise of grad psi, as in the two-step full-size test above)."""
    import dataclasses
    cfg = W.config("C4")
    prm = dataclasses.replace(cfg.params, reset_every=24)
    mesh = cfg.mesh()
    o = Oracle(cfg.ndims, cfg.order, mesh, prm)
    s = _solver(mesh, cfg.order, prm)
    x = o.coords()
    phi0 = torch.tensor(W.ic_phi(x, cfg.centre, cfg.radius, prm.eps_w))
    tgt = torch.tensor(W.ic_phi(x, W.adjoint_target_centre(cfg), cfg.radius, prm.eps_w))
    dt, nsteps, every = cfg.dt(mesh), 40, 16
    wq = o.disc.tdetJ[:, None] * o.disc.tW[None, :]
    with torch.no_grad():
        phiT_o, _, _ = o.run(phi0, None, 0.0, dt, nsteps)
    seed = wq * (phiT_o - tgt)
    ogp, _, oga, _ = _oracle_vjp(o, phi0, None, prm.vel_amp, 0.0, dt, nsteps, 0, seed, None)
    s.set_state(phi0, None, 0.0, 0)
    s.forward_ckpt(dt, nsteps, every)
    phiT = s.get_state(want_psi=False)[0]
    assert _rel(phiT, phiT_o) <= TOL
    gp, _, ga = s.adjoint(seed)
    gp = gp.cpu()
    scale = float(ogp.abs().max())
    band = (phi0 * (1 - phi0)) > 1e-4
    e_band = float(((gp - ogp) * band).abs().max()) / scale
    v = phi0 * (1 - phi0)
    e_dir = abs(float(torch.sum((gp - ogp) * v))) / abs(float(torch.sum(ogp * v)))
    print(f"[adjoint] 40 steps, reset at 24: dL/dA rel {abs(ga - oga) / abs(oga):.2e}, "
          f"band {e_band:.2e}, direction {e_dir:.2e}, all {_rel(gp, ogp):.2e}")
    assert abs(ga - oga) <= TOL * abs(oga), (ga, oga)
    assert e_band <= TOL and e_dir <= TOL


def test_adjoint_fp32_amplitude_gradient_at_full_horizon():
    """FP32 form of the adjoint workload at 512 steps against FP64: dL/dA within 5e-3
    relative. The FP32 forward run differs from FP64 by the rounding of ~2000 stages
    (interface L1 difference ~1e-6 of the loss's scale), and dL/dA is an integral of the
    adjoint against the velocity derivative, whose FP32 relative error grows like the
    forward one times the number of steps (a few 1e-4); measured 7.6e-4."""
    res = []
    for prec in ("fp64", "fp32"):
        cfg, mesh, s, phi0, tgt, wq = _c4_loss_setup(prec)
        s.set_state(phi0, None, 0.0, 0)
        s.forward_ckpt(cfg.dt(mesh), cfg.steps, 32)
        phiT = s.get_state(want_psi=False)[0]
        res.append(s.adjoint(wq.to(s.dtype) * (phiT - tgt.to(s.dtype)))[2])
        del s
    rel = abs(res[1] - res[0]) / abs(res[0])
    print(f"[adjoint] 512 steps: dL/dA fp64 {res[0]:.8e}, fp32 {res[1]:.8e}, rel {rel:.2e}")
    assert rel <= 5e-3
