"""Pins of the oracle's FR residual (§3.1) against mathematics.

P4  corrected gradient exact for globally continuous polynomials (zero jumps).
P5  FR == DG brute force: corrected gradient and corrected divergence equal the DG weak
    forms evaluated with an independent over-integrated quadrature, for discontinuous
    data (pins both lifting signs).
P6  constant state / free stream preservation; phi in {0, 1} gives R_phi = 0.
P7  mass conservation of every residual to round-off (periodic).
P8  p+1 convergence on smooth advection (upwind penalty tau = |v.n|/2).
P9  stationarity of the 1D tanh equilibrium at zero velocity.
P17 energy stability of the linear part (catches penalty/lifting sign errors).
P18 the sharpening flux with the regularised interface normal, exact on polynomials.
"""
import dataclasses
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import Oracle
from oracle import residual as res
from oracle.operators import ElementOperators, monomials


def T(a):
    return torch.as_tensor(a, dtype=torch.float64)


def make(d, p, shape, **kw):
    mesh, prm = W.small_case(d, p, shape, **kw)
    return Oracle(d, p, mesh, prm), mesh, prm


# ---------------------------------------------------------------------------------- P4
@pytest.mark.parametrize("d,p,shape,kw", [
    (2, 3, (3, 4), {}),
    (2, 4, (3, 3), {"perturb": 0.2}),
    (3, 2, (2, 3, 2), {"perturb": 0.2}),
    (2, 2, (4, 4), {"shear": 0.25}),
    (3, 2, (4, 5, 3), {"shear": (0.25, 0.05, 0.2)}),
])
def test_corrected_gradient_exact_on_polynomials(d, p, shape, kw):
    o, mesh, prm = make(d, p, shape, periodic=False, **kw)
    x = o.disc.xs
    sheared = bool(np.any(np.asarray(kw.get("shear", 0.0)) != 0.0))
    for e in monomials(d, p):
        if sheared and sum(e) > p:
            continue
        u = np.prod(x ** np.array(e), axis=-1)
        _, q = res.corrected_gradient(o.disc, T(u))
        for k in range(d):
            ek = np.array(e)
            if ek[k] == 0:
                g = np.zeros_like(u)
            else:
                e2 = ek.copy()
                e2[k] -= 1
                g = ek[k] * np.prod(x ** e2, axis=-1)
            assert np.max(np.abs(q[..., k].numpy() - g)) < 1e-10 * max(1.0, np.abs(g).max())


# ---------------------------------------------------------------------------------- P5
def _dg_weak(d, p, u_nodal, C_fpts, which):
    """Brute-force DG weak forms on the reference element with a (p+3)-point Gauss rule.

    gradient:   W_i q~_k,i = -int u dl_i/dxi_k + sum_faces int C nhat_k l_i
    divergence: W_i div_i  = -int f~ . grad l_i + sum_faces int F~ l_i
    u_nodal is [Nu] (scalar) or [Nu, d] (vector flux), C_fpts is [Nf].
    """
    ops = ElementOperators(d, p)
    b = ops.b
    nq = p + 3
    xq, wq = np.polynomial.legendre.leggauss(nq)
    grids = np.meshgrid(*([xq] * d), indexing="ij")
    Xq = np.stack([g.ravel() for g in grids], -1)             # [nq^d, d]
    Wq = np.prod(np.stack(np.meshgrid(*([wq] * d), indexing="ij"), -1).reshape(-1, d), axis=1)

    def lag(X):          # tensor Lagrange basis values [len(X), Nu]
        out = np.ones((X.shape[0], ops.nupts))
        for k in range(d):
            out *= b.lagrange(X[:, k])[:, ops.upt_idx[:, k]]
        return out

    def dlag(X, k):
        out = np.ones((X.shape[0], ops.nupts))
        for m in range(d):
            T_ = b.dlagrange(X[:, m]) if m == k else b.lagrange(X[:, m])
            out *= T_[:, ops.upt_idx[:, m]]
        return out

    Lq = lag(Xq)
    rhs = np.zeros((ops.nupts, d)) if which == "grad" else np.zeros(ops.nupts)
    if which == "grad":
        uq = Lq @ u_nodal
        for k in range(d):
            rhs[:, k] = -(dlag(Xq, k) * (Wq * uq)[:, None]).sum(0)
    else:
        for k in range(d):
            fq = Lq @ u_nodal[:, k]
            rhs -= (dlag(Xq, k) * (Wq * fq)[:, None]).sum(0)
    # face terms: C (or F~) interpolated on each face from its GL face points
    nfa = ops.nfpts_face
    xq1, wq1 = np.polynomial.legendre.leggauss(nq)
    for f in range(2 * d):
        k, s = divmod(f, 2)
        tdims = [m for m in range(d) if m != k]
        tg = np.meshgrid(*([xq1] * (d - 1)), indexing="ij")
        Tq = np.stack([g.ravel() for g in tg], -1)
        Twq = np.prod(np.stack(np.meshgrid(*([wq1] * (d - 1)), indexing="ij"), -1)
                      .reshape(-1, d - 1), axis=1)
        Xf = np.zeros((Tq.shape[0], d))
        Xf[:, k] = 2 * s - 1
        for q_, m in enumerate(tdims):
            Xf[:, m] = Tq[:, q_]
        # face Lagrange basis over the face's GL points
        Lface = np.ones((Tq.shape[0], nfa))
        for q_ in range(d - 1):
            Lface *= b.lagrange(Tq[:, q_])[:, ops.fpt_tang[f * nfa:(f + 1) * nfa, q_]]
        Cq = Lface @ C_fpts[f * nfa:(f + 1) * nfa]
        Lf = lag(Xf)
        if which == "grad":
            rhs[:, k] += (2 * s - 1) * (Lf * (Twq * Cq)[:, None]).sum(0)
        else:
            rhs += (Lf * (Twq * Cq)[:, None]).sum(0)
    Wn = ops.W
    return rhs / (Wn[:, None] if which == "grad" else Wn)


@pytest.mark.parametrize("d,p", [(2, 2), (2, 3), (2, 4), (3, 2), (3, 3)])
def test_fr_equals_dg_weak_forms(d, p):
    rng = np.random.default_rng(10 + 3 * d + p)
    ops = ElementOperators(d, p)
    u = rng.standard_normal(ops.nupts)
    C = rng.standard_normal(ops.nfpts)
    uf = ops.M0 @ u
    jump = C - uf
    qt = np.stack([ops.D[k] @ u + ops.LiftN[k] @ jump for k in range(d)], -1)
    ref = _dg_weak(d, p, u, C, "grad")
    assert np.max(np.abs(qt - ref)) < 1e-11 * max(1, np.abs(ref).max())
    # divergence with an arbitrary common normal flux
    f = rng.standard_normal((ops.nupts, d))
    F = rng.standard_normal(ops.nfpts)
    fperp = sum((ops.M0 @ f[:, k]) * ops.nhat[:, k] for k in range(d))
    div = sum(ops.D[k] @ f[:, k] for k in range(d)) + ops.LiftDiv @ (F - fperp)
    ref = _dg_weak(d, p, f, F, "div")
    assert np.max(np.abs(div - ref)) < 1e-11 * max(1, np.abs(ref).max())


# ---------------------------------------------------------------------------------- P6
@pytest.mark.parametrize("d,p,shape,kw", [
    (2, 3, (4, 5), {}),
    (2, 4, (4, 4), {"perturb": 0.2}),
    (2, 3, (4, 4), {"shear": 0.25}),
    (3, 3, (3, 3, 4), {"perturb": 0.2}),
    (3, 2, (4, 5, 3), {"shear": (0.25, 0.05, 0.2)}),
])
def test_free_stream_and_constant_state(d, p, shape, kw):
    """Uniform v: (a) on a periodic mesh a constant psi is preserved, and so is a
    constant phi in {0, 1} (where phi(1-phi) vanishes) for ANY psi; (b) on a copy-BC mesh
    a constant phi with a linear level set psi (|grad psi| = 1, so a constant normal) is
    preserved and psi is advected exactly: R_psi = -v.grad(psi). A constant psi leaves
    the normal undefined, so a constant phi strictly inside (0, 1) is not a steady state
    of the discrete system; that case is not asserted."""
    o, mesh, prm = make(d, p, shape, vel_u0=(0.7, -0.4, 0.3), **kw)
    E, Nu = o.disc.E, o.ops.nupts
    scale = 1.0 / min(o.disc.detJ) ** (1.0 / d)
    rng = np.random.default_rng(0)
    for c1, c2 in [(0.0, -0.2), (1.0, 0.5), (0.0, 2.0)]:
        Rp, Rs = o.residual(T(np.full((E, Nu), c1)), T(np.full((E, Nu), c2)), 0.0)
        assert float(Rp.abs().max()) < 1e-13 * scale
        assert float(Rs.abs().max()) < 1e-13 * scale
    psi = T(rng.standard_normal((E, Nu)))
    for c in (0.0, 1.0):
        Rp, _ = o.residual(T(np.full((E, Nu), c)), psi, 0.0)
        assert float(Rp.abs().max()) < 1e-12 * scale
    o2, _, _ = make(d, p, shape, vel_u0=(0.7, -0.4, 0.3), periodic=False, **kw)
    x = o2.disc.xs
    a = np.array([0.6, 0.8, 0.0][:d]) if d == 2 else np.array([0.48, 0.6, 0.64])
    lin = x @ a - 0.3
    v = np.array([0.7, -0.4, 0.3][:d])
    for c1 in (0.3, 0.9):
        Rp, Rs = o2.residual(T(np.full((E, Nu), c1)), T(lin), 0.0)
        assert float(Rp.abs().max()) < 1e-12 * scale
        assert float((Rs + float(v @ a)).abs().max()) < 1e-12 * scale


# ---------------------------------------------------------------------------------- P7
@pytest.mark.parametrize("d,p,shape,kind,kw", [
    (2, 3, (5, 4), W.VEL_UNIFORM, {"perturb": 0.2}),
    (2, 4, (6, 6), W.VEL_SINGLE_VORTEX, {"perturb": 0.2}),
    (3, 3, (3, 4, 3), W.VEL_LEVEQUE3D, {"perturb": 0.2}),
    (3, 2, (4, 5, 3), W.VEL_LEVEQUE3D, {"shear": (0.25, 0.05, 0.2)}),
])
def test_mass_conservation_per_residual(d, p, shape, kind, kw):
    o, mesh, prm = make(d, p, shape, vel_kind=kind, **kw)
    E, Nu = o.disc.E, o.ops.nupts
    rng = np.random.default_rng(1)
    phi = T(rng.uniform(0, 1, (E, Nu)))
    psi = T(rng.standard_normal((E, Nu)))
    for t in (0.0, 0.37):
        Rp, Rs = o.residual(phi, psi, t)
        sc = float(torch.sum(o.disc.tdetJ[:, None] * o.disc.tW * Rp.abs()))
        assert abs(float(o.integral(Rp))) < 1e-14 * max(1.0, sc)
        assert abs(float(o.integral(Rs))) < 1e-14 * max(1.0, sc)
    sgn = torch.tanh(psi)
    Rpc = o.precond_residual(psi, sgn)
    # the preconditioning residual conserves up to its source term
    _, q = res.corrected_gradient(o.disc, psi)
    S = sgn * (1 - torch.linalg.vector_norm(q, dim=-1))
    assert abs(float(o.integral(Rpc - S))) < 1e-13 * max(1.0, float(o.integral((Rpc - S).abs())))


# ---------------------------------------------------------------------------------- P8
@pytest.mark.parametrize("p", [2, 3])
def test_convergence_order_smooth_advection(p):
    errs = []
    Ns = [4, 8, 16]
    for N in Ns:
        mesh, prm = W.small_case(2, p, (N, N), vel_u0=(1.0, 1.0), gamma=0.0, eps=0.0,
                                 tau=0.5)
        o = Oracle(2, p, mesh, prm)
        x = o.disc.xs
        u0 = np.sin(2 * np.pi * x[..., 0]) * np.sin(2 * np.pi * x[..., 1])
        phi = T(u0)
        tend = 0.25
        nst = int(math.ceil(tend / (0.05 / N)))
        dt = tend / nst
        t = 0.0
        psi = phi.clone()
        for _ in range(nst):
            phi, psi = o.step(phi, psi, t, dt)
            t += dt
        xe = x - tend
        ue = np.sin(2 * np.pi * xe[..., 0]) * np.sin(2 * np.pi * xe[..., 1])
        err = math.sqrt(float(o.integral((phi - T(ue)) ** 2)))
        errp = math.sqrt(float(o.integral((psi - T(ue)) ** 2)))
        assert abs(err - errp) < 1e-12   # both rows are the same advection here
        errs.append(err)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] > p + 0.7, (errs, rates)


# ---------------------------------------------------------------------------------- P9
def test_tanh_equilibrium_closed_form():
    """With eps_w = eps/gamma and n = grad(d), eps grad(phi) = gamma phi(1-phi) n, so the
    viscous flux of the localized equation vanishes identically."""
    gamma, eps = 0.09, 0.06 / 64 / 3
    eps_w = eps / gamma
    x = np.linspace(-0.05, 0.05, 101)
    phi = W.tanh_profile(x, eps_w)
    dphi = (1 - np.tanh(x / (2 * eps_w)) ** 2) / (4 * eps_w)
    assert np.max(np.abs(eps * dphi - gamma * phi * (1 - phi))) < 1e-15 * np.max(eps * dphi) * 10


@pytest.mark.parametrize("p,N", [(3, 16), (4, 16)])
def test_tanh_equilibrium_discrete_drift(p, N):
    """Strip N x 2 (x copy-BC, y periodic), psi = x - 1/2, v = 0: the IC profile at the
    paper's eps is under-resolved, so it drifts, but by less than 1% of h over t = 1, with
    mass conserved."""
    h = 1.0 / N
    mesh, prm = W.small_case(2, p, (N, 2), periodic=[False, True], vel_u0=(0.0, 0.0))
    # planes for y: the strip has two elements of height h
    mesh = W.box_mesh([W.uniform_planes(N), W.uniform_planes(2, 0.0, 2 * h)], [False, True])
    prm = W.default_params(2, p, h, vel_u0=(0.0, 0.0, 0.0))
    o = Oracle(2, p, mesh, prm)
    x = o.disc.xs[..., 0]
    phi0 = T(W.tanh_profile(x - 0.5, prm.eps / prm.gamma))
    psi = T(x - 0.5)
    R, Rs = o.residual(phi0, psi, 0.0)
    assert float(Rs.abs().max()) < 1e-12
    dt = 0.1 * h / prm.gamma / 8
    nst = int(math.ceil(1.0 / dt))
    dt = 1.0 / nst
    phi = phi0
    m0 = float(o.mass(phi0))
    for _ in range(nst):
        phi, psi = o.step(phi, psi, 0.0, dt)
    drift = float(o.l1(phi, phi0)) / (2 * h)     # per unit interface length
    assert drift < 0.01 * h
    assert abs(float(o.mass(phi)) - m0) < 1e-13


def test_tanh_equilibrium_residual_converges():
    """At a fixed eps = 0.004 (eps_w = eps/gamma = 0.044, a resolved profile) the t = 0
    residual of the equilibrium profile drops by more than 3.5x per halving of h."""
    vals = []
    for N in (16, 32, 64):
        h = 1.0 / N
        mesh = W.box_mesh([W.uniform_planes(N), W.uniform_planes(1, 0.0, h)], [False, True])
        prm = W.default_params(2, 3, h, vel_u0=(0.0, 0.0, 0.0), eps=0.004)
        o = Oracle(2, 3, mesh, prm)
        x = o.disc.xs[..., 0]
        phi0 = T(W.tanh_profile(x - 0.5, prm.eps / prm.gamma))
        R, _ = o.residual(phi0, T(x - 0.5), 0.0)
        vals.append(float(R.abs().max()))
    assert vals[0] / vals[1] > 3.5 and vals[1] / vals[2] > 3.5, vals


# ---------------------------------------------------------------------------------- P17
def _assemble(o, which, E, Nu):
    n = E * Nu
    A = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        u = T(e.reshape(E, Nu))
        if which == "phi":
            R, _ = o.residual(u, torch.zeros_like(u), 0.0)
        else:
            _, R = o.residual(torch.zeros_like(u), u, 0.0)
        A[:, c] = R.reshape(-1).numpy()
    return A


@pytest.mark.parametrize("p", [2, 3])
def test_energy_stability_linear_operator(p):
    """gamma = 0 makes the phi row linear advection + LDG diffusion (|v| eps) + penalty;
    its symmetric part in the quadrature inner product must be negative semidefinite."""
    mesh, prm = W.small_case(2, p, (3, 3), vel_u0=(1.0, 0.5), gamma=0.0, eps=0.05, tau=0.1)
    o = Oracle(2, p, mesh, prm)
    E, Nu = o.disc.E, o.ops.nupts
    w = (o.disc.detJ[:, None] * o.ops.W[None, :]).reshape(-1)
    sq = np.sqrt(w)
    for which in ("phi", "psi"):
        A = _assemble(o, which, E, Nu)
        B = sq[:, None] * A / sq[None, :]
        S = 0.5 * (B + B.T)
        lam = np.linalg.eigvalsh(S)
        rho = np.max(np.abs(np.linalg.eigvals(A)))
        assert lam.max() < 1e-12 * rho, (which, lam.max(), rho)


def test_energy_stability_detects_flipped_penalty():
    """The same check fails with the literal (anti-dissipative) penalty sign."""
    mesh, prm = W.small_case(2, 2, (3, 3), vel_u0=(1.0, 0.5), gamma=0.0, eps=0.05, tau=-0.1)
    o = Oracle(2, 2, mesh, prm)
    E, Nu = o.disc.E, o.ops.nupts
    w = (o.disc.detJ[:, None] * o.ops.W[None, :]).reshape(-1)
    sq = np.sqrt(w)
    A = _assemble(o, "psi", E, Nu)
    B = sq[:, None] * A / sq[None, :]
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).max() > 1e-3


def test_residual_is_local_to_one_element_layer():
    """The residual of an element depends only on the elements within one layer of it
    (diagonals included): on a copy-boundary sub-block cut out of a periodic mesh, every
    element off the sub-block's outer layer has exactly the full-mesh residual. (The
    full-size GPU tests sample their outputs this way.)"""
    import torch as _t
    from oracle import residual as ores
    mesh, prm = W.small_case(3, 2, (9, 9, 9), perturb=0.2, vel_kind=W.VEL_LEVEQUE3D,
                             vel_period=3.0)
    o = Oracle(3, 2, mesh, prm)
    x = o.coords()
    c = (0.45, 0.5, 0.5)
    phi = _t.tensor(W.ic_phi(x, c, 0.25, 0.05))
    psi = _t.tensor(W.signed_distance_ball(x, c, 0.25))
    Rp, Rs = o.residual(phi, psi, 0.3)
    sgn = ores.smeared_sign(o.disc, prm, phi - 0.5)
    Rpc = o.precond_residual(psi, sgn)
    m, lo = 7, (1, 2, 1)
    planes = [np.asarray(mesh.planes[k])[lo[k]:lo[k] + m + 1] for k in range(3)]
    sub = W.box_mesh(planes, [False] * 3)
    e = np.arange(sub.nelem)
    ck = [(e // m ** k) % m for k in range(3)]
    full = _t.as_tensor((ck[0] + lo[0]) + 9 * ((ck[1] + lo[1]) + 9 * (ck[2] + lo[2])))
    inner = _t.as_tensor(np.all([(a >= 1) & (a <= m - 2) for a in ck], axis=0))
    os_ = Oracle(3, 2, sub, prm)
    rp, rs = os_.residual(phi[full], psi[full], 0.3)
    ssgn = ores.smeared_sign(os_.disc, prm, phi[full] - 0.5)
    rpc = os_.precond_residual(psi[full], ssgn)
    for a, b in ((rp, Rp), (rs, Rs), (ssgn, sgn), (rpc, Rpc)):
        assert _t.equal(a[inner], b[full][inner])
        assert float((a[~inner] - b[full][~inner]).abs().max()) > 0   # the boundary differs


def test_unpreconditioned_normal_reduces_to_psi_equal_phi():
    """The unpreconditioned form takes the interface normal from phi (the original
    conservative phase field, §2): its phi residual is the preconditioned one evaluated
    with psi := phi, for any psi, and its psi residual is unchanged."""
    import dataclasses
    import torch as _t
    mesh, prm = W.small_case(2, 3, (5, 4), vel_kind=W.VEL_SINGLE_VORTEX, vel_period=4.0)
    o0 = Oracle(2, 3, mesh, prm)
    o1 = Oracle(2, 3, mesh, dataclasses.replace(prm, normal_mode=W.NORMAL_PHI))
    x = o0.coords()
    rng = np.random.default_rng(4)
    phi = _t.tensor(W.ic_phi(x, (0.5, 0.55), 0.3, 0.05))
    psi = _t.tensor(rng.standard_normal(phi.shape))
    Rp1, Rs1 = o1.residual(phi, psi, 0.2)
    Rp0, _ = o0.residual(phi, phi, 0.2)
    _, Rs0 = o0.residual(phi, psi, 0.2)
    assert _t.equal(Rp1, Rp0)
    assert _t.equal(Rs1, Rs0)
    # and it differs from the preconditioned residual with the given psi
    Rpp, _ = o0.residual(phi, psi, 0.2)
    assert float((Rpp - Rp1).abs().max()) > 1e-3 * float(Rp1.abs().max())


@pytest.mark.parametrize("p", [2, 3])
def test_sharpening_flux_regularised_normal(p):
    """The sharpening part of the phi flux, max(gamma, |v|) gamma phi (1 - phi) n with the
    regularised normal n = grad psi / sqrt(|grad psi|^2 + delta_n^2) (§2; the regularisation
    is the reading recorded for |grad psi| -> 0). At rest (v = 0, so the multiplier is gamma)
    with eps = 0, psi = x and phi = a + b x on a non-periodic mesh (copy boundaries), every
    flux is a polynomial of degree <= p that FR differentiates exactly, so
    R_phi = -gamma^2 b (1 - 2a - 2b x) / sqrt(1 + delta_n^2). delta_n = 1 makes the
    regularisation visible (the factor 1/sqrt 2)."""
    mesh, prm = W.small_case(2, p, (3, 2), periodic=False, vel_u0=(0.0, 0.0, 0.0))
    prm = dataclasses.replace(prm, eps=0.0, delta_n=1.0)
    o = Oracle(2, p, mesh, prm)
    x = o.coords()
    a, b = 0.3, 0.2
    phi = torch.as_tensor(a + b * x[..., 0], dtype=torch.float64)
    psi = torch.as_tensor(x[..., 0], dtype=torch.float64)
    Rphi, Rpsi = o.residual(phi, psi, 0.0)
    g = prm.gamma
    expect = -g * g * b * (1.0 - 2.0 * a - 2.0 * b * x[..., 0]) / np.sqrt(2.0)
    assert np.abs(Rphi.numpy() - expect).max() < 1e-12
    assert float(torch.max(torch.abs(Rpsi))) < 1e-13
