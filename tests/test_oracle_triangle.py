"""Pins of the oracle's triangle element (§3.1 on triangles; the uniform split triangular
mesh of §4.2) against mathematics, with quadratures of the tests' own (a collapsed
Gauss-Legendre rule on the triangle, Gauss-Legendre on the edges) that share nothing with
the oracle's closed-form moments:

P2   interpolation to the flux points and derivatives at the solution points exact on P_p;
     the nodal weights W integrate P_p exactly
P5   FR == DG: the corrected gradient and divergence equal the DG weak forms with arbitrary
     (discontinuous) common values, evaluated by over-integration (pins both liftings)
P12  sensor modes: Parseval (sum chi^2 = int u^2), top modes orthogonal to P_{p-1}, a single
     top mode gives nu_max, degree p - 1 gives 0
P4   exact gradient of a global polynomial of degree <= p on a copy-boundary mesh
P6   constant state / free stream preservation, periodic and perturbed meshes
P7   mass conservation of every residual
P8   p + 1 convergence of smooth advection with the upwind-equivalent penalty
P17  energy stability of the linear part in the mass-matrix norm (and the flipped penalty
     fails it)
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import Oracle
from oracle import residual as res
from oracle.triangle import TriangleOperators


def T(a):
    return torch.as_tensor(a, dtype=torch.float64)


def collapsed_rule(n=12):
    """Points and weights on the reference triangle from the square [0,1]^2 by
    (a, b) -> (a, b (1 - a)), Jacobian 1 - a, Gauss-Legendre in each direction."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    A, B = np.meshgrid(x, x, indexing="ij")
    WA, WB = np.meshgrid(w, w, indexing="ij")
    r = A.reshape(-1)
    s = (B * (1.0 - A)).reshape(-1)
    wt = (WA * WB * (1.0 - A)).reshape(-1)
    return np.stack([r, s], -1), wt


def lagrange_at(ops, x):
    """Nodal basis values l_i(x) [N, Nu] and derivatives [2][N, Nu] at arbitrary points,
    from the oracle's coefficients (the basis itself is what is being pinned through the
    operators it produces)."""
    C = ops.lagrange_coeffs
    return ops.mono(x) @ C, [ops.mono(x, k) @ C for k in range(2)]


MONO = lambda x, a, b: x[..., 0] ** a * x[..., 1] ** b


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_operators_exact_on_polynomials(p):
    ops = TriangleOperators(p)
    xu, xf = ops.upt_ref, ops.fpt_ref
    qx, qw = collapsed_rule()
    for n in range(p + 1):
        for b in range(n + 1):
            a = n - b
            u = MONO(xu, a, b)
            assert np.abs(ops.M0 @ u - MONO(xf, a, b)).max() < 1e-12
            du = [a * MONO(xu, max(a - 1, 0), b) if a else 0 * u,
                  b * MONO(xu, a, max(b - 1, 0)) if b else 0 * u]
            for k in range(2):
                assert np.abs(ops.D[k] @ u - du[k]).max() < 1e-11
            assert abs(ops.W @ u - qw @ MONO(qx, a, b)) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_fr_equals_dg_weak_forms(p):
    """For every test function l_m: (M q~_k)_m = -int u d_k l_m + sum_edges int C nhat_k l_m
    and (M div)_m = -int f~ . grad l_m + sum_edges int F~ l_m, with u of degree p, C and F~
    arbitrary at the flux points (each interpolated along its edge by the degree-p
    polynomial through the edge's p + 1 Gauss points), all integrals over-integrated."""
    ops = TriangleOperators(p)
    rng = np.random.default_rng(p)
    Nu, Nf, n = ops.nupts, ops.nfpts, p + 1
    qx, qw = collapsed_rule()
    Lq, dLq = lagrange_at(ops, qx)
    M = (Lq * qw[:, None]).T @ Lq                       # mass matrix by over-integration
    u = rng.standard_normal(Nu)
    C = rng.standard_normal(Nf)
    f = rng.standard_normal((Nu, 2))
    F = rng.standard_normal(Nf)
    # edge integrals: high-order Gauss rule along each edge, the flux-point data
    # interpolated in the edge parameter
    xi_f, _ = np.polynomial.legendre.leggauss(n)
    xg, wg = np.polynomial.legendre.leggauss(3 * n + 4)
    verts = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    edges = [(0, 1), (1, 2), (2, 0)]

    def edge_integrals(vals):
        """sum over edges of int (interpolant of vals on the edge) l_m nhat ds -> [Nu, 2]
        and without nhat -> [Nu]"""
        out_n = np.zeros((Nu, 2))
        out = np.zeros(Nu)
        for e, (a, b) in enumerate(edges):
            va, vb = verts[a], verts[b]
            L = np.linalg.norm(vb - va)
            tang = (vb - va) / L
            nrm = np.array([tang[1], -tang[0]])
            pts = va[None, :] + 0.5 * (1 + xg)[:, None] * (vb - va)[None, :]
            # 1D Lagrange basis through the edge's Gauss points, at the fine points
            lag = np.ones((xg.size, n))
            for t in range(n):
                for q in range(n):
                    if q != t:
                        lag[:, t] *= (xg - xi_f[q]) / (xi_f[t] - xi_f[q])
            v = lag @ vals[e * n:(e + 1) * n]
            Lm, _ = lagrange_at(ops, pts)
            ds = 0.5 * L * wg
            out += (Lm * (v * ds)[:, None]).sum(0)
            out_n += (Lm * (v * ds)[:, None]).sum(0)[:, None] * nrm[None, :]
        return out_n, out

    uq = Lq @ u
    Cn, _ = edge_integrals(C)
    for k in range(2):
        qk = ops.D[k] @ u + ops.LiftN[k] @ (C - ops.M0 @ u)
        rhs = -(dLq[k] * (uq * qw)[:, None]).sum(0) + Cn[:, k]
        scale = (np.abs(M) @ np.abs(qk)).max() + np.abs(rhs).max()
        assert np.abs(M @ qk - rhs).max() < 1e-10 * scale
    fperp = sum((ops.M0 @ f[:, k]) * ops.nhat[:, k] for k in range(2))
    div = sum(ops.D[k] @ f[:, k] for k in range(2)) + ops.LiftDiv @ (F - fperp)
    _, Fi = edge_integrals(F)
    fq = Lq @ f
    rhs = -sum((dLq[k] * (fq[:, k] * qw)[:, None]).sum(0) for k in range(2)) + Fi
    scale = (np.abs(M) @ np.abs(div)).max() + np.abs(rhs).max()
    assert np.abs(M @ div - rhs).max() < 1e-10 * scale


@pytest.mark.parametrize("p", [2, 3, 4])
def test_sensor_modes(p):
    ops = TriangleOperators(p)
    rng = np.random.default_rng(10 + p)
    qx, qw = collapsed_rule()
    Lq, _ = lagrange_at(ops, qx)
    u = rng.standard_normal(ops.nupts)
    chi = ops.Vt_inv @ u
    # Parseval, to the floor of evaluating the interpolant at the quadrature points
    assert abs(np.sum(chi ** 2) - qw @ (Lq @ u) ** 2) < 1e-10 * np.sum(chi ** 2)
    # a polynomial of degree p - 1 has no top-mode energy
    xu = ops.upt_ref
    low = sum(rng.standard_normal() * MONO(xu, n - b, b) for n in range(p) for b in range(n + 1))
    chi = ops.Vt_inv @ low
    assert np.sum(ops.topmask * chi ** 2) < 1e-26 * np.sum(chi ** 2)
    # the sensor through the residual module: one top mode -> nu_max; degree p - 1 -> 0
    mesh = W.split_tri_mesh(2)
    prm = W.default_params(2, p, 0.5)
    o = Oracle(2, p, mesh, prm)
    E = o.disc.E
    # the top modes are exactly those orthogonal to P_{p-1} (found here by quadrature), and
    # each of them alone switches the sensor fully on
    ortho_low = []
    for j in range(ops.nupts):
        psi_q = Lq @ ops.Vt[:, j]
        ip = [abs(qw @ (psi_q * MONO(qx, n - b, b))) for n in range(p) for b in range(n + 1)]
        ortho_low.append(max(ip) < 1e-10)
    assert np.array_equal(np.array(ortho_low), ops.topmask > 0)
    assert int(ops.topmask.sum()) == p + 1
    for top in np.nonzero(ops.topmask)[0]:
        mode = ops.Vt[:, top]
        nu = res.sensor(o.disc, prm, T(np.tile(mode, (E, 1))))
        assert torch.allclose(nu, torch.full_like(nu, prm.nu_max), rtol=0, atol=1e-15)
    nu = res.sensor(o.disc, prm, T(np.tile(low, (E, 1))))
    assert float(nu.abs().max()) == 0.0


@pytest.mark.parametrize("p", [2, 3, 4])
def test_corrected_gradient_exact_on_polynomials(p):
    mesh = W.split_tri_mesh(3, periodic=False, perturb=0.15)
    prm = W.default_params(2, p, 1 / 3)
    o = Oracle(2, p, mesh, prm)
    x = o.disc.xs
    for n in range(p + 1):
        for b in range(n + 1):
            a = n - b
            u = MONO(x, a, b)
            _, q = res.corrected_gradient(o.disc, T(u))
            g = [a * MONO(x, max(a - 1, 0), b) if a else 0 * u,
                 b * MONO(x, a, max(b - 1, 0)) if b else 0 * u]
            for k in range(2):
                assert np.abs(q[..., k].numpy() - g[k]).max() < 1e-10 * max(1.0, np.abs(g[k]).max())


@pytest.mark.parametrize("p,perturb", [(2, 0.0), (3, 0.2), (4, 0.0)])
def test_free_stream_and_mass_conservation(p, perturb):
    mesh = W.split_tri_mesh(4, perturb=perturb)
    prm = W.default_params(2, p, 0.25, vel_u0=(0.7, -0.4, 0.0))
    o = Oracle(2, p, mesh, prm)
    E, Nu = o.disc.E, o.ops.nupts
    scale = 4.0
    for c1, c2 in [(0.0, -0.2), (1.0, 0.5)]:
        Rp, Rs = o.residual(T(np.full((E, Nu), c1)), T(np.full((E, Nu), c2)), 0.0)
        assert float(Rp.abs().max()) < 1e-12 * scale and float(Rs.abs().max()) < 1e-12 * scale
    rng = np.random.default_rng(p)
    psi = T(rng.standard_normal((E, Nu)))
    for c in (0.0, 1.0):
        Rp, _ = o.residual(T(np.full((E, Nu), c)), psi, 0.0)
        assert float(Rp.abs().max()) < 1e-11 * scale
    # conservation of every residual, vortex field
    prm2 = W.default_params(2, p, 0.25, vel_kind=W.VEL_SINGLE_VORTEX, vel_period=8.0)
    o2 = Oracle(2, p, mesh, prm2)
    phi = T(rng.uniform(0, 1, (E, Nu)))
    for t in (0.0, 0.9):
        Rp, Rs = o2.residual(phi, psi, t)
        sc = float(o2.integral(Rp.abs()))
        assert abs(float(o2.integral(Rp))) < 1e-14 * max(1.0, sc)
        assert abs(float(o2.integral(Rs))) < 1e-14 * max(1.0, sc)


@pytest.mark.parametrize("p", [2, 3])
def test_convergence_order_smooth_advection(p):
    errs = []
    Ns = [4, 8, 16]
    for N in Ns:
        mesh = W.split_tri_mesh(N)
        # tau = |v.n|/2 at most makes the penalty at least upwind on every edge
        prm = W.default_params(2, p, 1.0 / N, vel_u0=(1.0, 0.5, 0.0), gamma=0.0, eps=0.0,
                               tau=0.75)
        o = Oracle(2, p, mesh, prm)
        x = o.disc.xs
        phi = T(np.sin(2 * np.pi * x[..., 0]) * np.sin(2 * np.pi * x[..., 1]))
        tend = 0.2
        nst = int(math.ceil(tend / (0.04 / N)))
        dt = tend / nst
        t = 0.0
        psi = phi.clone()
        for _ in range(nst):
            phi, psi = o.step(phi, psi, t, dt)
            t += dt
        xe = x - np.array([1.0, 0.5]) * tend
        ue = np.sin(2 * np.pi * xe[..., 0]) * np.sin(2 * np.pi * xe[..., 1])
        errs.append(math.sqrt(float(o.integral((phi - T(ue)) ** 2))))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] > p + 0.6, (errs, rates)


def _stability_max(o, which):
    E, Nu = o.disc.E, o.ops.nupts
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
    # the mass-matrix inner product, element blocks det J M
    qx, qw = collapsed_rule()
    Lq, _ = lagrange_at(o.ops, qx)
    Mref = (Lq * qw[:, None]).T @ Lq
    Mg = np.zeros((n, n))
    for e in range(E):
        Mg[e * Nu:(e + 1) * Nu, e * Nu:(e + 1) * Nu] = o.disc.detJ[e] * Mref
    L = np.linalg.cholesky(Mg)
    S = 0.5 * (Mg @ A + (Mg @ A).T)
    Li = np.linalg.inv(L)
    lam = np.linalg.eigvalsh(Li @ S @ Li.T)
    rho = np.max(np.abs(np.linalg.eigvals(A)))
    return lam.max(), rho


@pytest.mark.parametrize("p", [2, 3])
def test_energy_stability_linear_operator(p):
    mesh = W.split_tri_mesh(2)
    prm = W.default_params(2, p, 0.5, vel_u0=(1.0, 0.5, 0.0), gamma=0.0, eps=0.05, tau=0.1)
    o = Oracle(2, p, mesh, prm)
    for which in ("phi", "psi"):
        lmax, rho = _stability_max(o, which)
        assert lmax < 1e-12 * rho, (which, lmax, rho)


def test_energy_stability_detects_flipped_penalty():
    mesh = W.split_tri_mesh(2)
    prm = W.default_params(2, 2, 0.5, vel_u0=(1.0, 0.5, 0.0), gamma=0.0, eps=0.05, tau=-0.1)
    o = Oracle(2, 2, mesh, prm)
    lmax, rho = _stability_max(o, "psi")
    assert lmax > 1e-3
