"""Pins of the oracle's preconditioning sub-solver (§2 reset and Eq. lsequation, §3.2).

P12 sensor and viscosity ramp: closed forms of Eqs. resolutionIndicator and nu_s on
    fields with a prescribed top-mode energy fraction.
P13 eikonal fixed point and the sign of the source term.
P14 the logit reset inverts the tanh kernel of §2 to the accuracy of float64.
Options of the printed forms: the smeared sign with the current |grad psi| (§2, text after
Eq. lsequation) against closed forms, and the RMS stop rule of §3.2 against its fixed point,
a closed-form first iterate and the first-crossing property.
"""
import math

import numpy as np
import pytest
import torch

import dataclasses

import workloads as W
from oracle import Oracle
from oracle import residual as res


def T(a):
    return torch.as_tensor(a, dtype=torch.float64)


def ramp(s, s0, kap, numax):
    if s < s0 - kap:
        return 0.0
    if s > s0 + kap:
        return numax
    return 0.5 * numax * (1 + math.sin(math.pi * (s - s0) / (2 * kap)))


@pytest.mark.parametrize("d,p", [(2, 3), (2, 4), (3, 3)])
def test_sensor_closed_form(d, p):
    targets = [-14.0, -10.0 - 1e-9, -9.5, -7.0, -5.0, -2.5, -1e-9, 0.0]
    shape = (len(targets),) + (1,) * (d - 1)
    mesh, prm = W.small_case(d, p, shape)
    o = Oracle(d, p, mesh, prm)
    b = o.ops.b
    xi = o.ops.upt_ref
    # modes (0,...,0) and (p, 0, ..., 0) of the orthonormal tensor Legendre basis
    m0 = np.prod([b.psi(0, xi[:, k]) for k in range(d)], axis=0)
    mt = b.psi(p, xi[:, 0]) * np.prod([b.psi(0, xi[:, k]) for k in range(1, d)], axis=0)
    psi = []
    for s in targets:
        r = 10.0 ** s
        a = math.sqrt(r / (1 - r)) if r < 1 else None
        psi.append(mt if a is None else m0 + a * mt)
    nu = o.sensor(T(np.array(psi))).numpy()
    for s, v in zip(targets, nu):
        assert abs(v - ramp(s, prm.s0, prm.kappa, prm.nu_max)) < 1e-12 * prm.nu_max, (s, v)
    assert abs(nu[-1] - prm.nu_max) < 1e-15          # a single top mode: s = 0 -> nu_max
    assert abs(nu[4] - 0.5 * prm.nu_max) < 1e-12 * prm.nu_max


@pytest.mark.parametrize("d,p", [(2, 2), (2, 4), (3, 3)])
def test_sensor_zero_below_top_degree(d, p):
    mesh, prm = W.small_case(d, p, (2,) * d, periodic=False)
    o = Oracle(d, p, mesh, prm)
    x = o.disc.xs
    rng = np.random.default_rng(5)
    # any polynomial of degree <= p-1 in each variable has no top mode
    u = np.zeros(x.shape[:-1])
    for e in np.ndindex(*([p] * d)):
        u += rng.standard_normal() * np.prod(x ** np.array(e), axis=-1)
    assert float(o.sensor(T(u)).abs().max()) == 0.0
    assert float(o.sensor(T(np.zeros_like(u))).abs().max()) == 0.0


def test_sensor_ramp_is_c1():
    s0, kap, numax = -5.0, 5.0, 1.0
    for edge in (s0 - kap, s0 + kap):
        e = 1e-6
        left = (ramp(edge, s0, kap, numax) - ramp(edge - e, s0, kap, numax)) / e
        right = (ramp(edge + e, s0, kap, numax) - ramp(edge, s0, kap, numax)) / e
        assert abs(left) < 1e-5 and abs(right) < 1e-5


@pytest.mark.parametrize("d,p", [(2, 3), (3, 2)])
def test_eikonal_fixed_point_and_sign(d, p):
    mesh, prm = W.small_case(d, p, (3,) * d, periodic=False, perturb=0.15)
    o = Oracle(d, p, mesh, prm)
    x = o.disc.xs
    a = np.zeros(d)
    a[0], a[1] = 0.6, 0.8
    psi = T(x @ a - 0.4)                         # |grad psi| = 1
    sgn = res.smeared_sign(o.disc, prm, psi)
    assert float(o.sensor(psi).abs().max()) == 0.0
    R = o.precond_residual(psi, sgn)
    assert float(R.abs().max()) < 1e-12
    # psi = 2(x - 1/2): |grad psi| = 2, so dpsi/dtau = sgn (1 - 2) = -sgn
    psi2 = T(2 * (x[..., 0] - 0.5))
    sgn2 = res.smeared_sign(o.disc, prm, psi2)
    assert float((sgn2 - torch.tanh(psi2 / 2)).abs().max()) < 1e-14
    R2 = o.precond_residual(psi2, sgn2)
    assert float((R2 + sgn2).abs().max()) < 1e-12
    # one pseudo step moves |grad psi| toward 1
    psi3, _ = o.precondition(T(x[..., 0] + 0.0) * 2 - 0.5, iters=1)


def test_logit_reset_inverts_kernel():
    mesh, prm = W.small_case(2, 3, (4, 4))
    prm.reset_mode = W.RESET_LOGIT
    o = Oracle(2, 3, mesh, prm)
    eps_w = prm.eps_w
    z = np.linspace(-20, 20, 4001)
    psi_d = z * eps_w
    phi = W.tanh_profile(psi_d, eps_w)
    psi = o.reset_psi(T(phi)).numpy()
    bound = 4e-16 * (1 + np.exp(np.abs(z))) * eps_w
    assert np.all(np.abs(psi - psi_d) <= bound)
    # the clamp keeps the transform finite at phi = 0 and 1
    ends = o.reset_psi(T(np.array([0.0, 1.0]))).numpy()
    assert np.all(np.isfinite(ends)) and ends[0] < 0 < ends[1]


def test_linear_reset_and_precondition_shape():
    cfg = W.config("C1")
    mesh = cfg.mesh()
    o = Oracle(2, 3, mesh, cfg.params)
    phi = T(W.ic_phi(o.coords(), cfg.centre, cfg.radius, cfg.params.eps_w))
    psi0 = o.reset_psi(phi)
    assert float((psi0 - (phi - 0.5)).abs().max()) == 0.0
    psi, sgn = o.precondition(phi)
    # the zero level set barely moves: sign of psi agrees with phi - 1/2 where
    # |phi - 1/2| > 0.25
    far = (phi - 0.5).abs() > 0.25
    assert bool(torch.all(torch.sign(psi[far]) == torch.sign((phi - 0.5)[far])))


@pytest.mark.parametrize("d,p", [(2, 3), (3, 2)])
def test_current_sign_closed_forms(d, p):
    mesh, prm = W.small_case(d, p, (3,) * d, periodic=False, perturb=0.15)
    cur = dataclasses.replace(prm, sgn_mode=W.SGN_CURRENT)
    o, oc = Oracle(d, p, mesh, prm), Oracle(d, p, mesh, cur)
    x = o.disc.xs
    rng = np.random.default_rng(4)
    psi0 = T(np.tanh(3 * (x[..., 0] - 0.45)) + 0.05 * rng.standard_normal(x.shape[:2]))
    # at psi = psi0 the printed sign is the sign of the reset
    R_reset = o.precond_residual(psi0, res.smeared_sign(o.disc, prm, psi0))
    assert torch.equal(oc.precond_residual(psi0, None, psi0), R_reset)
    # psi = 2(x - 1/2): no top modes (nu = 0), no jumps, |grad psi| = 2, so
    # dpsi/dtau = tanh(psi0 / 2) (1 - 2) with psi0 over the CURRENT gradient
    psi = T(2 * (x[..., 0] - 0.5))
    R = oc.precond_residual(psi, None, psi0)
    assert float((R + torch.tanh(psi0 / 2)).abs().max()) < 1e-12


def _linear_case(slope):
    """2D copy-boundary mesh and a phi whose linear reset is psi0 = slope (x - 1/2)."""
    mesh, prm = W.small_case(2, 3, (4, 3), periodic=False, perturb=0.1)
    prm = dataclasses.replace(prm, stop_mode=W.STOP_RMS, precond_iters=7)
    o = Oracle(2, 3, mesh, prm)
    x = o.disc.xs[..., 0]
    return o, prm, T(slope * (x - 0.5) + 0.5), slope * (x - 0.5)


def test_rms_stop_fixed_point():
    # psi0 = x - 1/2 is a distance function: R_pc = 0, so the first iterate repeats psi0,
    # the RMS is 0 and the rule stops after one iteration
    o, prm, phi, psi0 = _linear_case(1.0)
    psi, _ = o.precondition(phi)
    assert o.last_iters == 1 and o.last_rms < 1e-12
    assert float((psi - T(psi0)).abs().max()) < 1e-13


def test_rms_stop_first_iterate():
    # psi0 = 2(x - 1/2): dpsi/dtau = -tanh(psi0/2) at tau = 0 and |grad psi| moves by
    # O(dtau) over one iteration, so RMS((psi^1 - psi^0)/dtau) = RMS(tanh(psi0/2)) (1 + O(dtau))
    o, prm, phi, psi0 = _linear_case(2.0)
    o.precondition(phi, iters=1)
    want = math.sqrt(float(torch.mean(torch.tanh(T(psi0) / 2) ** 2)))
    assert o.last_iters == 1
    assert abs(o.last_rms - want) <= 20 * prm.dtau * want, (o.last_rms, want)


@pytest.mark.parametrize("sgn_mode", [W.SGN_PSI0, W.SGN_CURRENT])
def test_rms_stop_is_first_crossing(sgn_mode):
    mesh, prm = W.small_case(2, 3, (6, 6), periodic=True)
    prm = dataclasses.replace(prm, stop_mode=W.STOP_RMS, precond_iters=20, sgn_mode=sgn_mode)
    o = Oracle(2, 3, mesh, prm)
    phi = T(W.ic_phi(o.coords(), (0.5, 0.5), 0.3, 0.05))
    psi, _ = o.precondition(phi)
    k = o.last_iters
    assert 1 < k < 20 and o.last_rms <= 0.5
    # capped one short of k, the rule had not yet been met, and the iterates agree
    psi_short, _ = o.precondition(phi, iters=k - 1)
    assert o.last_iters == k - 1 and o.last_rms > 0.5
    fixed = Oracle(2, 3, mesh, dataclasses.replace(prm, stop_mode=W.STOP_FIXED))
    psi_k, _ = fixed.precondition(phi, iters=k)
    assert torch.equal(psi_k, psi)


@pytest.mark.parametrize("p", [2, 3])
def test_precond_penalty_flux_closed_form(p):
    """The common flux of the preconditioning system carries the penalty tau (psi_L - psi_R)
    (§3.2, with the interface flux of §3.1 Step 5). With psi constant in each element the
    sensor gives nu = 0 (no degree-p modes), the volume flux -nu grad psi vanishes, and with
    sgn = 0 the residual is the lifting of the penalty alone. On a periodic 2 x 2 mesh of
    squares of side h with psi = +1 in the left column and -1 in the right one, every x face
    of an element sees the jump 2 psi_e and every y face none, so at point (a, b)
    R = -(2 / h) (2 tau psi_e) (l_a(-1) / w_a + l_a(+1) / w_a),
    with the Gauss-Legendre nodes and weights and the Lagrange basis l_a computed here."""
    mesh, prm = W.small_case(2, p, (2, 2))
    prm = dataclasses.replace(prm, tau=0.37)
    o = Oracle(2, p, mesh, prm)
    x = o.coords()                                     # [E, Nu, 2]
    sign = np.where(x[:, 0, 0] < 0.5, 1.0, -1.0)       # element column
    psi = T(np.repeat(sign[:, None], x.shape[1], axis=1))
    nu = o.sensor(psi)
    assert float(torch.max(torch.abs(nu))) == 0.0
    R = o.precond_residual(psi, torch.zeros_like(psi))
    n = p + 1
    xi, w = np.polynomial.legendre.leggauss(n)

    def lag(a, s):
        return np.prod([(s - xi[c]) / (xi[a] - xi[c]) for c in range(n) if c != a])

    lift = np.array([(lag(a, -1.0) + lag(a, 1.0)) / w[a] for a in range(n)])
    h = 0.5
    # solution points of a quad: first index (x) fastest
    ia = np.tile(np.arange(n), n)
    expect = -(2.0 / h) * (2.0 * prm.tau * sign[:, None]) * lift[ia][None, :]
    assert np.abs(R.numpy() - expect).max() < 1e-12 * np.abs(expect).max()
