"""Pins of the oracle's preconditioning sub-solver (§2 reset and Eq. lsequation, §3.2).

P12 sensor and viscosity ramp: closed forms of Eqs. resolutionIndicator and nu_s on
    fields with a prescribed top-mode energy fraction.
P13 eikonal fixed point and the sign of the source term.
P14 the logit reset inverts the tanh kernel of §2 to the accuracy of float64.
"""
import math

import numpy as np
import pytest
import torch

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
