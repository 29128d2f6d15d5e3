"""Residuals of the FR-PCPF system (oracle; test infrastructure only).

Physical system (§2 localized conservative phase field, Eq. altconservativephasefieldeq,
written in the flux form of §3.1): u = [phi, psi], f = f_inv - f_vis with
  f_inv = [phi v; psi v],
  f_vis = [max(gamma, |v|) (eps grad(phi) - gamma phi (1 - phi) grad(psi)/|grad(psi)|); 0].
The multiplier sits inside the flux (conservative form); gamma = 0.09 both as the floor
on |v| and as the sharpening weight; |grad psi| is regularised as
sqrt(|grad psi|^2 + delta_n^2).

FR steps (§3.1):
  Step 1  u_f = M0 u
  Step 2  common solution C = (1/2 - beta) u_f + (1/2 + beta) u_f'    (beta = +-1/2, LDG)
  Step 3  q~ = D u + LiftN (C - u_f);  q = J^-T q~;  q_f = M0 q
  Step 4  f~ = |J| J^-1 f(u, q) at solution points;  f~perp = nhat . (M0 f~)
  Step 5  F = nhat . (f_inv + f_inv')/2 - nhat . [(1/2 + beta) f_vis + (1/2 - beta) f_vis']
              + tau (u - u')   (the penalty taken with the dissipative sign);
          F~ = s F with s = |J| |J^-T nhat|
  Step 6  div = sum_k D_k f~_k + LiftDiv (F~ - f~perp);  du/dt = -div / |J|

Preconditioning system (§3.2, Eq. peudoSystem1 / pseudotimesystem): psi only, flux
g = -nu_s grad(psi), common flux nhat.[(1/2+beta) g + (1/2-beta) g'] + tau (psi - psi'),
source S = sgn (1 - |q|), dpsi/dtau = -div/|J| + S. nu_s is the element's Persson-Peraire
viscosity (Eqs. resolutionIndicator and nu_s) computed from the modal coefficients of
psi.
"""
from __future__ import annotations

import math

import torch

from . import velocity as vel


def _M0(disc, a):
    """Interpolate a per-solution-point array [E, Nu, ...] to flux points [E, Nf, ...]."""
    return torch.einsum("fu,eu...->ef...", disc.tM0, a)


def corrected_gradient(disc, u: torch.Tensor):
    """§3.1 Steps 1-3: returns (u_f [E,Nf], q [E,Nu,d] physical corrected gradient)."""
    uf = u @ disc.tM0.T
    un = disc.neighbour(uf)
    beta = disc.tbeta
    C = (0.5 - beta) * uf + (0.5 + beta) * un
    jump = C - uf
    qt = torch.stack([u @ disc.tD[k].T + jump @ disc.tLiftN[k].T for k in range(disc.d)], -1)
    # q_i = sum_k (J^-1)_{k i} q~_k   (q = J^-T q~)
    q = torch.einsum("eki,euk->eui", disc.tJinv, qt)
    return uf, q


def _transform_flux(disc, f):
    """f~_k = |J| sum_i (J^-1)_{k i} f_i (§3.1 Step 4)."""
    return disc.tdetJ[:, None, None] * torch.einsum("eki,eui->euk", disc.tJinv, f)


def _divergence(disc, ft, Ft):
    """§3.1 Step 6 with the discontinuous normal flux of Step 4; returns -div/|J|."""
    fperp = sum((ft[..., k] @ disc.tM0.T) * disc.tnhat[:, k] for k in range(disc.d))
    div = sum(ft[..., k] @ disc.tD[k].T for k in range(disc.d))
    div = div + (Ft - fperp) @ disc.tLiftDiv.T
    return -div / disc.tdetJ[:, None]


def _unit(q, delta):
    return q / torch.sqrt(torch.sum(q * q, dim=-1, keepdim=True) + delta * delta)


def physical_residual(disc, prm, phi, psi, t, amp=None):
    """du/dt of the physical system at time t: returns (R_phi, R_psi), each [E, Nu].

    The interface normal of the sharpening flux is grad(psi)/|grad psi| (§2, the
    preconditioned method); with prm.normal_mode == 1 it is grad(phi)/|grad phi|, the
    normal of Eq. conservativephasefieldeq in its original (unpreconditioned) form."""
    A = prm.vel_amp if amp is None else amp
    kind, T, u0 = prm.vel_kind, prm.vel_period, prm.vel_u0
    vs = vel.velocity(kind, disc.txs, t, A, T, u0)          # [E, Nu, d]
    vf = vel.velocity(kind, disc.txf, t, A, T, u0)          # [E, Nf, d]
    vn = disc.neighbour(vf)
    gamma, eps, tau = prm.gamma, prm.eps, prm.tau

    phif, qphi = corrected_gradient(disc, phi)
    psif, qpsi = corrected_gradient(disc, psi)
    from_phi = getattr(prm, "normal_mode", 0) == 1
    qnrm = qphi if from_phi else qpsi          # the field the interface normal comes from

    # Step 4: fluxes at solution points
    m_s = torch.clamp(torch.linalg.vector_norm(vs, dim=-1), min=gamma)
    fvis_s = m_s[..., None] * (eps * qphi - gamma * (phi * (1 - phi))[..., None]
                               * _unit(qnrm, prm.delta_n))
    ft_phi = _transform_flux(disc, phi[..., None] * vs - fvis_s)
    ft_psi = _transform_flux(disc, psi[..., None] * vs)

    # Step 5: common normal fluxes
    n = disc.tnormal
    beta = disc.tbeta
    qphif, qnrmf = _M0(disc, qphi), _M0(disc, qnrm)
    m_f = torch.clamp(torch.linalg.vector_norm(vf, dim=-1), min=gamma)
    fvis_f = m_f[..., None] * (eps * qphif - gamma * (phif * (1 - phif))[..., None]
                               * _unit(qnrmf, prm.delta_n))
    fvis_n = disc.neighbour(fvis_f)
    phin, psin = disc.neighbour(phif), disc.neighbour(psif)

    def dot(a, b):
        return torch.sum(a * b, dim=-1)

    F_phi = 0.5 * dot(n, phif[..., None] * vf + phin[..., None] * vn) \
        - dot(n, (0.5 + beta)[..., None] * fvis_f + (0.5 - beta)[..., None] * fvis_n) \
        + tau * (phif - phin)
    F_psi = 0.5 * dot(n, psif[..., None] * vf + psin[..., None] * vn) + tau * (psif - psin)

    # Step 6
    R_phi = _divergence(disc, ft_phi, disc.tfscale * F_phi)
    R_psi = _divergence(disc, ft_psi, disc.tfscale * F_psi)
    return R_phi, R_psi


def sensor(disc, prm, psi):
    """Element viscosity nu_s (§3.2, Eqs. resolutionIndicator and nu_s).

    Modal coefficients chi from u = V chi (tensor orthonormal Legendre basis, so the
    inner product is sum chi^2); the truncated solution drops the modes whose highest
    one-dimensional degree is p; s_e = log10(<u-u^, u-u^> / <u, u>); nu_s = 0 when
    either energy is zero.
    """
    chi = psi @ disc.tVt_inv.T
    e_all = torch.sum(chi * chi, dim=1)
    e_top = torch.sum(disc.ttop * chi * chi, dim=1)
    ok = (e_all > 0) & (e_top > 0)
    ratio = torch.where(ok, e_top / torch.where(ok, e_all, torch.ones_like(e_all)),
                        torch.ones_like(e_all))
    s = torch.log10(ratio)
    s0, kap, numax = prm.s0, prm.kappa, prm.nu_max
    mid = 0.5 * numax * (1.0 + torch.sin(math.pi * (s - s0) / (2.0 * kap)))
    nu = torch.where(s < s0 - kap, torch.zeros_like(s),
                     torch.where(s > s0 + kap, torch.full_like(s, numax), mid))
    return torch.where(ok, nu, torch.zeros_like(nu))


def smeared_sign(disc, prm, psi0):
    """sgn = tanh(psi0 / max(|grad psi0|, delta_g)) (§2, text after Eq. lsequation), with
    |grad psi0| the corrected gradient of psi0 computed once at the reset."""
    _, q = corrected_gradient(disc, psi0)
    g = torch.clamp(torch.linalg.vector_norm(q, dim=-1), min=prm.delta_g)
    return torch.tanh(psi0 / g)


def precond_residual(disc, prm, psi, sgn, psi0=None):
    """dpsi/dtau of the preconditioning system (§3.2). The smeared sign is ``sgn``, fixed at
    the reset; with the printed form of the sign (sgn_mode 1, §2 text after Eq.
    lsequation) it is tanh(psi0 / max(|grad psi|, delta_g)) with the gradient of the
    current psi, and ``psi0`` must be given."""
    psif, q = corrected_gradient(disc, psi)
    if getattr(prm, "sgn_mode", 0) == 1:
        g = torch.clamp(torch.linalg.vector_norm(q, dim=-1), min=prm.delta_g)
        sgn = torch.tanh(psi0 / g)
    nu = sensor(disc, prm, psi)
    g = -nu[:, None, None] * q
    gt = _transform_flux(disc, g)
    g_f = -nu[:, None, None] * _M0(disc, q)
    g_n = disc.neighbour(g_f)
    beta = disc.tbeta
    n = disc.tnormal
    G = torch.sum(n * ((0.5 + beta)[..., None] * g_f + (0.5 - beta)[..., None] * g_n), -1) \
        + prm.tau * (psif - disc.neighbour(psif))
    R = _divergence(disc, gt, disc.tfscale * G)
    S = sgn * (1.0 - torch.linalg.vector_norm(q, dim=-1))
    return R + S
