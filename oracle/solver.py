"""Time stepping, reset/preconditioning and error measures (oracle; test infrastructure only).

* Classic four-stage Runge-Kutta in physical time and in pseudo time (§3.1 last
  paragraph, §3.2 stop-rule paragraph).
* Reset psi0 = phi - 1/2 at the start and every N physical steps (§2, Eq. after the psi
  transport equation; N = 1000 in §3.2), followed by a fixed number K of pseudo-time RK4
  iterations of the preconditioning system (the printed stop rule of §3.2 is garbled; a
  fixed count inside the quoted 5-20 range is the default). The stop rule itself is the
  option stop_mode 1: stop after the first iteration k whose RMS over all solution points
  of (psi^k - psi^(k-1)) / dtau is <= 1/2 (the printed "psi_n^2" read as the iterate
  psi^n), at most K iterations. The optional LOGIT reset psi0 = eps_w ln(phi/(1-phi))
  inverts the tanh kernel of §2 (phi clamped to [delta_phi, 1-delta_phi]).
* Error measures of §4: E_L1 = int |phi - phi_e|, E_r = E_L1 / int phi_e,
  E_m = (int phi - int phi_0) / int phi_e, integrals by the Gauss-Legendre quadrature of
  the solution points (|J| W).
"""
from __future__ import annotations

import torch

from .mesh import Discretisation
from .operators import ElementOperators
from . import residual as res

LINEAR, LOGIT = 0, 1


class Oracle:
    def __init__(self, ndims, order, mesh, prm):
        if getattr(mesh, "element", "tensor") == "triangle":
            from .triangle import TriangleDiscretisation, TriangleOperators
            self.ops = TriangleOperators(order)
            self.disc = TriangleDiscretisation.from_mesh(self.ops, mesh)
        else:
            self.ops = ElementOperators(ndims, order)
            self.disc = Discretisation.from_box(self.ops, mesh)
        self.prm = prm

    # -- building blocks -------------------------------------------------------------
    def residual(self, phi, psi, t, amp=None):
        return res.physical_residual(self.disc, self.prm, phi, psi, t, amp)

    def precond_residual(self, psi, sgn, psi0=None):
        return res.precond_residual(self.disc, self.prm, psi, sgn, psi0)

    def sensor(self, psi):
        return res.sensor(self.disc, self.prm, psi)

    def reset_psi(self, phi):
        prm = self.prm
        if prm.reset_mode == LOGIT:
            c = torch.clamp(phi, prm.delta_phi, 1.0 - prm.delta_phi)
            return prm.eps_w * torch.log(c / (1.0 - c))
        return phi - 0.5

    def precondition(self, phi, iters=None):
        """Reset + pseudo-time RK4 iterations (K, or until the stop rule holds); returns
        (psi, sgn), with psi0 in place of sgn under the printed form of the sign. The
        number of iterations and the last stop-rule RMS are kept in last_iters and
        last_rms."""
        prm = self.prm
        K = prm.precond_iters if iters is None else iters
        psi0 = self.reset_psi(phi)
        current = getattr(prm, "sgn_mode", 0) == 1
        sgn = None if current else res.smeared_sign(self.disc, prm, psi0)
        rms_stop = getattr(prm, "stop_mode", 0) == 1
        psi = psi0
        dtau = prm.dtau
        self.last_iters, self.last_rms = 0, float("nan")
        for k in range(K):
            new = rk4(lambda y: self.precond_residual(y, sgn, psi0), psi, dtau)
            self.last_iters = k + 1
            if rms_stop:
                self.last_rms = float(torch.sqrt(torch.mean(((new - psi) / dtau) ** 2)))
            psi = new
            if rms_stop and self.last_rms <= 0.5:
                break
        return psi, (psi0 if current else sgn)

    def step(self, phi, psi, t, dt, amp=None):
        def f(y, tt):
            return self.residual(y[0], y[1], tt, amp)
        k1 = f((phi, psi), t)
        k2 = f((phi + 0.5 * dt * k1[0], psi + 0.5 * dt * k1[1]), t + 0.5 * dt)
        k3 = f((phi + 0.5 * dt * k2[0], psi + 0.5 * dt * k2[1]), t + 0.5 * dt)
        k4 = f((phi + dt * k3[0], psi + dt * k3[1]), t + dt)
        phi = phi + dt / 6.0 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        psi = psi + dt / 6.0 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
        return phi, psi

    def run(self, phi, psi, t, dt, nsteps, step0=0, amp=None, callback=None):
        """nsteps of RK4 with a reset + preconditioning before every step whose index is
        a multiple of the reset interval (index 0 included); psi=None forces a reset."""
        N = self.prm.reset_every
        for i in range(nsteps):
            n = step0 + i
            if psi is None or (N > 0 and n % N == 0):
                psi, _ = self.precondition(phi)
            phi, psi = self.step(phi, psi, t, dt, amp)
            t = t + dt
            if callback is not None:
                callback(n + 1, phi, psi, t)
        return phi, psi, t

    # -- error measures ------------------------------------------------------------------
    def integral(self, a):
        return torch.sum(self.disc.tdetJ[:, None] * self.disc.tW[None, :] * a)

    def mass(self, phi):
        return self.integral(phi)

    def l1(self, phi, phi_e):
        return self.integral(torch.abs(phi - phi_e))

    def rel_error(self, phi, phi_e):
        return self.l1(phi, phi_e) / self.integral(phi_e)

    def mass_error(self, phi, phi0, phi_e):
        return (self.integral(phi) - self.integral(phi0)) / self.integral(phi_e)

    def coords(self):
        return self.disc.xs


def rk4(f, y, h):
    k1 = f(y)
    k2 = f(y + 0.5 * h * k1)
    k3 = f(y + 0.5 * h * k2)
    k4 = f(y + h * k3)
    return y + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
