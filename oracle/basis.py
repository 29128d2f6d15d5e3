"""1D nodal basis of the FR method (oracle; test infrastructure only).

* Solution points: Gauss-Legendre points (§3.1, solution-point paragraph).
* Nodal basis from the Vandermonde matrix of an orthonormal Legendre basis,
  l_i = sum_j (V^-1)_ij Psi_j with V_ij = Psi_i(x_j) (§3.1, nodal-basis equation).
* Correction functions: the paper only requires n.g_j = delta_ij at the flux points
  (§3.1 Step 3). The reading taken here is the DG choice: the right/left Radau
  polynomials g_R = (P_p + P_{p+1})/2 and g_L = (-1)^p (P_p - P_{p+1})/2, which make FR
  identical to nodal DG on Gauss-Legendre points.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def _legendre_coeffs(j: int) -> np.ndarray:
    c = np.zeros(j + 1)
    c[j] = 1.0
    return c


class Basis1D:
    """All 1D quantities of an order-p element; n = p + 1 solution points."""

    def __init__(self, p: int):
        if p < 1:
            raise ValueError("order must be >= 1")
        self.p = p
        self.n = n = p + 1
        self.xi, self.w = npleg.leggauss(n)
        # modes x points: V[j, a] = Psi_j(xi_a), Psi_j the orthonormal Legendre polynomial
        self.V = np.array([self.psi(j, self.xi) for j in range(n)])
        self.Vinv = np.linalg.inv(self.V)

    # orthonormal Legendre polynomial and its derivative
    def psi(self, j: int, x) -> np.ndarray:
        return np.sqrt((2 * j + 1) / 2.0) * npleg.legval(np.asarray(x, dtype=np.float64),
                                                         _legendre_coeffs(j))

    def dpsi(self, j: int, x) -> np.ndarray:
        return np.sqrt((2 * j + 1) / 2.0) * npleg.legval(np.asarray(x, dtype=np.float64),
                                                         npleg.legder(_legendre_coeffs(j)))

    def lagrange(self, x) -> np.ndarray:
        """l_a(x) for every node a: returns [len(x), n] (nodal-basis equation of §3.1)."""
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        Psi = np.array([self.psi(j, x) for j in range(self.n)])        # [n modes, len(x)]
        return (self.Vinv @ Psi).T

    def dlagrange(self, x) -> np.ndarray:
        """l_a'(x) for every node a: returns [len(x), n]."""
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        dPsi = np.array([self.dpsi(j, x) for j in range(self.n)])
        return (self.Vinv @ dPsi).T

    # correction functions (DG reading)
    def _P(self, k, x):
        return npleg.legval(np.asarray(x, dtype=np.float64), _legendre_coeffs(k))

    def _dP(self, k, x):
        return npleg.legval(np.asarray(x, dtype=np.float64), npleg.legder(_legendre_coeffs(k)))

    def g_right(self, x):
        p = self.p
        return 0.5 * (self._P(p, x) + self._P(p + 1, x))

    def g_left(self, x):
        p = self.p
        return 0.5 * (-1.0) ** p * (self._P(p, x) - self._P(p + 1, x))

    def dg_right(self, x):
        p = self.p
        return 0.5 * (self._dP(p, x) + self._dP(p + 1, x))

    def dg_left(self, x):
        p = self.p
        return 0.5 * (-1.0) ** p * (self._dP(p, x) - self._dP(p + 1, x))
