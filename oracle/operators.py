"""Dense tensor-product element operators (oracle; test infrastructure only).

Index conventions (shared with the box mesh description, not with any GPU code):
  solution point i <-> (i_0, ..., i_{d-1}), i = sum_k i_k n^k (i_0 fastest);
  face f = 2k + s, s = 0 at xi_k = -1, s = 1 at xi_k = +1;
  flux point j = f n^(d-1) + t, t = sum_m t_m n^m over the tangential dims of the face in
  ascending order (first tangential index fastest); its reference coordinate is
  xi_k = 2s - 1 and the Gauss-Legendre nodes xi_{t_m} along the tangential dims.

Each operator is the plain definition evaluated point by point:
  M0[j, i]      = l_i(x_j^f)                          §3.1 Step 1 (interpolation to flux points)
  D[k][i, i']   = d l_{i'} / d xi_k (x_i^u)           §3.1 Step 3 / Step 6 (nodal derivative)
  LiftDiv[i, j] = div g_j (x_i^u)                     §3.1 Step 6 (divergence correction)
  LiftN[k][i,j] = nhat_{j,k} div g_j (x_i^u)          §3.1 Step 3 (gradient correction,
                                                       read as the vector nhat_j times the
                                                       scalar divergence of g_j)
with the vector correction function of flux point j on face (k, s)
  g_j(x) = (2s-1) e_k c_s(x_k) prod_{m tangential} l_{t_m}(x_m),  c_1 = g_R, c_0 = g_L,
which satisfies nhat_j' . g_j(x_j') = delta_jj' (§3.1, correction-function property).
"""
from __future__ import annotations

import itertools

import numpy as np

from .basis import Basis1D


class ElementOperators:
    def __init__(self, ndims: int, p: int):
        if ndims not in (2, 3):
            raise ValueError("ndims must be 2 or 3")
        self.d = d = ndims
        self.p = p
        self.b = b = Basis1D(p)
        self.n = n = p + 1
        self.nupts = Nu = n ** d
        self.nfpts_face = nfa = n ** (d - 1)
        self.nfpts = Nf = 2 * d * nfa

        # multi-indices of solution points
        self.upt_idx = np.array([[(i // n ** k) % n for k in range(d)] for i in range(Nu)])
        self.upt_ref = b.xi[self.upt_idx]                         # [Nu, d]

        # flux points: face, tangential dims, reference coordinates, reference normals
        fpt_ref = np.zeros((Nf, d))
        fpt_face = np.zeros(Nf, dtype=int)
        fpt_tang = np.zeros((Nf, d - 1), dtype=int)
        nhat = np.zeros((Nf, d))
        for f in range(2 * d):
            k, s = divmod(f, 2)
            tdims = [m for m in range(d) if m != k]
            for t in range(nfa):
                tm = [(t // n ** q) % n for q in range(d - 1)]
                j = f * nfa + t
                fpt_face[j] = f
                fpt_tang[j] = tm
                fpt_ref[j, k] = 2 * s - 1
                for q, m in enumerate(tdims):
                    fpt_ref[j, m] = b.xi[tm[q]]
                nhat[j, k] = 2 * s - 1
        self.fpt_ref, self.fpt_face, self.fpt_tang, self.nhat = fpt_ref, fpt_face, fpt_tang, nhat

        # M0[j, i] = prod_k l_{i_k}(x_{j,k})
        L_f = [b.lagrange(fpt_ref[:, k]) for k in range(d)]       # each [Nf, n]
        M0 = np.ones((Nf, Nu))
        for k in range(d):
            M0 *= L_f[k][:, self.upt_idx[:, k]]
        self.M0 = M0

        # D[k][i, i'] = l'_{i'_k}(xi_{i_k}) prod_{m != k} l_{i'_m}(xi_{i_m})
        L_u = [b.lagrange(self.upt_ref[:, k]) for k in range(d)]  # [Nu, n]
        dL_u = [b.dlagrange(self.upt_ref[:, k]) for k in range(d)]
        self.D = []
        for k in range(d):
            Dk = np.ones((Nu, Nu))
            for m in range(d):
                T = dL_u[m] if m == k else L_u[m]
                Dk *= T[:, self.upt_idx[:, m]]
            self.D.append(Dk)

        # correction-function divergence at solution points
        LiftDiv = np.zeros((Nu, Nf))
        for j in range(Nf):
            k, s = divmod(fpt_face[j], 2)
            tdims = [m for m in range(d) if m != k]
            dc = b.dg_right if s == 1 else b.dg_left
            col = (2 * s - 1) * dc(self.upt_ref[:, k])
            for q, m in enumerate(tdims):
                col = col * b.lagrange(self.upt_ref[:, m])[:, fpt_tang[j, q]]
            LiftDiv[:, j] = col
        self.LiftDiv = LiftDiv
        self.LiftN = [LiftDiv * nhat[:, k][None, :] for k in range(d)]

        # quadrature weights at solution points
        self.W = np.prod(b.w[self.upt_idx], axis=1)

        # tensor Vandermonde (points x modes) for the sensor's modal coefficients u = V chi
        self.mode_idx = self.upt_idx.copy()                        # same ordering for modes
        Vt = np.ones((Nu, Nu))
        for k in range(d):
            Psi_k = np.array([b.psi(j, self.upt_ref[:, k]) for j in range(n)]).T   # [Nu, n]
            Vt *= Psi_k[:, self.mode_idx[:, k]]
        self.Vt = Vt
        self.Vt_inv = np.linalg.inv(Vt)
        # modes outside the order-(p-1) tensor space: max_k m_k == p
        self.topmask = (self.mode_idx.max(axis=1) == p).astype(np.float64)


def monomials(d: int, p: int):
    """Exponent tuples of every monomial of degree <= p in each variable separately."""
    return list(itertools.product(range(p + 1), repeat=d))
