"""Flux Reconstruction on triangles (oracle; test infrastructure only).

§3.1 places solution points in triangles by the Williams-Shunn distribution and builds the
nodal basis from a polynomial basis spanning P_p through its Vandermonde matrix; the paper
prints no coordinates. Reading used here (parity of this part rests on it): the interior
lattice with barycentric coordinates ((i + 1/3), (j + 1/3), (k + 1/3)) / (p + 1),
i + j + k = p, which is symmetric under the triangle's symmetries and unisolvent for P_p
(an affine image of the equispaced lattice). The method's exactness and conservation
properties hold for any unisolvent set; the choice changes only the interpolation's
conditioning.

Reference element T = {(r, s): r >= 0, s >= 0, r + s <= 1}, vertices v0 = (0, 0),
v1 = (1, 0), v2 = (0, 1); edges e0 = v0 -> v1, e1 = v1 -> v2, e2 = v2 -> v0 (counter-
clockwise), each carrying p + 1 Gauss-Legendre flux points in the edge's direction.
Physical map x = x0 + J (r, s) with J = [v1 - v0, v2 - v0] (§3.1 mapping).

Operators (dense, from the definitions):
  M0[j, i]      l_i at flux point j                               (Step 1)
  D_k[i, i']    d l_i' / d xi_k at solution point i               (Steps 3, 6)
  LiftDiv       M^-1 E with M the exact mass matrix int_T l_i l_i' and
                E[i, j] = w_j l_i(x_j) (w_j the edge's Gauss-Legendre weight times half
                the reference edge length): the DG correction functions, so that the
                corrected gradient and divergence equal the DG weak forms (FR == DG)
  LiftN_k       LiftDiv * nhat_k with nhat the unit outward reference normal of the edge
  W[i]          int_T l_i (the nodal quadrature of the solution points)
  Vt, Vt_inv    orthonormal modes of P_p (Gram-Schmidt of the monomials about the centroid
                in graded order with the exact inner product on T); topmask = the modes of
                total degree p
                (the sensor's truncation to P_{p-1}, §3.2)

LDG orientation (§3.1 Step 2, beta = +-1/2): a face is owned (beta = +1/2) by the element
whose outward physical unit normal n has n . w > 0, for the fixed switch vector
w = (1, 1/sqrt(2)) (no edge of the split-Cartesian meshes is orthogonal to it). On
axis-aligned quadrilaterals the same rule with w having positive components gives the
element on the - side of every face, the reading used for the quadrilaterals.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .mesh import pair_by_coordinates

SWITCH = np.array([1.0, 1.0 / math.sqrt(2.0)])


def monomial_exponents(p):
    """(a, b) with a + b <= p, graded by total degree, then by b."""
    return [(n - b, b) for n in range(p + 1) for b in range(n + 1)]


def monomial_integral(a, b):
    """int_T r^a s^b = a! b! / (a + b + 2)! on the reference triangle."""
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


CENTRE = 1.0 / 3.0   # the monomials are taken about the centroid (better conditioned)


def centred_integral(a, b):
    """int_T (r - 1/3)^a (s - 1/3)^b, by the binomial expansion into monomial_integral."""
    c = CENTRE
    tot = 0.0
    for i in range(a + 1):
        for j in range(b + 1):
            tot += (math.comb(a, i) * math.comb(b, j) * (-c) ** (a - i) * (-c) ** (b - j)
                    * monomial_integral(i, j))
    return tot


def solution_points(p):
    """The interior lattice ((i + 1/3), (j + 1/3)) / (p + 1), j outer, i inner."""
    pts = [((i + 1.0 / 3.0) / (p + 1), (j + 1.0 / 3.0) / (p + 1))
           for j in range(p + 1) for i in range(p + 1 - j)]
    return np.array(pts)


VERTS = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
EDGES = [(0, 1), (1, 2), (2, 0)]


class TriangleOperators:
    def __init__(self, p: int):
        self.d = 2
        self.p = p
        self.shape = "triangle"
        mons = monomial_exponents(p)
        self.mons = mons
        self.nupts = Nu = len(mons)
        self.nfpts_face = n = p + 1
        self.nfpts = Nf = 3 * n
        self.upt_ref = solution_points(p)
        xi, wq = np.polynomial.legendre.leggauss(n)
        fpt, nhat, wf, face = [], [], [], []
        for e, (a, b) in enumerate(EDGES):
            va, vb = VERTS[a], VERTS[b]
            L = float(np.linalg.norm(vb - va))
            tang = (vb - va) / L
            nrm = np.array([tang[1], -tang[0]])      # outward for a counter-clockwise walk
            for t in range(n):
                fpt.append(va + 0.5 * (1.0 + xi[t]) * (vb - va))
                nhat.append(nrm)
                wf.append(0.5 * L * wq[t])
                face.append(e)
        self.fpt_ref = np.array(fpt)
        self.nhat = np.array(nhat)
        self.wf = np.array(wf)
        self.fpt_face = np.array(face)

        def mono(x, diff=None):
            """Monomials about the centroid, (r - 1/3)^a (s - 1/3)^b (or their derivative
            along diff), at points x[N, 2] -> [N, Nu]."""
            X, Y = x[:, 0] - CENTRE, x[:, 1] - CENTRE
            out = np.zeros((x.shape[0], Nu))
            for m, (a, b) in enumerate(mons):
                if diff is None:
                    out[:, m] = X ** a * Y ** b
                elif diff == 0:
                    out[:, m] = a * X ** max(a - 1, 0) * Y ** b if a > 0 else 0.0
                else:
                    out[:, m] = b * X ** a * Y ** max(b - 1, 0) if b > 0 else 0.0
            return out

        self.mono = mono
        Vm = mono(self.upt_ref)                      # Vm[i, m] = mono_m(x_i)
        if np.linalg.matrix_rank(Vm) < Nu:
            raise ValueError("solution points are not unisolvent")
        C = np.linalg.inv(Vm)                        # l_i = sum_m C[m, i] mono_m
        self.lagrange_coeffs = C
        self.M0 = mono(self.fpt_ref) @ C
        self.D = [mono(self.upt_ref, k) @ C for k in range(2)]
        G = np.array([[centred_integral(a + a2, b + b2) for (a2, b2) in mons] for (a, b) in mons])
        self.mass = C.T @ G @ C
        self.W = C.T @ np.array([centred_integral(a, b) for (a, b) in mons])
        Emat = (self.M0 * self.wf[:, None]).T        # E[i, j] = w_j l_i(x_j)
        self.LiftDiv = np.linalg.solve(self.mass, Emat)
        self.LiftN = [self.LiftDiv * self.nhat[:, k][None, :] for k in range(2)]
        # orthonormal modes: psi = L^-1 mono with G = L L^T (graded order is kept)
        Lc = np.linalg.cholesky(G)
        self.ortho_coeffs = np.linalg.inv(Lc)        # psi_j = sum_m ortho[j, m] mono_m
        self.Vt = mono(self.upt_ref) @ self.ortho_coeffs.T
        self.Vt_inv = np.linalg.inv(self.Vt)
        self.topmask = np.array([1.0 if a + b == p else 0.0 for (a, b) in mons])


class TriangleDiscretisation:
    """Geometry, flux-point pairing and LDG orientation of a triangle mesh; exposes the
    same tensors as the quadrilateral Discretisation, so the residuals of
    ``oracle.residual`` apply unchanged."""

    def __init__(self, ops: TriangleOperators, x0, jac, period, periodic):
        x0 = np.asarray(x0, dtype=np.float64)
        jac = np.asarray(jac, dtype=np.float64)
        E = x0.shape[0]
        self.ops, self.d, self.E = ops, 2, E
        self.period = np.asarray(period, dtype=np.float64)
        self.periodic = tuple(bool(p) for p in periodic)
        self.xs = x0[:, None, :] + np.einsum("eij,uj->eui", jac, ops.upt_ref)
        self.xf = x0[:, None, :] + np.einsum("eij,fj->efi", jac, ops.fpt_ref)
        self.detJ = np.linalg.det(jac)
        if np.any(self.detJ <= 0):
            raise ValueError("non-positive Jacobian determinant")
        self.Jinv = np.linalg.inv(jac)
        JinvT_n = np.einsum("eki,fk->efi", self.Jinv, ops.nhat)
        mag = np.linalg.norm(JinvT_n, axis=-1)
        self.normal = JinvT_n / mag[..., None]
        self.fscale = self.detJ[:, None] * mag
        self.has_pair, self.pair_e, self.pair_j = pair_by_coordinates(
            self.xf, self.detJ, 2, self.period, self.periodic)
        nR = self.normal[self.pair_e, self.pair_j]
        if np.any(self.has_pair & (np.abs(np.sum(self.normal * nR, -1) + 1.0) > 1e-10)):
            raise ValueError("paired slots must have opposite normals")
        sw = self.normal @ SWITCH
        if np.any(self.has_pair & (np.abs(sw) < 1e-12)):
            raise ValueError("an edge is orthogonal to the LDG switch vector")
        self.beta = np.where(self.has_pair, np.where(sw > 0, 0.5, -0.5), 0.5)
        self._torch()

    def _torch(self):
        ops = self.ops
        T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)
        self.tM0 = T(ops.M0)
        self.tD = [T(Dk) for Dk in ops.D]
        self.tLiftDiv = T(ops.LiftDiv)
        self.tLiftN = [T(Lk) for Lk in ops.LiftN]
        self.tnhat = T(ops.nhat)
        self.tW = T(ops.W)
        self.tVt_inv = T(ops.Vt_inv)
        self.ttop = T(ops.topmask)
        self.tdetJ = T(self.detJ)
        self.tJinv = T(self.Jinv)
        self.tnormal = T(self.normal)
        self.tfscale = T(self.fscale)
        self.tbeta = T(self.beta)
        self.tpair_e = torch.as_tensor(self.pair_e, dtype=torch.long)
        self.tpair_j = torch.as_tensor(self.pair_j, dtype=torch.long)
        self.txs = T(self.xs)
        self.txf = T(self.xf)

    def neighbour(self, a: torch.Tensor) -> torch.Tensor:
        return a[self.tpair_e, self.tpair_j]

    @classmethod
    def from_mesh(cls, ops, mesh):
        return cls(ops, mesh.x0, mesh.jac, mesh.period, mesh.periodic)
