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
from fractions import Fraction

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


def _exact_inverse(A):
    """Inverse of a square matrix of Fractions by Gauss-Jordan elimination (exact)."""
    n = len(A)
    M = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        pv = M[c][c]
        M[c] = [x / pv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [row[n:] for row in M]


def _matmul(A, B):
    return [[sum(A[i][k] * B[k][j] for k in range(len(B))) for j in range(len(B[0]))]
            for i in range(len(A))]


class TriangleOperators:
    """The element's operators. The solution points, the centroid and the monomial moments
    are rational, so everything except the Gauss-Legendre edge points is built in exact
    rational arithmetic (Fractions) and rounded once at the end: the nodal mass matrix of
    the lattice points is ill conditioned (it costs float64 about 1e-11 at p = 4)."""

    _cache = {}

    def __new__(cls, p: int):
        if p not in cls._cache:
            obj = super().__new__(cls)
            obj._build(p)
            cls._cache[p] = obj
        return cls._cache[p]

    def __init__(self, p: int):
        pass

    def _build(self, p: int):
        self.d = 2
        self.p = p
        self.shape = "triangle"
        mons = monomial_exponents(p)
        self.mons = mons
        self.nupts = Nu = len(mons)
        self.nfpts_face = n = p + 1
        self.nfpts = 3 * n
        pts_q = [(Fraction(3 * i + 1, 3 * (p + 1)), Fraction(3 * j + 1, 3 * (p + 1)))
                 for j in range(p + 1) for i in range(p + 1 - j)]
        self.upt_ref = np.array([[float(x), float(y)] for x, y in pts_q])
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
        c = Fraction(1, 3)

        def mono_q(x, y, diff=None):
            """Centred monomials (or a derivative) at one point, exact."""
            X, Y = x - c, y - c
            out = []
            for a, b in mons:
                if diff is None:
                    out.append(X ** a * Y ** b)
                elif diff == 0:
                    out.append(a * X ** (a - 1) * Y ** b if a > 0 else Fraction(0))
                else:
                    out.append(b * X ** a * Y ** (b - 1) if b > 0 else Fraction(0))
            return out

        def mono(x, diff=None):
            """Centred monomials (r - 1/3)^a (s - 1/3)^b (or their derivative along diff) at
            float points x[N, 2] -> [N, Nu] (float64)."""
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
        Vm = [mono_q(x, y) for x, y in pts_q]                      # Vm[i][m]
        C = _exact_inverse(Vm)                                     # l_i = sum_m C[m][i] mono_m
        self.lagrange_coeffs = np.array([[float(v) for v in row] for row in C])
        fq = [(Fraction(float(x)), Fraction(float(y))) for x, y in self.fpt_ref]
        M0 = _matmul([mono_q(x, y) for x, y in fq], C)
        self.M0 = np.array([[float(v) for v in row] for row in M0])
        self.D = [np.array([[float(v) for v in row]
                            for row in _matmul([mono_q(x, y, k) for x, y in pts_q], C)])
                  for k in range(2)]
        # exact moments of the centred monomials, the nodal mass matrix and weights
        def cmom(a, b):
            tot = Fraction(0)
            for i in range(a + 1):
                for j in range(b + 1):
                    tot += (math.comb(a, i) * math.comb(b, j) * (-c) ** (a - i) * (-c) ** (b - j)
                            * Fraction(math.factorial(i) * math.factorial(j),
                                       math.factorial(i + j + 2)))
            return tot
        G = [[cmom(a + a2, b + b2) for (a2, b2) in mons] for (a, b) in mons]
        CT = [[C[m][i] for m in range(Nu)] for i in range(Nu)]
        Mass = _matmul(_matmul(CT, G), C)
        self.mass = np.array([[float(v) for v in row] for row in Mass])
        self.W = np.array([float(sum(CT[i][m] * cmom(*mons[m]) for m in range(Nu)))
                           for i in range(Nu)])
        # LiftDiv = M^-1 E with E[i][j] = w_j l_i(x_j) (exact given the float edge data)
        Minv = _exact_inverse(Mass)
        E = [[Fraction(float(self.wf[j])) * M0[j][i] for j in range(self.nfpts)] for i in range(Nu)]
        self.LiftDiv = np.array([[float(v) for v in row] for row in _matmul(Minv, E)])
        self.LiftN = [self.LiftDiv * self.nhat[:, k][None, :] for k in range(2)]
        # orthonormal modes: Gram-Schmidt of the centred monomials in graded order with the
        # exact inner product (orthogonal, exact), then each mode divided by its norm
        ortho = []      # coefficient rows over the monomials
        for m in range(Nu):
            v = [Fraction(int(k == m)) for k in range(Nu)]
            for u in ortho:
                num = sum(u[a] * G[a][b] * v[b] for a in range(Nu) for b in range(Nu))
                den = sum(u[a] * G[a][b] * u[b] for a in range(Nu) for b in range(Nu))
                f = num / den
                v = [vi - f * ui for vi, ui in zip(v, u)]
            ortho.append(v)
        norms = [math.sqrt(float(sum(u[a] * G[a][b] * u[b] for a in range(Nu) for b in range(Nu))))
                 for u in ortho]
        Vq = _matmul(Vm, [[ortho[j][m] for j in range(Nu)] for m in range(Nu)])   # phi~_j(x_i)
        self.Vt = np.array([[float(Vq[i][j]) / norms[j] for j in range(Nu)] for i in range(Nu)])
        self.ortho_coeffs = np.array([[float(v) / norms[j] for v in ortho[j]] for j in range(Nu)])
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
