"""Point coordinates, slot pairing and affine geometry (oracle; test infrastructure only).

* Mapping x = x0 + J (xi + 1) with a constant Jacobian per element (§3.1, mapping and
  Jacobian equations); |J| = det J.
* Flux points of neighbouring elements share physical coordinates (§3.1, flux-point
  paragraph): slots are paired here by searching for equal coordinates (modulo the
  period in periodic directions), independently of any adjacency table.
* Transformed quantities: q = J^-T q~ (§3.1 Step 3), f~ = |J| J^-1 f (§3.1 Step 4), and
  the common normal flux is scaled to reference space by s = |J| |J^-T nhat|, with the
  physical unit normal n = J^-T nhat / |J^-T nhat| (§3.1 Step 5, last sentence).
* LDG orientation (§3.1 Step 2, beta = +-1/2): beta = +1/2 on slots of a +xi_k face (the
  element on the - side of the face "owns" it: its common solution is the neighbour's
  trace and its viscous flux is its own), beta = -1/2 on slots of a -xi_k face.
* Boundary slots without a partner use the ghost state B(u) = u, B(q) = q (§3.3).
"""
from __future__ import annotations

import numpy as np
import torch
from scipy.spatial import cKDTree

from .operators import ElementOperators


class Discretisation:
    def __init__(self, ops: ElementOperators, x0, jac, period, periodic):
        d = ops.d
        x0 = np.asarray(x0, dtype=np.float64)
        jac = np.asarray(jac, dtype=np.float64)
        E = x0.shape[0]
        if x0.shape != (E, d) or jac.shape != (E, d, d):
            raise ValueError("x0/jac shapes")
        self.ops, self.d, self.E = ops, d, E
        self.period = np.asarray(period, dtype=np.float64)
        self.periodic = tuple(bool(p) for p in periodic)

        # physical coordinates of solution and flux points
        self.xs = x0[:, None, :] + np.einsum("eij,uj->eui", jac, ops.upt_ref + 1.0)
        self.xf = x0[:, None, :] + np.einsum("eij,fj->efi", jac, ops.fpt_ref + 1.0)

        # geometry
        self.detJ = np.linalg.det(jac)
        if np.any(self.detJ <= 0):
            raise ValueError("non-positive Jacobian determinant")
        self.Jinv = np.linalg.inv(jac)
        JinvT_n = np.einsum("eki,fk->efi", self.Jinv, ops.nhat)   # (J^-T nhat)_i = Jinv[k,i] nhat_k
        mag = np.linalg.norm(JinvT_n, axis=-1)
        self.normal = JinvT_n / mag[..., None]                   # [E, Nf, d]
        self.fscale = self.detJ[:, None] * mag                   # [E, Nf]

        self._pair_slots()

        # LDG beta per slot
        s = ops.fpt_face % 2
        self.beta = np.broadcast_to(np.where(s == 1, 0.5, -0.5), (E, ops.nfpts)).copy()
        pb = self.beta[self.pair_e, self.pair_j]
        bad = self.has_pair & (pb != -self.beta)
        if np.any(bad):
            raise ValueError("paired slots must lie on a +xi face and a -xi face")

        self._torch()

    # ------------------------------------------------------------------------------
    def _pair_slots(self):
        ops = self.ops
        self.has_pair, self.pair_e, self.pair_j = pair_by_coordinates(
            self.xf, self.detJ, self.d, self.period, self.periodic)
        # paired normals must be opposite
        nL = self.normal
        nR = self.normal[self.pair_e, self.pair_j]
        dot = np.sum(nL * nR, axis=-1)
        if np.any(self.has_pair & (np.abs(dot + 1.0) > 1e-10)):
            raise ValueError("paired slots must have opposite normals")

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
        self.thas = torch.as_tensor(self.has_pair)
        self.tpair_e = torch.as_tensor(self.pair_e, dtype=torch.long)
        self.tpair_j = torch.as_tensor(self.pair_j, dtype=torch.long)
        self.txs = T(self.xs)
        self.txf = T(self.xf)

    # ------------------------------------------------------------------------------
    def neighbour(self, a: torch.Tensor) -> torch.Tensor:
        """Value of a per-slot array [E, Nf, ...] at the paired slot; the ghost value
        (own value, §3.3) on unpaired boundary slots."""
        return a[self.tpair_e, self.tpair_j]

    @classmethod
    def from_box(cls, ops: ElementOperators, mesh) -> "Discretisation":
        return cls(ops, mesh.x0, mesh.jac, mesh.period, mesh.periodic)


def pair_by_coordinates(xf, detJ, d, period, periodic):
    """Pair every flux point [E, Nf, d] with the coincident flux point of another element,
    comparing physical coordinates (modulo the period in periodic directions). Returns
    (has_pair [E, Nf], pair_e, pair_j); unpaired points are paired with themselves."""
    E, Nf = xf.shape[:2]
    pts = xf.reshape(-1, d).copy()
    box = np.zeros(d)
    for k in range(d):
        if periodic[k]:
            box[k] = period[k]
            pts[:, k] = np.mod(pts[:, k], period[k])
            # points that round to the period itself belong at 0
            pts[:, k] = np.where(pts[:, k] >= period[k], 0.0, pts[:, k])
        else:
            pts[:, k] -= pts[:, k].min()
            box[k] = 4.0 * (pts[:, k].max() + 1.0)
    hmin = float(np.min(np.abs(detJ)) ** (1.0 / d))
    tol = 1e-8 * hmin
    tree = cKDTree(pts, boxsize=box)
    dist, idx = tree.query(pts, k=3)
    me = np.arange(pts.shape[0])
    # the nearest point is the slot itself (or a coincident partner)
    partner = np.full(pts.shape[0], -1)
    for c in range(3):
        cand = (dist[:, c] < tol) & (idx[:, c] != me)
        partner = np.where(cand & (partner < 0), idx[:, c], partner)
    ncoinc = np.sum(dist < tol, axis=1)
    if np.any(ncoinc > 2):
        raise ValueError("more than two coincident flux points")
    has = partner >= 0
    if np.any(has & (partner[np.maximum(partner, 0)] != me)):
        raise ValueError("slot pairing is not symmetric")
    if all(periodic) and not np.all(has):
        raise ValueError("unpaired flux point on a fully periodic mesh")
    pe, pj = np.divmod(np.where(has, partner, me), Nf)
    return has.reshape(E, Nf), pe.reshape(E, Nf), pj.reshape(E, Nf)
