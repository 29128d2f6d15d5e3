"""The dense description (pcpf_dense_mesh) of a split triangle mesh, shared by the triangle
tests: the library's own triangle operators (or given ones), geometry from the element
maps, the mesh's flux-point pairing, owners by the LDG switch vector."""
import numpy as np

from oracle.triangle import SWITCH


def tri_dense(p, mesh, ops=None):
    from paper_2006_10967_amd import DenseMeshArgs, _lib, triangle_operators
    ops = ops or triangle_operators(p)
    E = mesh.nelem
    nu, nf = ops["W"].size, ops["M0"].shape[0]
    jac = mesh.jac
    jinv = np.linalg.inv(jac)
    det = np.linalg.det(jac)
    JinvT_n = np.einsum("eki,fk->efi", jinv, ops["ref_fnorm"])
    mag = np.linalg.norm(JinvT_n, axis=-1)
    fnorm = JinvT_n / mag[..., None]
    nbr_slot = mesh.slot_pairs(p + 1)
    owner = np.where(nbr_slot >= 0, (fnorm.reshape(-1, 2) @ SWITCH) > 0, True)
    arr = dict(ops, jinv=jinv, detj=det, fnorm=fnorm, fscale=det[:, None] * mag, xorig=mesh.x0,
               jac=jac, nbr_slot=nbr_slot, owner=owner)
    period = [float(mesh.period[k]) if mesh.periodic[k] else 0.0 for k in range(2)]
    return DenseMeshArgs(2, p, E, nu, nf, arr, period, shape=_lib.PCPF_SHAPE_TRIANGLE), arr
