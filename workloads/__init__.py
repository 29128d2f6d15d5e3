"""Seeded synthetic inputs shaped like the paper's benchmark problems (§4).

This module is shared by the GPU path's callers (tests, bench, smoke) and by the CPU
oracle. It holds problem definitions only and none of the FR-PCPF method's arithmetic:

* box meshes: grid planes (uniform, or interior planes shifted by a seeded uniform
  perturbation), the element corner and the constant Jacobian of each affine element,
  and the element adjacency of the box (including periodic wrap);
* the initial condition of §4 (tanh profile of a signed distance, Eq. initialCond with the
  disc/sphere distance of Eq. discEq, or the distance to a slotted disc of §4.1),
  evaluated at coordinates the caller supplies;
* velocity-field identifiers and the parameter values the paper fixes (§2, §3.2, §4);
* the benchmark configurations (2D vortex, slotted-disc rotation and 3D deformation).

Coordinates of solution points are NOT computed here: each side maps its own reference
nodes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Sequence

import numpy as np

# velocity kinds (same numbering as the C-ABI enum)
VEL_UNIFORM = 0
VEL_ROTATION = 1
VEL_SINGLE_VORTEX = 2
VEL_LEVEQUE3D = 3

RESET_LINEAR = 0
RESET_LOGIT = 1
NORMAL_PSI = 0   # interface normal from the preconditioned level set psi (§2, the method)
NORMAL_PHI = 1   # normal from phi itself: the unpreconditioned conservative phase field
SGN_PSI0 = 0     # smeared sign with |grad psi0| of the reset (default reading)
SGN_CURRENT = 1  # smeared sign with the current |grad psi| (the printed form)
STOP_FIXED = 0   # a fixed number of pseudo-time iterations (default reading)
STOP_RMS = 1     # the printed RMS stop rule (threshold 1/2, capped)


# --------------------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------------------
@dataclass
class BoxMesh:
    """Axis-aligned (optionally x-sheared in 2D) box mesh of affine quads/hexes.

    Element index e = ex + nx*(ey + ny*ez). Face f = 2k + s: s = 0 is the face at
    reference coordinate xi_k = -1, s = 1 the face at xi_k = +1. nbr[e, f] is the element
    across face f (-1 on a non-periodic boundary); the face across from face 2k+1 of e is
    face 2k of nbr[e, 2k+1].
    """
    ndims: int
    shape: tuple
    planes: list              # per dim: array of n_k + 1 plane coordinates
    periodic: tuple
    x0: np.ndarray            # [E, d] physical image of the reference corner (-1, ..., -1)
    jac: np.ndarray           # [E, d, d] J[i, j] = dx_i / dxi_j (constant per element)
    nbr: np.ndarray           # [E, 2d] int32
    period: np.ndarray        # [d] domain length per dim (used for periodic wrap)
    shear: object = 0.0        # 2D: s_xy; 3D: (s_xy, s_xz, s_yz)

    @property
    def nelem(self) -> int:
        return int(np.prod(self.shape))


def uniform_planes(n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return lo + (hi - lo) * np.arange(n + 1, dtype=np.float64) / n


def perturbed_planes(n: int, amp_frac: float, rng: np.random.Generator,
                     lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Interior planes shifted by U(-amp_frac*h, amp_frac*h); the two end planes fixed."""
    p = uniform_planes(n, lo, hi)
    h = (hi - lo) / n
    p[1:-1] += rng.uniform(-amp_frac * h, amp_frac * h, size=n - 1)
    return p


def box_mesh(planes: Sequence[np.ndarray], periodic: Sequence[bool], shear=0.0) -> BoxMesh:
    """Build the element maps and adjacency of a box mesh from its grid planes.

    ``shear`` in 2D (a number s) maps (x, y) -> (x + s*y, y); with periodic y the wrap then
    connects column ex to column ex + s*nx, so s*nx must be an integer and the x planes
    uniform. In 3D it is a triple (s_xy, s_xz, s_yz) (see ``_skew_mesh_3d``).
    """
    d = len(planes)
    if d == 3 and np.any(np.asarray(shear, dtype=np.float64) != 0.0):
        return _skew_mesh_3d(planes, periodic, tuple(float(x) for x in shear))
    shape = tuple(len(p) - 1 for p in planes)
    E = int(np.prod(shape))
    idx = np.arange(E)
    coords = []
    rem = idx.copy()
    for k in range(d):
        coords.append(rem % shape[k])
        rem = rem // shape[k]
    x0 = np.zeros((E, d))
    jac = np.zeros((E, d, d))
    for k in range(d):
        lo = planes[k][coords[k]]
        hi = planes[k][coords[k] + 1]
        x0[:, k] = lo
        jac[:, k, k] = 0.5 * (hi - lo)
    period = np.array([planes[k][-1] - planes[k][0] for k in range(d)])
    shift = 0
    if np.any(np.asarray(shear) != 0.0):
        shear = float(shear)
        x0[:, 0] += shear * x0[:, 1]
        jac[:, 0, 1] = shear * jac[:, 1, 1]
        nx = shape[0]
        s = shear * nx * (period[1] / period[0])
        if periodic[1] and abs(s - round(s)) > 1e-12:
            raise ValueError("shear*nx must be an integer for a periodic y direction")
        shift = int(round(s))
    strides = [int(np.prod(shape[:k])) for k in range(d)]
    nbr = np.full((E, 2 * d), -1, dtype=np.int32)
    for k in range(d):
        for s, step in ((0, -1), (1, 1)):
            c = coords[k] + step
            ok = (c >= 0) & (c < shape[k])
            if periodic[k]:
                c = c % shape[k]
                ok = np.ones(E, dtype=bool)
            e2 = idx + (c - coords[k]) * strides[k]
            if shear != 0.0 and k == 1 and periodic[1]:
                # crossing the y wrap moves the column by the shear shift
                ex = coords[0].copy()
                wrap_up = (coords[1] + step) >= shape[1]
                wrap_dn = (coords[1] + step) < 0
                ex = np.where(wrap_up, (ex + shift) % shape[0], ex)
                ex = np.where(wrap_dn, (ex - shift) % shape[0], ex)
                e2 = ex + shape[0] * c
            nbr[:, 2 * k + s] = np.where(ok, e2, -1).astype(np.int32)
    return BoxMesh(ndims=d, shape=shape, planes=[np.asarray(p) for p in planes],
                   periodic=tuple(bool(x) for x in periodic), x0=x0, jac=jac, nbr=nbr,
                   period=period, shear=shear)


def _skew_mesh_3d(planes, periodic, shear) -> BoxMesh:
    """A box grid mapped by the unit upper-triangular matrix
    S = [[1, s_xy, s_xz], [0, 1, s_yz], [0, 0, 1]]: x = S b for every point b of the box
    grid, so every element is affine with J = S diag(h_k / 2), a full (non-diagonal)
    Jacobian whose faces have non-axis normals.

    With periodic directions the mesh stays periodic under the axis-aligned periods of
    the box (L_x, L_y, L_z): crossing the y wrap moves the x index by s_xy L_y / h_x cells,
    crossing the z wrap moves it by (s_xz - s_xy s_yz) L_z / h_x cells and the y index by
    s_yz L_z / h_y cells. These must be whole numbers and the x and y planes uniform
    (the z planes may be perturbed). Tangential axes of neighbouring faces point the same
    way (every element has the same S)."""
    sxy, sxz, syz = shear
    S = np.array([[1.0, sxy, sxz], [0.0, 1.0, syz], [0.0, 0.0, 1.0]])
    shape = tuple(len(p) - 1 for p in planes)
    nx, ny, nz = shape
    E = nx * ny * nz
    idx = np.arange(E)
    ix, iy, iz = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    L = np.array([planes[k][-1] - planes[k][0] for k in range(3)])
    h = L / np.array(shape)

    def whole(v, what):
        if abs(v - round(v)) > 1e-9:
            raise ValueError(f"skew: {what} must be a whole number of cells (got {v})")
        return int(round(v))

    for k in (0, 1):
        if not np.allclose(np.diff(planes[k]), h[k], rtol=0, atol=1e-12 * L[k]):
            raise ValueError("skew: the x and y planes must be uniform")
    kx_y = whole(sxy * L[1] / h[0], "s_xy L_y / h_x") if periodic[1] else 0
    kx_z = whole((sxz - sxy * syz) * L[2] / h[0], "(s_xz - s_xy s_yz) L_z / h_x") if periodic[2] else 0
    ky_z = whole(syz * L[2] / h[1], "s_yz L_z / h_y") if periodic[2] else 0
    lo = np.stack([planes[0][ix], planes[1][iy], planes[2][iz]], -1)
    hi = np.stack([planes[0][ix + 1], planes[1][iy + 1], planes[2][iz + 1]], -1)
    x0 = lo @ S.T
    jac = np.einsum("ij,ej->eij", S, 0.5 * (hi - lo))
    nbr = np.full((E, 6), -1, dtype=np.int32)
    for k in range(3):
        for sd, step in ((0, -1), (1, 1)):
            c = [ix.copy(), iy.copy(), iz.copy()]
            c[k] = c[k] + step
            ok = np.ones(E, dtype=bool)
            # leave the box through z: wrap z and shift x, y; then y (shifts x); then x
            up, dn = c[2] >= nz, c[2] < 0
            if periodic[2]:
                c[0] = c[0] + np.where(up, kx_z, 0) - np.where(dn, kx_z, 0)
                c[1] = c[1] + np.where(up, ky_z, 0) - np.where(dn, ky_z, 0)
                c[2] = c[2] % nz
            else:
                ok &= ~(up | dn)
            while True:
                up, dn = c[1] >= ny, c[1] < 0
                if not (up.any() or dn.any()):
                    break
                if periodic[1]:
                    c[0] = c[0] + np.where(up, kx_y, 0) - np.where(dn, kx_y, 0)
                    c[1] = np.where(up, c[1] - ny, np.where(dn, c[1] + ny, c[1]))
                else:
                    ok &= ~(up | dn)
                    c[1] = np.clip(c[1], 0, ny - 1)
            if periodic[0]:
                c[0] = c[0] % nx
            else:
                ok &= (c[0] >= 0) & (c[0] < nx)
                c[0] = np.clip(c[0], 0, nx - 1)
            e2 = c[0] + nx * (c[1] + ny * c[2])
            nbr[:, 2 * k + sd] = np.where(ok, e2, -1).astype(np.int32)
    return BoxMesh(ndims=3, shape=shape, planes=[np.asarray(p) for p in planes],
                   periodic=tuple(bool(x) for x in periodic), x0=x0, jac=jac, nbr=nbr,
                   period=L, shear=shear)


@dataclass
class TriMesh:
    """Triangle mesh from diagonally split grid cells (§4.2, the uniform split triangular
    mesh). Triangle corners v0, v1, v2 counter-clockwise; affine map x = x0 + J (r, s) with
    J = [v1 - v0, v2 - v0] from the reference triangle {r, s >= 0, r + s <= 1}. Edge
    f = 0, 1, 2 runs v0 -> v1, v1 -> v2, v2 -> v0. nbr[e, f] = (element, edge) across edge f,
    or (-1, -1) on a boundary; the two elements traverse a shared edge in opposite
    directions."""
    ndims: int
    shape: tuple
    periodic: tuple
    x0: np.ndarray            # [E, 2]
    jac: np.ndarray           # [E, 2, 2]
    nbr: np.ndarray           # [E, 3, 2] int32: neighbour element and its edge
    period: np.ndarray
    planes: tuple = None      # the grid lines of the split cells (x, y)
    element: str = "triangle"

    @property
    def nelem(self) -> int:
        return self.x0.shape[0]

    def slot_pairs(self, npe: int) -> np.ndarray:
        """Partner flux point e' 3 npe + f' npe + t' of every flux point e 3 npe + f npe + t
        (npe points per edge, ordered along the edge), -1 on boundaries: the shared edge is
        walked the other way by the neighbour, so t' = npe - 1 - t."""
        E = self.nelem
        out = np.full((E, 3, npe), -1, dtype=np.int64)
        t = np.arange(npe)
        for f in range(3):
            en, fn = self.nbr[:, f, 0], self.nbr[:, f, 1]
            ok = en >= 0
            part = (en[:, None] * 3 + fn[:, None]) * npe + (npe - 1 - t)[None, :]
            out[:, f, :] = np.where(ok[:, None], part, -1)
        return out.reshape(-1)


def split_tri_mesh(n: int, periodic=True, lo: float = 0.0, hi: float = 1.0,
                   perturb: float = 0.0, seed: int = 1, planes=None) -> TriMesh:
    """n x n grid cells of [lo, hi]^2, each split along its lower-left to upper-right
    diagonal into the triangles A = (c00, c10, c11) and B = (c00, c11, c01). Cell (i, j),
    triangle A = element 2 (i + n j), B = element 2 (i + n j) + 1. ``perturb`` shifts the
    interior grid lines by U(-perturb h, perturb h) (seeded), keeping every triangle affine.
    ``planes`` (two arrays of n + 1 grid lines) replaces the generated ones."""
    if planes is None:
        rng = np.random.default_rng(seed)
        planes = [perturbed_planes(n, perturb, rng, lo, hi) if perturb > 0
                  else uniform_planes(n, lo, hi) for _ in range(2)]
    else:
        planes = [np.asarray(q, dtype=np.float64) for q in planes]
        assert all(q.shape == (n + 1,) for q in planes)
        lo, hi = float(planes[0][0]), float(planes[0][-1])
    per = periodic if isinstance(periodic, (list, tuple)) else (periodic, periodic)
    E = 2 * n * n
    px, py = (np.asarray(q, dtype=np.float64) for q in planes)
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")   # cell (i, j), i fastest
    ii, jj = ii.reshape(-1), jj.reshape(-1)
    c00 = np.stack([px[ii], py[jj]], 1)
    c10 = np.stack([px[ii + 1], py[jj]], 1)
    c11 = np.stack([px[ii + 1], py[jj + 1]], 1)
    c01 = np.stack([px[ii], py[jj + 1]], 1)
    A, B = 2 * (ii + n * jj), 2 * (ii + n * jj) + 1
    x0 = np.zeros((E, 2))
    jac = np.zeros((E, 2, 2))
    x0[A], jac[A] = c00, np.stack([c10 - c00, c11 - c00], 2)
    x0[B], jac[B] = c00, np.stack([c11 - c00, c01 - c00], 2)
    nbr = np.full((E, 3, 2), -1, dtype=np.int32)

    def cell(i, j):
        # neighbouring cell index (wrapped in periodic directions), -1 outside the mesh
        if per[0]:
            i = i % n
        if per[1]:
            j = j % n
        ok = (i >= 0) & (i < n) & (j >= 0) & (j < n)
        return np.where(ok, i + n * j, -1)

    # A: edge 0 (c00 -> c10) bottom, edge 1 (c10 -> c11) right, edge 2 (c11 -> c00) diagonal;
    # B: edge 0 (c00 -> c11) diagonal, edge 1 (c11 -> c01) top, edge 2 (c01 -> c00) left
    def link(el, edge, other_cell, other_off, other_edge):
        ok = other_cell >= 0
        nbr[el[ok], edge, 0] = 2 * other_cell[ok] + other_off
        nbr[el[ok], edge, 1] = other_edge

    link(A, 2, (A // 2), 1, 0)
    link(B, 0, (B // 2), 0, 2)
    link(A, 0, cell(ii, jj - 1), 1, 1)
    link(A, 1, cell(ii + 1, jj), 1, 2)
    link(B, 1, cell(ii, jj + 1), 0, 0)
    link(B, 2, cell(ii - 1, jj), 0, 1)
    period = np.array([float(q[-1] - q[0]) for q in planes])
    return TriMesh(ndims=2, shape=(n, n), periodic=tuple(bool(x) for x in per), x0=x0,
                   jac=jac, nbr=nbr, period=period, planes=tuple(planes))


# --------------------------------------------------------------------------------------
# initial condition (§4, Eq. initialCond with the distance of Eq. discEq)
# --------------------------------------------------------------------------------------
def signed_distance_ball(x: np.ndarray, centre: Sequence[float], radius: float) -> np.ndarray:
    """psi_d = r - |x - x_c| (positive inside); x has shape [..., d]."""
    c = np.asarray(centre, dtype=np.float64)
    return radius - np.sqrt(np.sum((x - c) ** 2, axis=-1))


def _segment_distance(x: np.ndarray, a, b) -> np.ndarray:
    """Distance from points x[..., 2] to the segment [a, b]."""
    a = np.asarray(a, dtype=np.float64)
    ab = np.asarray(b, dtype=np.float64) - a
    s = np.clip(np.sum((x - a) * ab, axis=-1) / float(ab @ ab), 0.0, 1.0)
    return np.sqrt(np.sum((x - (a + s[..., None] * ab)) ** 2, axis=-1))


def signed_distance_slotted_disc(x: np.ndarray, centre: Sequence[float], radius: float,
                                 half_width: float, slot_top: float) -> np.ndarray:
    """Signed distance (positive inside) to the slotted disc of §4.1: the disc of Eq. discEq
    less the slot {|x - x_c| <= half_width, y <= slot_top}, which opens at the bottom of the
    disc.

    The boundary is the circle arc outside the slot and the three slot walls (the two
    vertical sides from the circle up to ``slot_top`` and the top). The distance to the arc
    is the radial distance where the radial projection lands on the arc and the distance to
    the nearer arc end otherwise; the distance to the boundary is the least over the four
    pieces, with the sign of membership."""
    c = np.asarray(centre, dtype=np.float64)
    w, top = float(half_width), float(slot_top)
    if not (0.0 < w < radius and c[1] - radius < top < c[1] + radius):
        raise ValueError("the slot must cut the bottom of the disc and end inside it")
    ybot = c[1] - math.sqrt(radius ** 2 - w ** 2)        # the walls meet the circle here
    left, right = (c[0] - w, ybot), (c[0] + w, ybot)
    rel = x - c
    rho = np.sqrt(np.sum(rel ** 2, axis=-1))
    safe = np.where(rho > 0.0, rho, 1.0)
    proj = c + radius * rel / safe[..., None]             # nearest point of the full circle
    on_arc = ~((np.abs(proj[..., 0] - c[0]) < w) & (proj[..., 1] < top)) & (rho > 0.0)
    d_arc = np.where(on_arc, np.abs(rho - radius),
                     np.minimum(np.sqrt(np.sum((x - np.asarray(left)) ** 2, axis=-1)),
                                np.sqrt(np.sum((x - np.asarray(right)) ** 2, axis=-1))))
    d = np.minimum.reduce([d_arc,
                           _segment_distance(x, left, (c[0] - w, top)),
                           _segment_distance(x, right, (c[0] + w, top)),
                           _segment_distance(x, (c[0] - w, top), (c[0] + w, top))])
    inside = (rho <= radius) & ~((np.abs(x[..., 0] - c[0]) <= w) & (x[..., 1] <= top))
    return np.where(inside, d, -d)


def tanh_profile(psi_d: np.ndarray, eps_w: float) -> np.ndarray:
    """phi = (1 + tanh(psi_d / (2 eps_w))) / 2, i.e. Eq. initialCond with beta = 1/(2 eps_w)."""
    return 0.5 * (1.0 + np.tanh(psi_d / (2.0 * eps_w)))


def ic_phi(x: np.ndarray, centre, radius, eps_w) -> np.ndarray:
    return tanh_profile(signed_distance_ball(x, centre, radius), eps_w)


def random_state(shape, rng: np.random.Generator, lo=0.0, hi=1.0) -> np.ndarray:
    return rng.uniform(lo, hi, size=shape)


# --------------------------------------------------------------------------------------
# parameters and configurations
# --------------------------------------------------------------------------------------
@dataclass
class Params:
    """Method parameters. Values from §2 (gamma, eps), §3.2 (s0, kappa, nu_max, reset
    interval N) and §4 (IC sharpness); the rest are readings of silent points."""
    gamma: float
    eps: float
    eps_w: float
    tau: float = 0.1
    nu_max: float = 0.0
    s0: float = -5.0
    kappa: float = 5.0
    dtau: float = 0.0
    delta_n: float = 1e-12
    delta_g: float = 1e-12
    delta_phi: float = 1e-12
    reset_every: int = 1000
    precond_iters: int = 10
    reset_mode: int = RESET_LINEAR
    vel_kind: int = VEL_UNIFORM
    vel_amp: float = 1.0
    vel_period: float = 1.0
    vel_u0: tuple = (0.0, 0.0, 0.0)
    normal_mode: int = NORMAL_PSI
    sgn_mode: int = SGN_PSI0
    stop_mode: int = STOP_FIXED


def default_params(ndims: int, order: int, h: float, *, eps_w: Optional[float] = None,
                   dtau_coeff: Optional[float] = None, **over) -> Params:
    """gamma = 0.09, eps = 0.06 h/p (§2); nu_max = 0.15 h/p, s0 = -5 (§3.2);
    eps_w = 2h/(3p), the width of the IC with beta = 3p/(4h) (§4)."""
    if dtau_coeff is None:
        dtau_coeff = {(2, 1): 0.05, (2, 2): 0.04, (2, 3): 0.025, (2, 4): 0.015, (2, 5): 0.01,
                      (3, 1): 0.04, (3, 2): 0.025, (3, 3): 0.015, (3, 4): 0.010,
                      (3, 5): 0.007}.get((ndims, order), 0.01)
    p = Params(gamma=0.09, eps=0.06 * h / order,
               eps_w=(2.0 * h / (3.0 * order)) if eps_w is None else eps_w,
               nu_max=0.15 * h / order, dtau=dtau_coeff * h)
    return replace(p, **over)


VMAX = {VEL_UNIFORM: None, VEL_ROTATION: None, VEL_SINGLE_VORTEX: 1.0, VEL_LEVEQUE3D: 2.0}


@dataclass
class Config:
    name: str
    ndims: int
    order: int
    n: int                       # elements per direction
    periodic: bool = True
    perturb: float = 0.0         # interior-plane perturbation as a fraction of h
    perturb_seed: int = 1
    centre: tuple = (0.5, 0.5)
    radius: float = 0.15
    cfl: float = 0.1
    steps: int = 200
    params: Params = None
    vmax: float = 1.0
    description: str = ""
    length: float = 1.0          # the domain is [0, length]^d
    slot: Optional[tuple] = None  # (half width, top) of a slotted disc (§4.1)
    element: str = "tensor"      # "tensor" (quads / hexes) or "triangle" (split n x n cells)

    @property
    def h(self) -> float:
        return self.length / self.n

    @property
    def nelem(self) -> int:
        return 2 * self.n * self.n if self.element == "triangle" else self.n ** self.ndims

    @property
    def nupts(self) -> int:
        if self.element == "triangle":
            return (self.order + 1) * (self.order + 2) // 2
        return (self.order + 1) ** self.ndims

    @property
    def nfpts(self) -> int:
        if self.element == "triangle":
            return 3 * (self.order + 1)
        return 2 * self.ndims * (self.order + 1) ** (self.ndims - 1)

    @property
    def dof(self) -> int:
        return self.nelem * self.nupts

    def mesh(self):
        if self.element == "triangle":
            return split_tri_mesh(self.n, self.periodic, hi=self.length, perturb=self.perturb,
                                  seed=self.perturb_seed)
        rng = np.random.default_rng(self.perturb_seed)
        planes = []
        for _ in range(self.ndims):
            if self.perturb > 0:
                planes.append(perturbed_planes(self.n, self.perturb, rng, hi=self.length))
            else:
                planes.append(uniform_planes(self.n, hi=self.length))
        return box_mesh(planes, [self.periodic] * self.ndims)

    def distance(self, x: np.ndarray) -> np.ndarray:
        """Signed distance of the initial shape (disc/sphere, or slotted disc)."""
        if self.slot is None:
            return signed_distance_ball(x, self.centre, self.radius)
        return signed_distance_slotted_disc(x, self.centre, self.radius, *self.slot)

    def initial_phi(self, x: np.ndarray) -> np.ndarray:
        """Eq. initialCond at the points x[..., d] with beta = 1/(2 eps_w)."""
        return tanh_profile(self.distance(x), self.params.eps_w)

    def hmin(self, mesh=None) -> float:
        """Shortest grid spacing (quads / hexes), or shortest triangle leg."""
        mesh = mesh or self.mesh()
        if self.element == "triangle":
            return float(np.min(np.linalg.norm(mesh.jac, axis=1)))
        return float(min(np.min(np.diff(p)) for p in mesh.planes))

    def dt(self, mesh: Optional[BoxMesh] = None) -> float:
        """dt = CFL * h_min / |v|_max (|v|_max the analytic peak of the field)."""
        return self.cfl * self.hmin(mesh) / self.vmax


def _cfg_c1() -> Config:
    h = 1.0 / 16
    prm = default_params(2, 3, h, eps_w=h / 4, dtau_coeff=0.025, vel_kind=VEL_UNIFORM,
                         vel_u0=(1.0, 0.5, 0.0))
    return Config("advect2d_16x16_p3", 2, 3, 16, centre=(0.5, 0.5), cfl=0.1, steps=200,
                  params=prm, vmax=math.hypot(1.0, 0.5),
                  description="2D periodic unit square, 16x16 quads, p=3, uniform velocity "
                              "(1,0.5), tanh circle r=0.15 at (0.5,0.5), eps_w=h/(p+1), RK4 "
                              "CFL 0.1, 200 steps")


def _cfg_c2() -> Config:
    h = 1.0 / 128
    prm = default_params(2, 4, h, dtau_coeff=0.015, vel_kind=VEL_SINGLE_VORTEX,
                         vel_period=8.0)
    return Config("vortex2d_128x128_p4", 2, 4, 128, centre=(0.5, 0.75), cfl=0.05,
                  steps=20480, params=prm, vmax=1.0,
                  description="2D 128x128 quads, p=4, time-reversing single vortex T=8, "
                              "circle r=0.15 at (0.5,0.75)")


def _cfg_c3() -> Config:
    h = 1.0 / 64
    prm = default_params(3, 3, h, dtau_coeff=0.015, vel_kind=VEL_LEVEQUE3D, vel_period=3.0)
    return Config("deform3d_64cube_p3", 3, 3, 64, centre=(0.35, 0.35, 0.35), cfl=0.05,
                  steps=100, params=prm, vmax=2.0,
                  description="3D periodic unit cube, 64^3 hexes, p=3, LeVeque deformation "
                              "T=3, sphere r=0.15 at (0.35,0.35,0.35), 100 RK4 steps")


def _cfg_c4() -> Config:
    h = 1.0 / 64
    prm = default_params(2, 3, h, dtau_coeff=0.025, vel_kind=VEL_SINGLE_VORTEX,
                         vel_period=4.0)
    return Config("adjoint2d_64x64_p3", 2, 3, 64, centre=(0.5, 0.75), cfl=0.1, steps=512,
                  params=prm, vmax=1.0,
                  description="2D 64x64 quads, p=3, single vortex T=4, 512 RK4 steps, "
                              "checkpoint every 32")


def _cfg_c5() -> Config:
    h = 1.0 / 96
    prm = default_params(3, 4, h, dtau_coeff=0.010, vel_kind=VEL_LEVEQUE3D, vel_period=3.0)
    return Config("deform3d_96cube_p4_perturbed", 3, 4, 96, perturb=0.2, perturb_seed=1,
                  centre=(0.35, 0.35, 0.35), cfl=0.03, steps=100, params=prm, vmax=2.0,
                  description="3D 96^3 hexes, interior planes perturbed +-20% h, p=4, "
                              "LeVeque deformation, 100 RK4 steps")


def _vortex_tri(n: int, order: int) -> Config:
    h = 1.0 / n
    prm = default_params(2, order, h, dtau_coeff=0.008, vel_kind=VEL_SINGLE_VORTEX,
                         vel_period=8.0)
    return Config(f"vortex2d_tri{n}_p{order}", 2, order, n, centre=(0.5, 0.75), cfl=0.02,
                  steps=100, params=prm, vmax=1.0, element="triangle",
                  description=f"2D periodic unit square, {n}x{n} cells split into "
                              f"{2 * n * n} triangles, p={order}, time-reversing single vortex "
                              "T=8, circle r=0.15 at (0.5,0.75)")


def _cfg_t1() -> Config:
    """The single vortex on the split triangle mesh of 128 x 128 cells, p = 4 (the largest
    of the triangle meshes of §4.2, at an order of its table)."""
    return _vortex_tri(128, 4)


def _cfg_t2() -> Config:
    """The same flow on 1024 x 1024 cells (2.1 M triangles, 31 M DOF): a single-GPU-sized
    triangle mesh whose state does not fit in the caches."""
    return _vortex_tri(1024, 4)


ROTATION_CFL = {2: 0.05, 3: 0.05, 4: 0.05, 5: 0.03}


def zalesak(n: int, order: int) -> Config:
    """Zalesak's slotted disc (§4.1): r = 0.15 at (0.5, 0.75), slot |x - 0.5| <= 0.025,
    y <= 0.85, rigid rotation (0.5 - y, x - 0.5) for one turn (t = 2 pi) on n x n quads;
    dt is the CFL step rounded down so that a whole number of steps makes the turn."""
    h = 1.0 / n
    prm = default_params(2, order, h, vel_kind=VEL_ROTATION, vel_u0=(0.5, 0.5, 0.0))
    cfl = ROTATION_CFL.get(order, 0.03)
    vmax = math.sqrt(0.5)                               # at the corners of the square
    steps = int(math.ceil(2.0 * math.pi / (cfl * h / vmax)))
    return Config(f"zalesak2d_{n}x{n}_p{order}", 2, order, n, centre=(0.5, 0.75),
                  radius=0.15, cfl=cfl, steps=steps, params=prm, vmax=vmax,
                  slot=(0.025, 0.85),
                  description=f"Zalesak slotted disc, {n}x{n} quads, p={order}, one rotation")


def rudman(order: int, n: int = 200) -> Config:
    """Rudman's slotted disc (§4.1): [0, 4]^2, r = 0.5 at (2, 2.75), slot |x - 2| <= 0.06,
    y <= 2.65, rigid rotation (2 - y, x - 2) for one turn on n x n quads."""
    L = 4.0
    h = L / n
    prm = default_params(2, order, h, vel_kind=VEL_ROTATION, vel_u0=(2.0, 2.0, 0.0))
    cfl = ROTATION_CFL.get(order, 0.03)
    vmax = 2.0 * math.sqrt(2.0)
    steps = int(math.ceil(2.0 * math.pi / (cfl * h / vmax)))
    return Config(f"rudman2d_{n}x{n}_p{order}", 2, order, n, centre=(2.0, 2.75),
                  radius=0.5, cfl=cfl, steps=steps, params=prm, vmax=vmax, length=L,
                  slot=(0.06, 2.65),
                  description=f"Rudman slotted disc on [0,4]^2, {n}x{n} quads, p={order}, "
                              "one rotation")


def vortex(n: int, order: int) -> Config:
    """The time-reversing single vortex of §4.2 on n x n quads (T = 8, circle r = 0.15 at
    (0.5, 0.75)), run to t = T; CFL 0.05 (0.03 for p = 5) on |v|max = 1."""
    h = 1.0 / n
    prm = default_params(2, order, h, vel_kind=VEL_SINGLE_VORTEX, vel_period=8.0)
    cfl = ROTATION_CFL.get(order, 0.03)
    steps = int(math.ceil(8.0 / (cfl * h)))
    return Config(f"vortex2d_{n}x{n}_p{order}", 2, order, n, centre=(0.5, 0.75), cfl=cfl,
                  steps=steps, params=prm, vmax=1.0,
                  description=f"single vortex T=8, {n}x{n} quads, p={order}, to t = T")


LEVEQUE_CFL = {2: 0.05, 3: 0.05, 4: 0.03, 5: 0.02}


def leveque(n: int, order: int) -> Config:
    """The LeVeque 3D deformation test of §4.3 on n^3 hexes (T = 3, sphere r = 0.15 at
    (0.35, 0.35, 0.35)), run to t = T; CFL 0.05 / 0.05 / 0.03 / 0.02 for p = 2..5 on
    |v|max = 2."""
    h = 1.0 / n
    prm = default_params(3, order, h, vel_kind=VEL_LEVEQUE3D, vel_period=3.0)
    cfl = LEVEQUE_CFL.get(order, 0.02)
    steps = int(math.ceil(3.0 / (cfl * h / 2.0)))
    return Config(f"deform3d_{n}cube_p{order}", 3, order, n, centre=(0.35, 0.35, 0.35),
                  cfl=cfl, steps=steps, params=prm, vmax=2.0,
                  description=f"LeVeque deformation T=3, {n}^3 hexes, p={order}, to t = T")


def vortex_dt(cfg: Config) -> float:
    """The step of a run to t = T (vortex or deformation) in cfg.steps steps."""
    return cfg.params.vel_period / cfg.steps


def rotation_dt(cfg: Config) -> float:
    """The step of a rotation workload: one turn (t = 2 pi) in cfg.steps steps."""
    return 2.0 * math.pi / cfg.steps


CONFIGS = {"C1": _cfg_c1, "C2": _cfg_c2, "C3": _cfg_c3, "C4": _cfg_c4, "C5": _cfg_c5,
           "T1": _cfg_t1, "T2": _cfg_t2}


def config(name: str) -> Config:
    return CONFIGS[name]()


def adjoint_target_centre(cfg: Config, seed: int = 0) -> np.ndarray:
    """Centre of the target profile of the adjoint workload: the IC centre moved by a
    seeded U(-2h, 2h) offset per coordinate."""
    rng = np.random.default_rng(seed)
    return np.asarray(cfg.centre) + rng.uniform(-2 * cfg.h, 2 * cfg.h, cfg.ndims)


def small_case(ndims: int, order: int, shape: Sequence[int], *, vel_kind=VEL_UNIFORM,
               vel_u0=None, vel_period=8.0, perturb: float = 0.0,
               periodic=True, seed: int = 3, shear: float = 0.0, **over):
    """A small mesh + parameter set for parity tests (non-cubic shapes give ragged
    element chunks). vel_u0 defaults to (1, 0.5, 0.25) for the uniform field and to the
    centre of the unit square for the rotation."""
    if vel_u0 is None:
        vel_u0 = (0.5, 0.5, 0.0) if vel_kind == VEL_ROTATION else (1.0, 0.5, 0.25)
    rng = np.random.default_rng(seed)
    planes = []
    for n in shape:
        planes.append(perturbed_planes(n, perturb, rng) if perturb > 0 else uniform_planes(n))
    per = periodic if isinstance(periodic, (list, tuple)) else [periodic] * ndims
    mesh = box_mesh(planes, per, shear=shear)
    h = 1.0 / max(shape)
    prm = default_params(ndims, order, h, vel_kind=vel_kind, vel_u0=tuple(vel_u0),
                         vel_period=vel_period, **over)
    return mesh, prm
