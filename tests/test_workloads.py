"""Pins of the synthetic inputs: the slotted-disc signed distance of §4.1 and the rigid
rotation field (both shared by the GPU path's callers and by the oracle).

The distance is checked against brute force (the least distance to a dense sampling of
the boundary: the circle arc outside the slot and the three slot walls) and its sign
against membership in the disc less the slot; the rotation field against the kinematics
of a rigid rotation."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import velocity as ovel


def _boundary_samples(c, r, w, top, n=40_000):
    th = np.linspace(0.0, 2 * math.pi, n, endpoint=False)
    arc = np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th)], -1)
    keep = ~((np.abs(arc[:, 0] - c[0]) < w) & (arc[:, 1] < top))
    ybot = c[1] - math.sqrt(r * r - w * w)
    s = np.linspace(0.0, 1.0, n // 10)
    walls = [np.stack([np.full_like(s, c[0] - w), ybot + s * (top - ybot)], -1),
             np.stack([np.full_like(s, c[0] + w), ybot + s * (top - ybot)], -1),
             np.stack([c[0] - w + s * 2 * w, np.full_like(s, top)], -1)]
    return np.concatenate([arc[keep]] + walls), 2 * math.pi * r / n + (top - ybot) / (n // 10)


def _brute(x, pts):
    out = np.empty(len(x))
    for i in range(0, len(x), 256):
        d = np.sqrt(((x[i:i + 256, None, :] - pts[None, :, :]) ** 2).sum(-1))
        out[i:i + 256] = d.min(1)
    return out


def _case(name):
    g = dict(zalesak=((0.5, 0.75), 0.15, 0.025, 0.85), rudman=((2.0, 2.75), 0.5, 0.06, 2.65))
    return g[name]


def test_slotted_disc_distance_brute_force():
    rng = np.random.default_rng(11)
    for name in ("zalesak", "rudman"):
        c, r, w, top = _case(name)
        # points in a box around the disc, denser near the slot
        x = np.concatenate([rng.uniform([c[0] - 1.5 * r, c[1] - 1.5 * r],
                                        [c[0] + 1.5 * r, c[1] + 1.5 * r], (600, 2)),
                            rng.uniform([c[0] - 3 * w, c[1] - 1.2 * r],
                                        [c[0] + 3 * w, top + 2 * w], (600, 2))])
        sd = W.signed_distance_slotted_disc(x, c, r, w, top)
        pts, spacing = _boundary_samples(c, r, w, top)
        assert np.max(np.abs(np.abs(sd) - _brute(x, pts))) <= spacing
        inside = (np.hypot(x[:, 0] - c[0], x[:, 1] - c[1]) < r) & \
            ~((np.abs(x[:, 0] - c[0]) <= w) & (x[:, 1] <= top))
        far = np.abs(sd) > 1e-9
        assert np.all((sd[far] > 0) == inside[far])


def test_slotted_disc_distance_special_points():
    c, r, w, top = _case("zalesak")
    pts = np.array([[0.5, 0.75],          # slot middle: half width to either wall
                    [0.5, 0.865],         # above the slot top: 0.015 to it, 0.035 to the circle
                    [0.5, 0.95],          # above the disc: 0.05 outside
                    [0.25, 0.75],         # left of the disc, far from the slot
                    [0.5 + w, 0.9 - r]])  # on a wall
    want = [-w, 0.015, -0.05, -0.1, 0.0]
    got = W.signed_distance_slotted_disc(pts, c, r, w, top)
    assert np.allclose(got, want, atol=1e-15), got
    # away from the slot it is the disc distance of Eq. discEq
    th = np.linspace(0.2, math.pi - 0.2, 50)
    for rho in (0.05, 0.14, 0.2):
        q = np.stack([c[0] + rho * np.cos(th), c[1] + rho * np.sin(th)], -1)
        q = q[q[:, 1] > top + 0.01]
        assert np.allclose(W.signed_distance_slotted_disc(q, c, r, w, top),
                           W.signed_distance_ball(q, c, r), atol=1e-15)


def test_rotation_field_is_rigid():
    rng = np.random.default_rng(5)
    for cen in ((0.5, 0.5), (2.0, 2.0)):
        x = torch.as_tensor(rng.uniform(-1, 5, (200, 2)))
        v = ovel.spatial(ovel.ROTATION, x, (cen[0], cen[1], 0.0))
        rel = x - torch.tensor(cen, dtype=torch.float64)
        assert float((v * rel).sum(-1).abs().max()) < 1e-13            # v is normal to x - c
        assert torch.allclose(v.norm(dim=-1), rel.norm(dim=-1), atol=1e-13)  # unit rate
        assert float((rel[:, 0] * v[:, 1] - rel[:, 1] * v[:, 0]).min()) > 0  # counter-clockwise
        assert float(ovel.spatial(ovel.ROTATION, torch.tensor([cen], dtype=torch.float64),
                                  (cen[0], cen[1], 0.0)).abs().max()) == 0.0


@pytest.mark.parametrize("shape,shear,periodic", [
    ((4, 5, 3), (0.25, 0.05, 0.2), (True, True, True)),
    ((3, 3, 4), (1.0 / 3, -2.0 / 9, 1.0 / 3), (True, True, True)),
    ((4, 3, 3), (0.3, -0.2, 0.1), (False, False, False)),
    ((4, 5, 3), (0.25, 0.05, 0.2), (True, False, True)),
])
def test_skewed_3d_mesh_adjacency(shape, shear, periodic):
    """The skewed hex mesh (x = S b with a unit upper-triangular S): a full Jacobian, and
    its face adjacency equals the pairing of flux points by physical coordinates that the
    oracle builds independently (modulo the axis-aligned periods)."""
    from oracle.mesh import Discretisation
    from oracle.operators import ElementOperators
    planes = [W.uniform_planes(n) for n in shape]
    mesh = W.box_mesh(planes, periodic, shear=shear)
    assert np.abs(mesh.jac[:, 0, 1]).max() > 0 or shear[0] == 0
    assert np.abs(mesh.jac[:, 0, 2]).max() > 0 and np.abs(mesh.jac[:, 1, 2]).max() > 0
    ops = ElementOperators(3, 2)
    disc = Discretisation.from_box(ops, mesh)
    nfa = 9
    for e in range(mesh.nelem):
        for f in range(6):
            slots = np.arange(f * nfa, (f + 1) * nfa)
            en = mesh.nbr[e, f]
            if en < 0:
                assert not disc.has_pair[e, slots].any()
                continue
            assert disc.has_pair[e, slots].all()
            assert np.all(disc.pair_e[e, slots] == en)
            # the partner slots lie on the opposite face of the neighbour, in the same order
            g = f ^ 1
            assert np.array_equal(disc.pair_j[e, slots], np.arange(g * nfa, (g + 1) * nfa))
