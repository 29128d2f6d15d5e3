"""The parameter values the paper prints (tests/golden/paper_parameters.json, each with
its citation) against the defaults the workloads use."""
import json
import math
import os

import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


def test_defaults_follow_paper():
    for d, p, N in [(2, 3, 16), (2, 4, 128), (3, 3, 64), (3, 4, 96)]:
        h = 1.0 / N
        prm = W.default_params(d, p, h)
        assert prm.gamma == GOLD["gamma"]["value"]
        assert math.isclose(prm.eps, GOLD["eps_times_p_over_h"]["value"] * h / p, rel_tol=1e-15)
        assert prm.s0 == GOLD["s0"]["value"]
        assert math.isclose(prm.nu_max, GOLD["nu_max_times_p_over_h"]["value"] * h / p, rel_tol=1e-15)
        assert prm.reset_every == GOLD["reset_every"]["value"]
        lo, hi = GOLD["pseudo_iterations"]["value"]
        assert lo <= prm.precond_iters <= hi
        # IC width: phi = (1 + tanh(beta psi_d))/2 with beta = 3p/(4h) = 1/(2 eps_w)
        beta = GOLD["ic_beta_times_h_over_p"]["value"] * p / h
        assert math.isclose(prm.eps_w, 1.0 / (2 * beta), rel_tol=1e-15)
        # the equilibrium width eps/gamma of the localized equation equals eps_w
        assert math.isclose(prm.eps / prm.gamma, prm.eps_w, rel_tol=1e-14)
    # kappa: the printed 5x10^3 is read as 5 (a ramp over [s0 - 5, s0 + 5])
    assert GOLD["kappa_printed"]["value"] == 5000.0 and W.default_params(2, 3, 0.1).kappa == 5.0


def test_workload_shapes():
    c2 = W.config("C2")
    assert c2.dof == 409600 and c2.params.vel_period == GOLD["vortex_period"]["value"]
    assert tuple(c2.centre) == tuple(GOLD["disk"]["centre"]) and c2.radius == GOLD["disk"]["radius"]
    c3 = W.config("C3")
    assert c3.dof == 64 ** 3 * 64 and c3.params.vel_period == GOLD["leveque_period"]["value"]
    assert tuple(c3.centre) == tuple(GOLD["sphere"]["centre"])
    c5 = W.config("C5")
    assert c5.dof == 96 ** 3 * 125
    assert W.config("C1").dof == 4096


def test_slotted_disc_workloads():
    z, r = GOLD["zalesak"], GOLD["rudman"]
    for n in z["meshes"]:
        for p in (2, 3, 4, 5):
            c = W.zalesak(n, p)
            assert c.dof == n * n * (p + 1) ** 2 and c.length == 1.0
            assert tuple(c.centre) == tuple(z["centre"]) and c.radius == z["radius"]
            assert c.slot == (z["slot_half_width"], z["slot_top"])
            assert tuple(c.params.vel_u0[:2]) == tuple(z["rotation_centre"])
            assert c.params.vel_kind == W.VEL_ROTATION
            # a whole number of steps makes exactly one turn, inside the CFL bound
            assert math.isclose(W.rotation_dt(c) * c.steps, 2 * math.pi, rel_tol=1e-15)
            assert W.rotation_dt(c) <= c.dt()
    for p in (2, 3, 4, 5):
        c = W.rudman(p)
        assert c.n == r["mesh"] and c.length == r["domain"] and math.isclose(c.h, 0.02)
        assert tuple(c.centre) == tuple(r["centre"]) and c.radius == r["radius"]
        assert c.slot == (r["slot_half_width"], r["slot_top"])
        assert tuple(c.params.vel_u0[:2]) == tuple(r["rotation_centre"])
        assert float(c.mesh().planes[0][-1]) == r["domain"]
