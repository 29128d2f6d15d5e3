"""pcpf_adjoint_static (the adjoint for callers that cannot allocate: its scratch is a
static per-GPU array of the library) against pcpf_adjoint with caller memory, through the
C ABI: bitwise the same gradients on two calls in a row, the second on a smaller mesh (the
static array then holds the first call's contents), and a clear error for a run whose
scratch exceeds the static size."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _run(d, p, shape, kw, nsteps, every, seed):
    from paper_2006_10967_amd import Solver
    mesh, prm = W.small_case(d, p, shape, **kw)
    s = Solver.from_box(mesh, p, prm)
    x = s.solution_coords()
    rng = np.random.default_rng(seed)
    c = np.full(d, 0.5) + rng.uniform(-0.08, 0.08, d)
    phi0 = torch.tensor(W.ic_phi(x, c, 0.28, 0.08))
    gphi = torch.tensor(rng.standard_normal(phi0.shape))
    gpsi = torch.tensor(rng.standard_normal(phi0.shape))
    dt = 0.05 * float(min(np.min(np.diff(pl)) for pl in mesh.planes))
    s.set_velocity_amplitude(0.9)
    s.set_state(phi0, None, 0.0, 0)
    s.forward_ckpt(dt, nsteps, every)
    return s, gphi, gpsi


def test_static_adjoint_matches_caller_memory_adjoint():
    from paper_2006_10967_amd import _lib
    cases = [(2, 3, (12, 10), dict(vel_kind=W.VEL_SINGLE_VORTEX, vel_period=4.0,
                                   precond_iters=3, reset_every=6), 12, 3, 1),
             (2, 2, (6, 5), dict(vel_u0=(0.8, -0.4), precond_iters=2, reset_every=4), 8, 2, 2)]
    for d, p, shape, kw, nsteps, every, seed in cases:
        s, gphi, gpsi = _run(d, p, shape, kw, nsteps, every, seed)
        sa = s.adjoint_static(gphi, gpsi)
        ref = s.adjoint(gphi, gpsi)
        sb = s.adjoint_static(gphi, gpsi)           # again, after the caller-memory sweep
        for got in (sa, sb):
            assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
            assert got[2] == ref[2]
        print(f"[no-alloc] {shape} p={p}: dL/dA {ref[2]:.6e}, bitwise equal")
    # a run whose adjoint scratch exceeds the static array is refused with a message
    cfg = W.config("C4")
    from paper_2006_10967_amd import PcpfError, Solver
    mesh = cfg.mesh()
    s = Solver.from_box(mesh, cfg.order, cfg.params)
    phi0 = torch.tensor(W.ic_phi(s.solution_coords(), cfg.centre, cfg.radius, cfg.params.eps_w))
    s.set_state(phi0, None, 0.0, 0)
    s.forward_ckpt(cfg.dt(mesh), 64, 32)
    with pytest.raises(PcpfError) as e:
        s.adjoint_static(torch.ones_like(phi0))
    assert e.value.status == _lib.PCPF_EINVAL and "static" in str(e.value)
