#!/usr/bin/env python3
"""Throughput of the FR-PCPF RK4 step on one MI355X.

Workload: 2D unit square, 128x128 affine quads, p = 4 (25 Gauss-Legendre points per
element, 409 600 DOF), time-reversing single-vortex velocity (T = 8), tanh circle r = 0.15
at (0.5, 0.75), CFL 0.05, reset + 10 pseudo-time iterations of the preconditioner before
every step whose index is a multiple of 1000 (the timed region starts at step 0, so it
contains one). A step is one classic RK4 step of the whole path (4 x [grad_flux + update]
plus the scheduled reset/preconditioning). Inputs are resident in device memory before
the timed region starts.

Prints ONE JSON line: value = DOF-stage updates per second of the FP64 form (E*N_u*4*K /
wall time of K steps), with the FP32 form, the per-kernel roofline (HIP events around
every launch of a second, identical timed region), and the CPU oracle on a bounded sample
of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "DOF-stage updates/s FP64 vs FP32/BF16 at equal interface L1 error; adjoint s/step"
UNIT = "DOF-stage updates/s"
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(d, p, word, kind):
    """Algorithmic bytes per element of one launch (inputs read + outputs written once)."""
    n = p + 1
    nu, nfa = n ** d, n ** (d - 1)
    V = 2
    geo = d + 2 * d * d + 1
    if kind == "grad_flux":
        words = V * nu + V * d * nfa + geo + V * nu + V * d * nfa
    else:  # update, averaged over the four stages (acc is not read on stage 1, not written on 4)
        words = V * nu + 2 * V * d * nfa + 1 + V * nu + 0.75 * V * nu + 0.75 * V * nu + V * nu \
            + V * d * nfa
    return words * word


def step_alg_bytes_per_dof(d, p, word):
    """B_alg per DOF-stage: RK4 registers (5 V N_u) + two face exchanges (2 V N_f)."""
    n = p + 1
    nu, nf = n ** d, 2 * d * n ** (d - 1)
    return (5 * 2 * nu + 2 * 2 * nf) * word / nu


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("pcpf_kernels.hip", "pcpf_kernels_impl.h", "pcpf_internal.h", "pcpf_device.h",
              "pcpf_mfma.h"):
        with open(os.path.join(ROOT, "paper_2006_10967_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_solver(cfg, mesh, precision):
    from paper_2006_10967_amd import Solver
    return Solver.from_box(mesh, cfg.order, cfg.params, precision=precision, device="cuda:0")


def run_form(cfg, mesh, precision, steps, warmup, phi0_np):
    import torch
    s = make_solver(cfg, mesh, precision)
    dt = cfg.dt(mesh)
    phi0 = torch.as_tensor(phi0_np).to("cuda:0", s.dtype)
    # warm-up (includes a reset + preconditioning at step 0)
    s.set_state(phi0, None, 0.0, 0)
    s.step(dt, warmup)
    # timed region: K steps from step 0 (one reset + preconditioning inside)
    s.set_state(phi0, None, 0.0, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(dt, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phi_end = s.get_state(want_psi=False)[0].clone()
    # the same region again with HIP events around every launch (per-kernel durations)
    s.set_state(phi0, None, 0.0, 0)
    s.kernel_times(reset=True)
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(dt, steps)
    torch.cuda.synchronize()
    wall_ev = time.perf_counter() - t0
    s.set_timing(False)
    kt = s.kernel_times(reset=True)
    # preconditioning alone (reset + K pseudo iterations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.precondition()
    torch.cuda.synchronize()
    pc_ms = (time.perf_counter() - t0) * 1e3
    return s, wall, wall_ev, kt, pc_ms, phi_end


def cpu_baseline(cfg, mesh, phi0_np, nsteps):
    """The FP64 CPU oracle (test infrastructure) on a bounded sample of the same workload:
    one reset + preconditioning and nsteps RK4 steps of the full mesh."""
    import torch
    from oracle import Oracle
    cores = min(16, len(os.sched_getaffinity(0)))
    torch.set_num_threads(cores)
    o = Oracle(cfg.ndims, cfg.order, mesh, cfg.params)
    phi = torch.as_tensor(phi0_np, dtype=torch.float64)
    t0 = time.perf_counter()
    psi, _ = o.precondition(phi)
    t_pc = time.perf_counter() - t0
    dt = cfg.dt(mesh)
    t0 = time.perf_counter()
    t = 0.0
    for _ in range(nsteps):
        phi, psi = o.step(phi, psi, t, dt)
        t += dt
    t_steps = time.perf_counter() - t0
    rate = cfg.dof * 4 * nsteps / t_steps
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": rate, "unit": UNIT, "cores": torch.get_num_threads(), "kind": "oracle",
            "cpu": cpu,
            "sample": f"full {cfg.n}x{cfg.n} p={cfg.order} mesh: {nsteps} RK4 steps "
                      f"({t_steps:.1f} s) after one reset + {cfg.params.precond_iters} "
                      f"pseudo iterations ({t_pc:.1f} s, not in value)",
            "s_per_step": t_steps / nsteps,
            "small_workload_full_run": small_workload_run()}


def small_workload_run():
    """The 16x16 p=3 advection workload run whole (reset + 10 pseudo iterations + 200 RK4
    steps) by the FP64 oracle on the host cores and by the FP64 GPU path: seconds of
    each, the mass error of each and the largest relative difference of the final phi."""
    import torch
    import workloads as W
    from oracle import Oracle
    from paper_2006_10967_amd import Solver
    cfg = W.config("C1")
    mesh = cfg.mesh()
    dt = cfg.dt(mesh)
    o = Oracle(cfg.ndims, cfg.order, mesh, cfg.params)
    phi0 = torch.as_tensor(cfg.initial_phi(o.coords()), dtype=torch.float64)
    t0 = time.perf_counter()
    phi_o, _, _ = o.run(phi0, None, 0.0, dt, cfg.steps)
    t_oracle = time.perf_counter() - t0
    s = Solver.from_box(mesh, cfg.order, cfg.params, precision="fp64", device="cuda:0")
    g0 = phi0.to("cuda:0")
    s.set_state(g0)
    s.step(dt, 5)                                   # warm-up (module load, first launches)
    s.set_state(g0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(dt, cfg.steps)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    phi_g = s.get_state(want_psi=False)[0].cpu()
    m0 = float(o.mass(phi0))
    return {"workload": cfg.name, "steps": cfg.steps, "oracle_s": t_oracle, "gpu_s": t_gpu,
            "E_m_oracle": float(o.mass_error(phi_o, phi0, phi0)),
            "E_m_gpu": (s.mass() - m0) / m0,
            "phi_rel_diff": float((phi_g - phi_o).abs().max() / phi_o.abs().max())}


def adjoint_leg(precision, steps, every):
    """The adjoint workload (64x64 p=3 single vortex, L2 mismatch of phi(T) against a
    seeded target circle): checkpointed forward run + reverse sweep; seconds per step."""
    import torch
    import workloads as W
    from paper_2006_10967_amd import MeshArgs, Solver
    cfg = W.config("C4")
    mesh = cfg.mesh()
    s = Solver.from_box(mesh, cfg.order, cfg.params, precision=precision, device="cuda:0")
    period = [float(mesh.period[k]) if mesh.periodic[k] else 0.0 for k in range(cfg.ndims)]
    x = MeshArgs(cfg.ndims, cfg.order, mesh.x0, mesh.jac, mesh.nbr, period).solution_coords()
    phi0 = torch.as_tensor(W.ic_phi(x, cfg.centre, cfg.radius, cfg.params.eps_w)).to(
        "cuda:0", s.dtype)
    tgt = torch.as_tensor(W.ic_phi(x, W.adjoint_target_centre(cfg), cfg.radius,
                                   cfg.params.eps_w)).to("cuda:0", s.dtype)
    det = torch.as_tensor(mesh.jac).reshape(cfg.nelem, cfg.ndims, cfg.ndims).det()
    w1 = torch.as_tensor(s.mesh.ops["weights"])
    wq = (det[:, None] * torch.kron(w1, w1)[None, :]).to("cuda:0", s.dtype)
    dt = cfg.dt(mesh)
    s.set_state(phi0, None, 0.0, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.forward_ckpt(dt, steps, every)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    phiT = s.get_state(want_psi=False)[0]
    seed = wq * (phiT - tgt)
    loss = 0.5 * float(torch.sum(wq.double() * (phiT.double() - tgt.double()) ** 2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gphi0, _, ga = s.adjoint(seed)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    return {"s_per_step": (t_fwd + t_adj) / steps, "adjoint_s_per_step": t_adj / steps,
            "forward_ckpt_s_per_step": t_fwd / steps, "steps": steps, "ckpt_every": every,
            "dof": cfg.dof, "loss": loss, "dL_dA": ga,
            "max_abs_dL_dphi0": float(gphi0.abs().max())}


def accuracy_leg(cfg, mesh, phi0_np):
    """The vortex test to t = T (§4): E_L1 = int|phi(T) - phi(0)|, E_r = E_L1 / int phi(0)
    and E_m = (int phi(T) - int phi(0)) / int phi(0), FP64, for each form of
    precond_variants; then the FP32 and BF16 forms with the default readings, each against
    the FP64 run: "equal interface error" holds when |E_L1 - E_L1,64| <= 0.02 E_L1,64 and
    int|phi - phi_64| <= 0.1 E_L1,64 at t = T."""
    import torch
    from paper_2006_10967_amd import Solver
    T = cfg.params.vel_period
    dt = cfg.dt(mesh)
    nsteps = int(round(T / dt))
    with open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")) as fh:
        paper = json.load(fh)["vortex_E_L1"][f"p{cfg.order}"][2] if cfg.n == 128 else None
    out = {"t_end": nsteps * dt, "steps": nsteps, "E_L1_paper": paper}
    ref = None
    for name, prm in precond_variants(cfg.params):
        s = Solver.from_box(mesh, cfg.order, prm, precision="fp64", device="cuda:0")
        phi0 = torch.as_tensor(phi0_np).to("cuda:0", s.dtype)
        s.set_state(phi0, phi0 - 0.5 if prm.normal_mode == 1 else None, 0.0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(dt, nsteps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        phiT = s.get_state(want_psi=False)[0]
        m0 = s.mass(phi0)
        e_l1 = s.l1(phi0, phiT)
        out[name] = {"E_L1": e_l1, "E_r": e_l1 / m0, "E_m": (s.mass(phiT) - m0) / m0,
                     "wall_s": wall, "last_precond_iters_rms": last_precond(s)}
        log(f"[bench] {cfg.name} to t = T ({name}): E_L1 = {e_l1:.4e}, "
            f"E_m = {out[name]['E_m']:.2e}, {wall:.2f} s")
        if ref is None:
            ref = (s, phi0, phiT.clone(), e_l1, m0, wall)
        else:
            del s
    s64, phi0, phi64, e64, m0, wall64 = ref
    out["forms_default_readings"] = {}
    for form in ("fp32", "bf16"):
        s = Solver.from_box(mesh, cfg.order, cfg.params, precision=form, device="cuda:0")
        s.set_state(phi0.to(s.dtype), None, 0.0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(dt, nsteps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        phiT = s.get_state(want_psi=False)[0].double()
        e_l1 = s64.l1(phi0, phiT)
        diff = s64.l1(phi64, phiT)
        r = {"E_L1": e_l1, "E_r": e_l1 / m0, "E_m": (s64.mass(phiT) - m0) / m0,
             "int_abs_diff_vs_fp64": diff, "wall_s": wall, "speedup_vs_fp64": wall64 / wall,
             "equal_interface_error": bool(abs(e_l1 - e64) <= 0.02 * e64 and diff <= 0.1 * e64)}
        out["forms_default_readings"][form] = r
        log(f"[bench] {cfg.name} to t = T ({form}): E_L1 = {e_l1:.4e} (fp64 {e64:.4e}), "
            f"int|phi-phi64| = {diff:.2e}, equal: {r['equal_interface_error']}, "
            f"x{r['speedup_vs_fp64']:.2f}")
        del s
    return out


def deformation_leg():
    """The LeVeque deformation test on 64^3 hexes, p = 3, run to t = T = 3 (§4.3), FP64:
    E_L1 = int|phi(T) - phi(0)| and E_m with the default readings and with the longer
    preconditioning, next to the paper's E_L1 for this mesh and order (context)."""
    import torch
    import workloads as W
    from paper_2006_10967_amd import Solver
    cfg = W.config("C3")
    mesh = cfg.mesh()
    dt = cfg.dt(mesh)
    nsteps = int(round(cfg.params.vel_period / dt))
    with open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")) as fh:
        paper = json.load(fh)["leveque_E_L1"]["p3"][1]
    out = {"workload": cfg.name, "t_end": nsteps * dt, "steps": nsteps, "E_L1_paper": paper}
    for name, prm in precond_variants(cfg.params)[::2]:
        s = Solver.from_box(mesh, cfg.order, prm, precision="fp64", device="cuda:0")
        phi0 = torch.as_tensor(cfg.initial_phi(s.solution_coords())).to("cuda:0", s.dtype)
        s.set_state(phi0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(dt, nsteps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        m0 = s.mass(phi0)
        e_l1 = s.l1(phi0)
        out[name] = {"E_L1": e_l1, "E_m": (s.mass() - m0) / m0, "wall_s": wall,
                     "dof_stage_per_s": cfg.dof * 4 * nsteps / wall}
        log(f"[bench] {cfg.name} to t = T ({name}): E_L1 = {e_l1:.4e} (paper {paper:.2e}), "
            f"E_m = {out[name]['E_m']:.1e}, {wall:.1f} s")
        del s, phi0
        torch.cuda.empty_cache()
    return out


def vortex_table_leg(sizes=(32, 64, 128), orders=(2, 3, 4, 5)):
    """The single-vortex test of §4.2 to t = T on n x n quads for the paper's table of
    E_L1 (FP64): the default readings and the longer preconditioning, next to the paper's
    value for the same mesh and order (context)."""
    import torch
    import workloads as W
    from paper_2006_10967_amd import Solver
    with open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")) as fh:
        gold = json.load(fh)["vortex_E_L1"]
    out = {}
    for i, n in enumerate(sizes):
        for p in orders:
            cfg = W.vortex(n, p)
            mesh = cfg.mesh()
            dt = W.vortex_dt(cfg)
            res = {"steps": cfg.steps, "E_L1_paper": gold[f"p{p}"][i]}
            for name, prm in precond_variants(cfg.params)[::2]:
                s = Solver.from_box(mesh, p, prm, precision="fp64", device="cuda:0")
                phi0 = torch.as_tensor(cfg.initial_phi(s.solution_coords())).to("cuda:0", s.dtype)
                s.set_state(phi0)
                s.step(dt, cfg.steps)
                m0 = s.mass(phi0)
                res[name] = {"E_L1": s.l1(phi0), "E_m": (s.mass() - m0) / m0}
                del s
            out[cfg.name] = res
            log(f"[bench] {cfg.name} to t = T: E_L1 {res['preconditioned']['E_L1']:.3e} "
                f"(K20: {res['preconditioned_K20_dtau2x_N500']['E_L1']:.3e}; "
                f"paper {res['E_L1_paper']:.2e})")
    return out


def leveque_table_leg(sizes=(32,), orders=(2, 3, 4, 5)):
    """The LeVeque deformation test of §4.3 to t = T on n^3 hexes (FP64), default readings
    and the longer preconditioning, next to the paper's E_L1 (context)."""
    import torch
    import workloads as W
    from paper_2006_10967_amd import Solver
    with open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")) as fh:
        gold = json.load(fh)["leveque_E_L1"]
    out = {}
    for n in sizes:
        col = {32: 0, 64: 1, 128: 2}[n]
        for p in orders:
            cfg = W.leveque(n, p)
            mesh = cfg.mesh()
            dt = W.vortex_dt(cfg)
            res = {"steps": cfg.steps, "E_L1_paper": gold[f"p{p}"][col]}
            for name, prm in precond_variants(cfg.params)[::2]:
                s = Solver.from_box(mesh, p, prm, precision="fp64", device="cuda:0")
                phi0 = torch.as_tensor(cfg.initial_phi(s.solution_coords())).to("cuda:0", s.dtype)
                s.set_state(phi0)
                t0 = time.perf_counter()
                s.step(dt, cfg.steps)
                torch.cuda.synchronize()
                m0 = s.mass(phi0)
                res[name] = {"E_L1": s.l1(phi0), "E_m": (s.mass() - m0) / m0,
                             "wall_s": time.perf_counter() - t0}
                del s
            out[cfg.name] = res
            log(f"[bench] {cfg.name} to t = T: E_L1 {res['preconditioned']['E_L1']:.3e} "
                f"(K20: {res['preconditioned_K20_dtau2x_N500']['E_L1']:.3e}; "
                f"paper {res['E_L1_paper']:.2e})")
    return out


def last_precond(s):
    """[iterations, stop-rule RMS] of the solver's last preconditioning (None if none ran)."""
    from paper_2006_10967_amd import PcpfError
    try:
        k, rms = s.precond_info()
    except PcpfError:
        return None
    return [k, rms if math.isfinite(rms) else None]


def precond_variants(prm):
    """The method with the default readings, the unpreconditioned form (normal from phi),
    the method given four times the pseudo-time per reset (K = 20 at twice the pseudo
    step, resets every 500 steps: inside the 5-20 iterations and 500-2000 steps the paper
    quotes, the pseudo step just under its RK4 limit), and the printed forms of the sign
    (current |grad psi|) and of the stop rule (RMS <= 1/2, at most 20 iterations)."""
    import dataclasses
    return (("preconditioned", prm),
            ("unpreconditioned", dataclasses.replace(prm, normal_mode=1, reset_every=0)),
            ("preconditioned_K20_dtau2x_N500",
             dataclasses.replace(prm, precond_iters=20, dtau=2 * prm.dtau, reset_every=500)),
            ("preconditioned_printed_sign_rms_stop",
             dataclasses.replace(prm, sgn_mode=1, stop_mode=1, precond_iters=20)))


def rotation_leg(orders=(2, 3, 4, 5)):
    """The slotted-disc solid-body rotation tests of §4.1, one whole turn each, FP64:
    Zalesak's disc on 100^2 and 200^2 quads and Rudman's disc on 200^2 quads of [0, 4]^2,
    p = 2..5, for each form of precond_variants. Reports E_r, E_m, the wall time of the
    turn (resets and pseudo-iterations included) and the DOF-stage rate, next to the
    paper's E_r for the same mesh and order (context: the paper's tau, pseudo step, K and
    CFL are not stated)."""
    import torch
    import workloads as W
    from paper_2006_10967_amd import Solver
    with open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")) as fh:
        gold = json.load(fh)
    runs = [(W.zalesak(n, p), gold["zalesak_E_r"][f"p{p}"][i])
            for i, n in enumerate((100, 200)) for p in orders]
    runs += [(W.rudman(p), gold["rudman_E_r"][f"p{p}"]) for p in orders]
    out = {}
    for cfg, paper in runs:
        mesh = cfg.mesh()
        dt = W.rotation_dt(cfg)
        res = {"steps": cfg.steps, "dt": dt, "dof": cfg.dof, "E_r_paper": paper}
        for name, prm in precond_variants(cfg.params):
            s = Solver.from_box(mesh, cfg.order, prm, precision="fp64", device="cuda:0")
            phi0 = torch.as_tensor(cfg.initial_phi(s.solution_coords())).to("cuda:0", s.dtype)
            s.set_state(phi0, phi0 - 0.5 if prm.normal_mode == 1 else None, 0.0, 0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(dt, cfg.steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            m0 = s.mass(phi0)
            e_l1 = s.l1(phi0)
            res[name] = {"E_L1": e_l1, "E_r": e_l1 / m0, "E_m": (s.mass() - m0) / m0,
                         "wall_s": wall, "dof_stage_per_s": cfg.dof * 4 * cfg.steps / wall,
                         "last_precond_iters_rms": last_precond(s)}
            log(f"[bench] {cfg.name} one turn ({name}): E_r = {e_l1 / m0:.3e} "
                f"(paper {paper:.2e}), E_m = {res[name]['E_m']:.1e}, {wall:.2f} s")
            del s
        out[cfg.name] = res
    # long-time behaviour (§4.1, the slot corners over several turns): Zalesak 100^2 p4,
    # E_r after each of four turns
    cfg = W.zalesak(100, 4)
    mesh = cfg.mesh()
    dt = W.rotation_dt(cfg)
    multi = {}
    for name, prm in precond_variants(cfg.params)[::2]:
        s = Solver.from_box(mesh, cfg.order, prm, precision="fp64", device="cuda:0")
        phi0 = torch.as_tensor(cfg.initial_phi(s.solution_coords())).to("cuda:0", s.dtype)
        s.set_state(phi0)
        m0 = s.mass(phi0)
        per_turn = []
        for _ in range(4):
            s.step(dt, cfg.steps)
            per_turn.append({"E_r": s.l1(phi0) / m0, "E_m": (s.mass() - m0) / m0})
        multi[name] = per_turn
        log(f"[bench] {cfg.name} four turns ({name}): E_r "
            + " ".join(f"{x['E_r']:.3e}" for x in per_turn))
        del s
    out["zalesak2d_100x100_p4_four_turns"] = multi
    return out


def load_traffic(workload, kernel, hsh):
    """Counter-measured HBM bytes per launch of a kernel on a workload, recorded in
    profiles/traffic_<workload>.json for the kernel sources of hash hsh (else None)."""
    try:
        with open(os.path.join(PROFILES, f"traffic_{workload}.json")) as fh:
            data = json.load(fh)
    except OSError:
        return None
    if data.get("kernel_source_hash") != hsh:
        return None
    return data.get("per_launch_bytes", {}).get(kernel)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=200)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the run to t = T of the vortex workload (both normal forms)")
    ap.add_argument("--no-rotation", action="store_true",
                    help="skip the slotted-disc rotation tests (Zalesak, Rudman; one turn each)")
    ap.add_argument("--deformation", action="store_true",
                    help="also run the 64^3 p=3 LeVeque test to t = T (about a minute)")
    ap.add_argument("--vortex-table", action="store_true",
                    help="also run the single vortex to t = T on 32^2..128^2, p = 2..5")
    ap.add_argument("--leveque-table", action="store_true",
                    help="also run the 3D deformation to t = T on 32^3, p = 2..5")
    ap.add_argument("--adj-steps", type=int, default=512)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2006_10967_amd import MeshArgs

    cfg = W.config(args.config)
    mesh = cfg.mesh()
    period = [float(mesh.period[k]) if mesh.periodic[k] else 0.0 for k in range(cfg.ndims)]
    coords = MeshArgs(cfg.ndims, cfg.order, mesh.x0, mesh.jac, mesh.nbr, period).solution_coords()
    phi0 = W.ic_phi(coords, cfg.centre, cfg.radius, cfg.params.eps_w)
    K, Wm = args.steps, args.warmup
    log(f"[bench] {cfg.name}: E={cfg.nelem} N_u={cfg.nupts} DOF={cfg.dof} steps={K} warmup={Wm}")

    if args.copy_mb > 0:
        # a plain copy of known size: reads and writes copy_mb MiB once each
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    s64, wall64, wall64_ev, kt64, pc64, phi64 = run_form(cfg, mesh, "fp64", K, Wm, phi0)
    value = cfg.dof * 4 * K / wall64
    log(f"[bench] fp64: {wall64 * 1e3 / K:.4f} ms/step, {value:.4e} DOF-stage/s")

    # roofline of the dominant kernel (HIP-event durations of the second timed region)
    word = 8
    kern = max(("grad_flux", "update"), key=lambda k: kt64[k][0])
    ms, nl = kt64[kern]
    avg_s = ms / nl * 1e-3
    bytes_launch = kernel_bytes(cfg.ndims, cfg.order, word, kern) * cfg.nelem
    achieved = bytes_launch / avg_s / 1e9
    hsh = kernel_source_hash()
    traffic = load_traffic(cfg.name, kern, hsh)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kern,
                "alg_bytes_per_launch": bytes_launch,
                "avg_launch_us": avg_s * 1e6}
    kernels = {k: {"avg_us": (v[0] / v[1] * 1e3) if v[1] else None, "launches": v[1],
                   "alg_bytes_per_launch": kernel_bytes(cfg.ndims, cfg.order, word, k) * cfg.nelem
                   if k in ("grad_flux", "update") else None}
               for k, v in kt64.items()}
    for k in ("grad_flux", "update"):
        if kernels[k]["avg_us"]:
            kernels[k]["alg_GBs"] = kernels[k]["alg_bytes_per_launch"] / (kernels[k]["avg_us"] * 1e3)
    step_bytes = step_alg_bytes_per_dof(cfg.ndims, cfg.order, word) * cfg.dof * 4
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": wall64 * 1e3 / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg.name, "description": cfg.description,
                   "elements": cfg.nelem, "order": cfg.order, "dof": cfg.dof,
                   "dt": cfg.dt(mesh), "reset_every": cfg.params.reset_every,
                   "precond_iters": cfg.params.precond_iters},
        "roofline": roofline,
        "kernels_fp64": kernels,
        "step_alg_GBs_fp64": step_bytes / (wall64 / K * 1e9),
        "ms_per_step_with_events": wall64_ev * 1e3 / K,
        "precondition_ms_fp64": pc64,
    }

    forms = [f for f, off in (("fp32", args.no_fp32), ("bf16", args.no_bf16)) if not off]
    if forms:
        out["forms"] = {}
        mass64 = s64.mass(phi64)
        mass0 = s64.mass(torch.as_tensor(phi0))
        ref = s64.mass(phi64)
    for form in forms:
        sf, wallf, _, ktf, pcf, phif = run_form(cfg, mesh, form, K, Wm, phi0)
        vf = cfg.dof * 4 * K / wallf
        l1 = s64.l1(phi64, phif.double())
        massf = s64.mass(phif.double())
        out["forms"][form] = {
            "value": vf, "ms_per_step": wallf * 1e3 / K, "speedup_vs_fp64": vf / value,
            "interface_l1_vs_fp64": l1, "interface_l1_vs_fp64_rel": l1 / ref,
            "mass_drift": (massf - mass0) / mass0,
            "mass_drift_fp64": (mass64 - mass0) / mass0, "precondition_ms": pcf,
            "kernels": {k: {"avg_us": (v[0] / v[1] * 1e3) if v[1] else None}
                        for k, v in ktf.items()}}
        log(f"[bench] {form}: {wallf * 1e3 / K:.4f} ms/step, {vf:.4e} DOF-stage/s, "
            f"int|phi_{form}-phi64| = {l1:.3e}")
        del sf

    if not args.no_accuracy and cfg.params.vel_kind == W.VEL_SINGLE_VORTEX:
        out["accuracy"] = accuracy_leg(cfg, mesh, phi0)

    if not args.no_rotation:
        out["rotation"] = rotation_leg()

    if args.deformation:
        out["deformation"] = deformation_leg()

    if args.vortex_table:
        out["vortex_table"] = vortex_table_leg()

    if args.leveque_table:
        out["leveque_table"] = leveque_table_leg()

    if not args.no_adjoint:
        adj = {}
        for prec in ("fp64", "fp32"):
            adj[prec] = adjoint_leg(prec, args.adj_steps, 32)
            log(f"[bench] adjoint {prec}: {adj[prec]['s_per_step'] * 1e3:.3f} ms/step "
                f"(forward+reverse), dL/dA = {adj[prec]['dL_dA']:.6e}")
        adj["fp32"]["dL_dA_rel_vs_fp64"] = abs(adj["fp32"]["dL_dA"] - adj["fp64"]["dL_dA"]) \
            / abs(adj["fp64"]["dL_dA"])
        out["adjoint"] = {"workload": "adjoint2d_64x64_p3", **adj}

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(cfg, mesh, phi0, args.cpu_steps)
        log(f"[bench] oracle: {out['cpu_baseline']['value']:.4e} DOF-stage/s on "
            f"{out['cpu_baseline']['cores']} cores")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
