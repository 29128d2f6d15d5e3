#!/usr/bin/env python3
"""Throughput of the FR-PCPF RK4 step on one MI355X.

Headline workload: the 3D deformation test of §4.3 on the unit cube, 96^3 affine hexes whose
interior grid planes are shifted by U(-0.2h, 0.2h) (seed 1), p = 4 (125 Gauss-Legendre
points per element, 110 592 000 DOF), LeVeque field with T = 3, sphere r = 0.15 at
(0.35, 0.35, 0.35), CFL 0.03 on the smallest spacing. It is the largest of the benchmark
configurations that fits one GPU, and the one the BF16 form is quoted on.

A step is one classic RK4 step of the whole path: 4 x [grad_flux + update]. The reset
and the preconditioning (10 pseudo-time RK4 iterations) run before step 0; the timed
region starts after them and after the warm-up steps, so it holds K plain steps (a reset
lands inside only if the region crosses a multiple of the reset interval, 1000). The reset
+ preconditioning is timed on its own and reported beside. Inputs are resident in device
memory before the timed region starts.

Prints ONE JSON line:
  value        DOF-stage updates per second of the FP64 form, E N_u 4 K / wall time;
  forms        the FP32 and BF16 forms on the same workload: rate, speed-up, and after
               100 steps from the same initial state the interface L1 difference
               int|phi_form - phi_64| and the mass drift of each form;
  roofline     the RK stage (grad_flux + update, HIP events around every launch of a
               second timed region) against HBM: algorithmic bytes per stage
               (5 V N_u + 2 V N_f words per element) over the stage's kernel time, with
               the two-launch implementation's bytes and the counter-measured bytes beside;
  legs         the same measurements on the 64^3 p = 3 deformation workload, the
               128^2 p = 4 single-vortex workload (cache-resident) and the single vortex
               on 1024^2 split-Cartesian cells of triangles (p = 4, 2.1 M elements; dense
               per-element operators), and the adjoint workload (64^2 p = 3, checkpoints
               every 32 of 512 steps);
  cpu_baseline the FP64 oracle on the host cores on an 8^3 sub-mesh of the same kind
               (the full mesh does not fit a bounded CPU run).
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
WORD = {"fp64": 8, "fp32": 4, "bf16": 4}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sync():
    import torch
    torch.cuda.synchronize()


def stage_words(d, p, element="tensor", lifted=False, tables=False):
    """Words per element of one RK stage.

    alg:  5 V N_u + 2 V N_f (read the stage input and u_n, read and write the accumulator,
          write the next stage input; write and read the face traces and common fluxes);
    impl: what the two launches of a stage read and write, each array once, averaged over
          the four stages (the accumulator is not read on stage 1 nor written on stage 4).
          Tensor elements: grad_flux reads u, the pushed + face traces, geometry and the
          adjacency (2 d int32 per element), and with tables the per-element velocity tables
          (2 values at the n nodes and both ends of each axis), and writes the partial
          divergence P and the common flux of each + face point (one slot); update reads P,
          the fluxes of both faces of each direction (only the - faces when lifted: the line
          kernel has added the + faces' lifting to P), |J|, the adjacency, u_n and the
          accumulator, and writes the accumulator, the next stage input and the - face
          traces pushed to the owners.
    """
    V = 2
    if element == "triangle":
        # every flux point has its own trace and flux slot: grad_flux reads u, the own and
        # the partner's traces, geometry and the slot table (one 4-byte code per point, half
        # a word), writes P and the common flux of the owned half of its points (all of its
        # boundary points); update reads P, the flux of every point (own or partner slot),
        # u_n, the accumulator, geometry and the slot table, writes the accumulator, the
        # next stage input and its own traces
        nu, nf = (p + 1) * (p + 2) // 2, 3 * (p + 1)
        geo = 11
        alg = 5 * V * nu + 2 * V * nf
        gf = V * nu + 2 * V * nf + geo + 0.5 * nf + V * nu + 0.5 * V * nf
        up = (V * nu + V * nf + geo + 0.5 * nf + V * nu + 0.75 * V * nu + 0.75 * V * nu
              + V * nu + V * nf)
        return {"alg": alg, "impl": gf + up, "grad_flux": gf, "update": up}
    n = p + 1
    nu, nfa = n ** d, n ** (d - 1)
    nf = 2 * d * nfa
    npf = d * nfa
    geo = d + 2 * d * d + 1
    adj = d                                   # 2 d int32 neighbours per element
    tab = 2 * d * (n + 2) if tables else 0
    alg = 5 * V * nu + 2 * V * nf
    gf = V * nu + V * npf + geo + adj + tab + V * nu + V * npf
    up = (V * nu + (1 if lifted else 2) * V * npf + 1 + adj + V * nu + 0.75 * V * nu
          + 0.75 * V * nu + V * nu + V * npf)
    return {"alg": alg, "impl": gf + up, "grad_flux": gf, "update": up}


def stage_words_of(cfg, form):
    """stage_words for a workload and form: the line kernel (3D; 2D in FP32, and in FP64
    from p = 4; not the BF16 form) lifts the + face fluxes into P; the trigonometric fields
    on the workloads' box meshes (axis-aligned elements) read the per-element velocity
    tables."""
    import workloads as W
    lifted = cfg.element == "tensor" and form != "bf16" and (cfg.ndims == 3 or form == "fp32"
                                                             or cfg.order >= 4)
    tables = cfg.element == "tensor" and cfg.params.vel_kind in (W.VEL_SINGLE_VORTEX, W.VEL_LEVEQUE3D)
    return stage_words(cfg.ndims, cfg.order, cfg.element, lifted, tables)


# dense MFMA peaks of MI355X (TFLOP/s) of the instructions the triangle kernel issues
MFMA_PEAK_TFS = {"fp64": 78.6, "fp32": 157.3}
TRI_MFMA_PER_TILE = 72          # operator products x 4 K-steps per 16-element tile


def tri_mfma_flops(cfg, form):
    """Matrix-core flops of one launch of the triangle MFMA grad_flux (p <= 4, FP64 and
    FP32): 72 instructions of 16 x 16 x 4 (2048 flops each, zero padding included) per
    tile of 16 elements; None where that kernel does not run."""
    if cfg.element != "triangle" or cfg.order > 4 or form not in MFMA_PEAK_TFS:
        return None
    tiles = (cfg.nelem + 15) // 16
    return tiles * TRI_MFMA_PER_TILE * 16 * 16 * 4 * 2


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("pcpf_kernels.hip", "pcpf_kernels_impl.h", "pcpf_internal.h", "pcpf_device.h",
              "pcpf_mfma.h", "pcpf_tri.hip", "pcpf_tri.h"):
        with open(os.path.join(ROOT, "paper_2006_10967_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_solver(cfg, mesh, precision, prm=None):
    from paper_2006_10967_amd import Solver
    if cfg.element == "triangle":
        return Solver.from_triangles(mesh, cfg.order, prm or cfg.params, precision=precision,
                                     device="cuda:0")
    return Solver.from_box(mesh, cfg.order, prm or cfg.params, precision=precision,
                           device="cuda:0")


def initial_state(cfg, mesh):
    import workloads as W
    from paper_2006_10967_amd import DenseMeshArgs, MeshArgs
    if cfg.element == "triangle":
        x = DenseMeshArgs.from_triangles(mesh, cfg.order).solution_coords()
        return W.ic_phi(x, cfg.centre, cfg.radius, cfg.params.eps_w)
    period = [float(mesh.period[k]) if mesh.periodic[k] else 0.0 for k in range(cfg.ndims)]
    x = MeshArgs(cfg.ndims, cfg.order, mesh.x0, mesh.jac, mesh.nbr, period).solution_coords()
    return W.ic_phi(x, cfg.centre, cfg.radius, cfg.params.eps_w)


def run_form(cfg, mesh, phi0_np, precision, K, Wm, acc_steps):
    """One form on one workload: the timed K-step region, a second K-step region with HIP
    events around every launch, the reset + preconditioning alone, and a separate
    acc_steps-step run from the initial state whose final phi is returned (on the device,
    in float64) for the interface comparison."""
    import torch
    s = make_solver(cfg, mesh, precision)
    dt = cfg.dt(mesh)
    phi0 = torch.as_tensor(phi0_np).to("cuda:0", s.dtype)
    # reset + preconditioning (step 0 is on the schedule), then the warm-up steps
    s.set_state(phi0, None, 0.0, 0)
    s.step(dt, 1 + Wm)
    sync()
    t0 = time.perf_counter()
    s.step(dt, K)
    sync()
    wall = time.perf_counter() - t0
    # the next K steps with per-launch events (kernel durations)
    s.kernel_times(reset=True)
    s.set_timing(True)
    sync()
    s.step(dt, K)
    sync()
    s.set_timing(False)
    kt = s.kernel_times(reset=True)
    # the reset + preconditioning alone
    sync()
    t0 = time.perf_counter()
    s.precondition()
    sync()
    pc_ms = (time.perf_counter() - t0) * 1e3
    # accuracy run
    phi_acc = None
    if acc_steps > 0:
        s.set_state(phi0, None, 0.0, 0)
        s.step(dt, acc_steps)
        phi_acc = s.get_state(want_psi=False)[0].double()
    mass_fn = s.mass
    res = {"wall": wall, "kt": kt, "pc_ms": pc_ms}
    return s, res, phi_acc, mass_fn


def load_traffic(workload, precision, hsh):
    """Counter-measured HBM bytes per launch of grad_flux and update on a workload,
    recorded in profiles/traffic_<workload>.json for the kernel sources of hash hsh (else
    None)."""
    try:
        with open(os.path.join(PROFILES, f"traffic_{workload}.json")) as fh:
            data = json.load(fh)
    except OSError:
        return None
    if data.get("kernel_source_hash") != hsh:
        return None
    per = data.get("per_launch_bytes", {})
    if isinstance(per.get(precision), dict):
        per = per[precision]
    elif precision != "fp64":
        return None
    if "grad_flux" not in per or "update" not in per:
        return None
    return {"grad_flux": per["grad_flux"], "update": per["update"],
            "stage": per["grad_flux"] + per["update"]}


def workload_leg(name, forms, K, Wm, acc_steps, hsh):
    """Rates, roofline and interface comparison of the given forms on one workload."""
    import torch
    import workloads as W
    cfg = W.config(name)
    mesh = cfg.mesh()
    phi0 = initial_state(cfg, mesh)
    log(f"[bench] {cfg.name}: E={cfg.nelem} N_u={cfg.nupts} DOF={cfg.dof} K={K} warmup={Wm}")
    out = {"workload": cfg.name, "description": cfg.description, "elements": cfg.nelem,
           "order": cfg.order, "dof": cfg.dof, "dt": cfg.dt(mesh),
           "reset_every": cfg.params.reset_every, "precond_iters": cfg.params.precond_iters,
           "forms": {}}
    ref = None
    for form in forms:
        s, r, phi_acc, _ = run_form(cfg, mesh, phi0, form, K, Wm, acc_steps)
        rate = cfg.dof * 4 * K / r["wall"]
        word = WORD[form]
        gf_ms, gf_n = r["kt"]["grad_flux"]
        up_ms, up_n = r["kt"]["update"]
        gf_us = gf_ms / gf_n * 1e3
        up_us = up_ms / up_n * 1e3
        stage_us = gf_us + up_us
        words = stage_words_of(cfg, form)
        alg = words["alg"] * word * cfg.nelem
        impl = words["impl"] * word * cfg.nelem
        achieved = alg / (stage_us * 1e-6) / 1e9
        traffic = load_traffic(cfg.name, form, hsh)
        f = {"value": rate, "ms_per_step": r["wall"] * 1e3 / K,
             "precondition_ms": r["pc_ms"],
             "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                          "traffic": traffic["stage"] if traffic else None,
                          "kernel": "RK stage: grad_flux + update",
                          "alg_bytes_per_stage": alg, "impl_bytes_per_stage": impl,
                          "stage_us": stage_us},
             "kernels": {"grad_flux": {"avg_us": gf_us, "launches": gf_n,
                                       "impl_bytes": words["grad_flux"] * word * cfg.nelem,
                                       "counter_bytes": traffic["grad_flux"] if traffic else None},
                         "update": {"avg_us": up_us, "launches": up_n,
                                    "impl_bytes": words["update"] * word * cfg.nelem,
                                    "counter_bytes": traffic["update"] if traffic else None}}}
        for k in ("grad_flux", "update"):
            kk = f["kernels"][k]
            kk["impl_GBs"] = kk["impl_bytes"] / (kk["avg_us"] * 1e3)
            if kk["counter_bytes"]:
                kk["counter_GBs"] = kk["counter_bytes"] / (kk["avg_us"] * 1e3)
        if traffic:
            f["roofline"]["traffic_over_alg"] = traffic["stage"] / alg
        mf = tri_mfma_flops(cfg, form)
        if mf:
            tf = mf / (gf_us * 1e-6) / 1e12
            f["mfma"] = {"kernel": "k_tri_grad_flux_mf", "flops_per_launch": mf,
                         "achieved": tf, "peak": MFMA_PEAK_TFS[form], "unit": "TFLOP/s",
                         "frac": tf / MFMA_PEAK_TFS[form]}
        if phi_acc is not None:
            m0 = s.mass(torch.as_tensor(phi0).to("cuda:0", s.dtype))
            if ref is None:
                ref = (s, phi_acc, m0)
                f["after_steps"] = {"steps": acc_steps, "mass_drift": (s.mass(phi_acc.to(s.dtype)) - m0) / m0}
            else:
                s64, phi64, m64 = ref
                l1 = s64.l1(phi64, phi_acc)
                f["after_steps"] = {"steps": acc_steps,
                                    "interface_l1_vs_fp64": l1,
                                    "interface_l1_vs_fp64_rel": l1 / m64,
                                    "mass_drift": (s64.mass(phi_acc) - m64) / m64}
        if ref is not None and form != forms[0]:
            f["speedup_vs_fp64"] = rate / out["forms"][forms[0]]["value"]
        out["forms"][form] = f
        log(f"[bench] {cfg.name} {form}: {f['ms_per_step']:.4f} ms/step, {rate:.4e} DOF-stage/s, "
            f"stage {stage_us:.1f} us (grad_flux {gf_us:.1f} + update {up_us:.1f}), "
            f"{achieved:.0f} GB/s alg ({achieved / HBM_PEAK_GBS:.3f} of HBM), "
            f"reset+precond {r['pc_ms']:.2f} ms"
            + (f", int|phi-phi64| {f['after_steps'].get('interface_l1_vs_fp64', 0):.2e}" if phi_acc is not None else "")
            + (f", MFMA {f['mfma']['achieved']:.1f} TFLOP/s ({f['mfma']['frac']:.3f} of peak)" if "mfma" in f else ""))
        if ref is None or s is not ref[0]:
            del s
        torch.cuda.empty_cache()
    del ref
    torch.cuda.empty_cache()
    return out


def cpu_baseline(name, target_s=12.0):
    """The FP64 CPU oracle (test infrastructure), untuned, on all visible host cores, on a
    bounded sample of the workload: the same kind of mesh, order, field and IC on 8^3
    elements (3D) or the full mesh (2D); one reset + preconditioning (timed, not in the
    value), then as many RK4 steps as fit about target_s seconds."""
    import torch
    import workloads as W
    from dataclasses import replace
    from oracle import Oracle
    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    cfg = W.config(name)
    if cfg.ndims == 3:
        n = 8
        h = 1.0 / n
        prm = W.default_params(3, cfg.order, h, vel_kind=cfg.params.vel_kind,
                               vel_period=cfg.params.vel_period)
        cfg = replace(cfg, n=n, params=prm)
    mesh = cfg.mesh()
    o = Oracle(cfg.ndims, cfg.order, mesh, cfg.params)
    phi = torch.as_tensor(cfg.initial_phi(o.coords()), dtype=torch.float64)
    t0 = time.perf_counter()
    psi, _ = o.precondition(phi)
    t_pc = time.perf_counter() - t0
    dt = cfg.dt(mesh)
    t0 = time.perf_counter()
    phi, psi = o.step(phi, psi, 0.0, dt)
    t1 = time.perf_counter() - t0
    nsteps = max(1, min(500, int(target_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    t = dt
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
    mesh_s = f"{cfg.n}^3" if cfg.ndims == 3 else f"{cfg.n}x{cfg.n}"
    return {"value": rate, "unit": UNIT, "cores": torch.get_num_threads(), "kind": "oracle",
            "cpu": cpu,
            "sample": f"{mesh_s} p={cfg.order} mesh ({cfg.dof} DOF) of the workload's kind "
                      f"(same order, field, IC{', plane perturbation' if cfg.perturb else ''}): "
                      f"{nsteps} RK4 steps ({t_steps:.1f} s) after one reset + "
                      f"{cfg.params.precond_iters} pseudo iterations ({t_pc:.1f} s, not in "
                      f"value)",
            "s_per_step": t_steps / nsteps}


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


def full_period_leg(name, forms, chunk=2000):
    """A workload run to t = T (the LeVeque field's period, where the interface is back at
    its start) in the FP64 form and the given reduced forms, the equal-interface-error
    protocol at t = T: E_L1 = int|phi(T) - phi(0)| of each form, E_m, and int|phi - phi_64|,
    "equal" when |E_L1 - E_L1,64| <= 0.02 E_L1,64 and int|phi - phi_64| <= 0.1 E_L1,64. The
    steps run in chunks with a progress line per chunk."""
    import torch
    import workloads as W
    cfg = W.config(name)
    mesh = cfg.mesh()
    dt = cfg.dt(mesh)
    nsteps = int(round(cfg.params.vel_period / dt))
    phi0_np = initial_state(cfg, mesh)
    out = {"workload": cfg.name, "t_end": nsteps * dt, "steps": nsteps}
    ref = None
    for form in forms:
        s = make_solver(cfg, mesh, form)
        phi0 = torch.as_tensor(phi0_np).to("cuda:0", s.dtype)
        s.set_state(phi0, None, 0.0, 0)
        sync()
        t0 = time.perf_counter()
        done = 0
        while done < nsteps:
            k = min(chunk, nsteps - done)
            s.step(dt, k)
            done += k
            log(f"[bench] {cfg.name} {form}: {done}/{nsteps} steps, {time.perf_counter() - t0:.0f} s")
        sync()
        wall = time.perf_counter() - t0
        phiT = s.get_state(want_psi=False)[0].double()
        if ref is None:
            m0 = s.mass(phi0)
            e64 = s.l1(phi0, phiT)
            ref = (s, phi0.double(), phiT, e64, m0, wall)
            out[form] = {"E_L1": e64, "E_r": e64 / m0, "E_m": (s.mass(phiT) - m0) / m0,
                         "wall_s": wall}
            log(f"[bench] {cfg.name} to t = T ({form}): E_L1 = {e64:.4e}, E_m = {out[form]['E_m']:.2e}, {wall:.0f} s")
            del phiT
            continue
        s64, p0, phi64, e64, m0, wall64 = ref
        e_l1 = s64.l1(p0, phiT)
        diff = s64.l1(phi64, phiT)
        out[form] = {"E_L1": e_l1, "E_r": e_l1 / m0, "E_m": (s64.mass(phiT) - m0) / m0,
                     "int_abs_diff_vs_fp64": diff, "wall_s": wall,
                     "speedup_vs_fp64": wall64 / wall,
                     "equal_interface_error": bool(abs(e_l1 - e64) <= 0.02 * e64 and diff <= 0.1 * e64)}
        log(f"[bench] {cfg.name} to t = T ({form}): E_L1 = {e_l1:.4e} (fp64 {e64:.4e}), "
            f"int|phi-phi64| = {diff:.2e}, equal: {out[form]['equal_interface_error']}, "
            f"x{out[form]['speedup_vs_fp64']:.2f}")
        del s, phiT
        torch.cuda.empty_cache()
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


def dense_gemm_leg():
    """The operator products of one RK stage in the dense form of §3.1 (M0, D_k, the
    lifting, as dense matrices) on the tensor workloads, run as library GEMMs on the matrix
    cores (torch.matmul / addmm, the reference operators times the values of all elements
    at once, random data of the right shapes): a lower bound for a dense-form stage, which
    would add the pointwise work, the face exchanges and the RK combine. A measurement of
    the design alternative, not the product path."""
    import torch
    out = {}
    for dtype, tag in ((torch.float64, "fp64"), (torch.float32, "fp32")):
        for name, n, p in (("C3", 64, 3), ("C5", 96, 4)):
            d, V, E = 3, 2, n ** 3
            N = p + 1
            NU, NF = N ** d, 2 * d * N ** (d - 1)
            g = torch.Generator(device="cuda").manual_seed(0)

            def rnd(*shape):
                return torch.randn(*shape, device="cuda", dtype=dtype, generator=g)
            M0, Dk, LN = rnd(NF, NU), rnd(NU, NU), rnd(NU, NF)
            u, jf, qd = rnd(NU, V * E), rnd(NF, V * E), rnd(NU, d * V * E)
            out_f = torch.empty(NF, d * V * E, device="cuda", dtype=dtype)
            out_u = torch.empty(NU, V * E, device="cuda", dtype=dtype)
            out_uf = torch.empty(NF, V * E, device="cuda", dtype=dtype)

            def stage():
                torch.matmul(M0, u, out=out_uf)                     # Step 1: traces
                for _ in range(d):                                  # Step 3: gradient
                    torch.matmul(Dk, u, out=out_u)
                    torch.addmm(out_u, LN, jf, out=out_u)
                torch.matmul(M0, qd, out=out_f)                     # Step 3: q at flux points
                torch.matmul(M0, qd, out=out_f)                     # Step 4: normal flux
                for k in range(d):                                  # Step 6: divergence
                    torch.matmul(Dk, qd[:, k * V * E:(k + 1) * V * E], out=out_u)
                torch.addmm(out_u, LN, jf, out=out_u)
            flops = 2 * V * E * (NF * NU + d * (NU * NU + NU * NF) + 2 * d * NF * NU
                                 + d * NU * NU + NU * NF)
            for _ in range(3):
                stage()
            sync()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 10
            e0.record()
            for _ in range(reps):
                stage()
            e1.record()
            sync()
            us = e0.elapsed_time(e1) / reps * 1e3
            out[f"{name}_{tag}"] = {"operator_gemm_us_per_stage": us, "gflop": flops / 1e9,
                                    "tflops": flops / (us * 1e-6) / 1e12}
            log(f"[bench] dense operator GEMMs {name} {tag}: {us:.0f} us per stage, "
                f"{flops / 1e9:.1f} GFLOP at {flops / (us * 1e-6) / 1e12:.1f} TFLOP/s")
            del M0, Dk, LN, u, jf, qd, out_f, out_u, out_uf
            torch.cuda.empty_cache()
    return out


def pseudo_sweep_leg():
    """The single vortex on 128^2 quads, p = 4, to t = T (FP64) with the pseudo-time per
    reset swept: K iterations at the default pseudo step for K = 0, 5, 10, 20, 40, resets
    every 1000 steps; E_L1 = int|phi(T) - phi(0)| of each."""
    import dataclasses
    import torch
    import workloads as W
    cfg = W.config("C2")
    mesh = cfg.mesh()
    dt = cfg.dt(mesh)
    nsteps = int(round(cfg.params.vel_period / dt))
    phi0_np = initial_state(cfg, mesh)
    out = {"workload": cfg.name, "steps": nsteps, "dtau": cfg.params.dtau}
    for K in (0, 5, 10, 20, 40):
        prm = dataclasses.replace(cfg.params, precond_iters=K)
        s = make_solver(cfg, mesh, "fp64", prm)
        phi0 = torch.as_tensor(phi0_np).to("cuda:0", s.dtype)
        s.set_state(phi0)
        s.step(dt, nsteps)
        m0 = s.mass(phi0)
        e = s.l1(phi0)
        out[f"K{K}"] = {"pseudo_time_over_h": K * cfg.params.dtau / cfg.h, "E_L1": e,
                        "E_m": (s.mass() - m0) / m0}
        log(f"[bench] pseudo sweep K={K} (K dtau = {K * cfg.params.dtau / cfg.h:.3f} h): "
            f"E_L1 = {e:.3e}")
        del s
    return out


LEG_MIN_STEPS = {"C3": 50, "C2": 1000, "C1": 200, "C4": 200, "T1": 1000, "T2": 20}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed RK4 steps of the headline workload")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="C5",
                    help="headline workload (C1..C5; default C5, the 96^3 p=4 perturbed mesh)")
    ap.add_argument("--forms", default="fp64,fp32,bf16")
    ap.add_argument("--acc-steps", type=int, default=100,
                    help="steps of the per-form interface comparison run (0: skip)")
    ap.add_argument("--legs", default="C3,C2,T2",
                    help="further workloads measured the same way (comma list, '' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target length of the oracle's timed step loop")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-small-run", action="store_true",
                    help="skip the 16x16 p=3 workload run whole on the oracle and the GPU")
    ap.add_argument("--adj-steps", type=int, default=512)
    ap.add_argument("--accuracy", action="store_true",
                    help="the 128^2 p=4 vortex to t = T: E_L1 of the method's variants and "
                         "the equal-interface-error protocol of the FP32 and BF16 forms")
    ap.add_argument("--rotation", action="store_true",
                    help="the slotted-disc rotation tests (Zalesak, Rudman; one turn each)")
    ap.add_argument("--deformation", action="store_true",
                    help="the 64^3 p=3 LeVeque test to t = T (about a minute)")
    ap.add_argument("--vortex-table", action="store_true",
                    help="the single vortex to t = T on 32^2..128^2, p = 2..5")
    ap.add_argument("--leveque-table", action="store_true",
                    help="the 3D deformation to t = T on 32^3, p = 2..5")
    ap.add_argument("--pseudo-sweep", action="store_true",
                    help="the 128^2 p=4 vortex to t = T with K = 0..40 pseudo iterations")
    ap.add_argument("--dense-gemm", action="store_true",
                    help="one stage's operator products in the dense form, as library GEMMs")
    ap.add_argument("--full-period", default="",
                    help="run this workload to t = T in the forms of --full-forms (FP64 first)")
    ap.add_argument("--full-forms", default="fp64,fp32")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W

    if args.copy_mb > 0:
        # a plain copy of known size: reads and writes copy_mb MiB once each
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        sync()
        dst.copy_(src)
        sync()
        del src, dst

    forms = [f for f in args.forms.split(",") if f]
    if forms[0] != "fp64":
        raise SystemExit("the first form must be fp64 (the reference of the comparison)")
    K, Wm = args.steps, args.warmup
    hsh = kernel_source_hash()
    head = workload_leg(args.workload, forms, K, Wm, args.acc_steps, hsh)
    f64 = head["forms"]["fp64"]
    cfg = W.config(args.workload)
    out = {
        "metric": METRIC, "value": f64["value"], "unit": UNIT, "n_gpus": 1, "steps": K,
        "warmup": Wm, "ms_per_step": f64["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": head["workload"], "description": head["description"],
                   "elements": head["elements"], "order": head["order"], "dof": head["dof"],
                   "dt": head["dt"], "reset_every": head["reset_every"],
                   "precond_iters": head["precond_iters"],
                   "timed_region": f"{K} RK4 steps after the step-0 reset + preconditioning "
                                   f"and {Wm} warm-up steps"},
        "roofline": f64["roofline"],
        "kernels_fp64": f64["kernels"],
        "precondition_ms_fp64": f64["precondition_ms"],
        "forms": {k: v for k, v in head["forms"].items() if k != "fp64"},
        "fp64_after_steps": f64.get("after_steps"),
        "kernel_source_hash": hsh,
    }
    legs = [x for x in args.legs.split(",") if x and x != args.workload]
    if legs:
        out["legs"] = {}
    for name in legs:
        kl = max(K, LEG_MIN_STEPS.get(name, K))
        lf = forms if W.config(name).ndims == 3 else [f for f in forms if f != "bf16"]
        out["legs"][name] = workload_leg(name, lf, kl, Wm, args.acc_steps, hsh)

    if not args.no_adjoint:
        adj = {}
        for prec in ("fp64", "fp32"):
            adj[prec] = adjoint_leg(prec, args.adj_steps, 32)
            log(f"[bench] adjoint {prec}: {adj[prec]['s_per_step'] * 1e3:.3f} ms/step "
                f"(forward+reverse), dL/dA = {adj[prec]['dL_dA']:.6e}")
        adj["fp32"]["dL_dA_rel_vs_fp64"] = abs(adj["fp32"]["dL_dA"] - adj["fp64"]["dL_dA"]) \
            / abs(adj["fp64"]["dL_dA"])
        out["adjoint"] = {"workload": "adjoint2d_64x64_p3", **adj}

    if args.accuracy:
        c2 = W.config("C2")
        m2 = c2.mesh()
        out["accuracy"] = accuracy_leg(c2, m2, initial_state(c2, m2))
    if args.rotation:
        out["rotation"] = rotation_leg()
    if args.deformation:
        out["deformation"] = deformation_leg()
    if args.vortex_table:
        out["vortex_table"] = vortex_table_leg()
    if args.leveque_table:
        out["leveque_table"] = leveque_table_leg()
    if args.pseudo_sweep:
        out["pseudo_sweep"] = pseudo_sweep_leg()
    if args.dense_gemm:
        out["dense_gemm"] = dense_gemm_leg()
    if args.full_period:
        ff = [f for f in args.full_forms.split(",") if f]
        if not ff or ff[0] != "fp64":
            sys.exit("--full-forms must start with fp64 (the reference of the comparison)")
        out["full_period"] = full_period_leg(args.full_period, ff)

    if not args.no_small_run:
        out["small_workload_full_run"] = small_workload_run()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
        log(f"[bench] oracle: {out['cpu_baseline']['value']:.4e} DOF-stage/s on "
            f"{out['cpu_baseline']['cores']} cores ({out['cpu_baseline']['sample']})")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
