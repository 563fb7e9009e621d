#!/usr/bin/env python3
"""Throughput benchmark of the DGFEM S_n sweep hot path on one MI355X.

Workload (default): blocky_scatter -- unit cube, 64^3 hexahedra, S8 (80
directions), 8 groups, 8x8x8 random material blocks (sigma_t lognormal
clipped to [0.1, 50], scattering ratio U[0, 0.9]), q = 1, vacuum; FP32
Gaussian-elimination local solver.  One step = one source iteration: source
build, one full sweep (all hyperplanes, octants, directions, groups), octant
reduction and the FP64 residual.  value = cell*direction*group solves per
second over the timed steps.

Also reported: the roofline of the dominant kernel (the sweep kernel chosen
by the autotuner -- one dataflow launch per sweep or one launch per tile
hyperplane -- HBM-bound by its algorithmic bytes), timed with HIP events
around every sweep launch, and the FP64 CPU oracle on a bounded sample of the
same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# vector issue of MI355X: 256 CUs x 4 SIMDs, 2.4 GHz peak clock; a wave64
# VALU instruction holds its SIMD for 4 cycles at the non-packed FP32 rate
# (16 lanes per cycle: 78.6 TFLOP/s of FMA), so the chip issues at most
# 1024 * 2.4e9 / 4 = 614.4 G wave instructions per second
SIMDS = 1024
CLOCK_HZ = 2.4e9
VALU_CYCLES_PER_INST = 4
ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_PROFILES = {
    # dominant kernel -> committed rocprofv3 memory-counter summary
    ("dataflow", 2): "profiles/sweep_flow_ge_f32_tile2_blocky_scatter_64cube_S8_G8_hbm_traffic.txt",
}
SQ_PROFILES = {
    # dominant kernel -> committed rocprofv3 SQ-counter summary
    ("dataflow", 2): "profiles/sweep_flow_ge_f32_tile2_blocky_scatter_64cube_S8_G8_sq.txt",
}


def kernel_source_digest():
    """Digest of the HIP sources; a traffic profile applies only to the kernel
    it was measured on."""
    d = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1906_04017_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp", ".cpp", ".h")):
            d.update(name.encode())
            with open(os.path.join(csrc, name), "rb") as f:
                d.update(f.read())
    return d.hexdigest()[:16]


def profile_value(table, key, sched, tile, workload):
    """A figure of the dominant kernel from its committed rocprofv3 summary,
    or None if there is none for this kernel and workload or the kernel
    sources changed since the counters were taken."""
    rel = table.get((sched, tile))
    if rel is None or workload != "blocky_scatter_64^3_S8_G8":
        return None
    path = os.path.join(ROOT, rel)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_digest") != kernel_source_digest() or key not in kv:
        return None
    return float(kv[key])


def measured_traffic(sched, tile, workload):
    """HBM bytes per launch of the dominant kernel (FETCH_SIZE and WRITE_SIZE
    scaled by a copy of known size)."""
    return profile_value(TRAFFIC_PROFILES, "traffic_bytes_per_launch", sched, tile, workload)


def other_bounds(st, sched, tile, workload, groups, cells, kernel_ms):
    """The bounds beside the algorithmic-byte roofline: the compulsory bytes
    (each cell's sigma_t, 8 sources and 8 fluxes per group once, fronts never
    leaving the chip), the measured DRAM bytes, and the vector-issue bound
    from the SQ counters (VALU wave instructions x 4 cycles over 1024 SIMDs
    at 2.4 GHz)."""
    real = st["algo_bytes_per_sweep"] / (24.0 * st["solves_per_sweep"] + 17.0 * cells * groups)
    comp = real * 17.0 * cells * groups
    sec = kernel_ms * 1e-3
    out = {"compulsory": {"bytes_per_sweep": comp,
                          "achieved_gbs": round(comp / sec / 1e9, 1),
                          "frac": round(comp / sec / 1e9 / HBM_PEAK_GBS, 4)}}
    traffic = measured_traffic(sched, tile, workload)
    out["dram_measured"] = None if traffic is None else {
        "bytes_per_sweep": traffic, "achieved_gbs": round(traffic / sec / 1e9, 1),
        "frac": round(traffic / sec / 1e9 / HBM_PEAK_GBS, 4)}
    insts = profile_value(SQ_PROFILES, "valu_insts_per_launch", sched, tile, workload)
    if insts is None:
        out["valu"] = None
    else:
        min_s = insts * VALU_CYCLES_PER_INST / (SIMDS * CLOCK_HZ)
        out["valu"] = {"bound": "alu", "valu_insts_per_sweep": insts,
                       "issue_peak_insts_per_s": SIMDS * CLOCK_HZ / VALU_CYCLES_PER_INST,
                       "min_ms": round(min_s * 1e3, 4), "frac": round(min_s / sec, 4)}
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--groups", type=int, default=8)
    ap.add_argument("--order", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (memory-counter scale)")
    ap.add_argument("--skip-extras", action="store_true",
                    help="skip the FP64 and the ANN-vs-GE side measurements")
    ap.add_argument("--ann", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "paper_1906_04017_amd", "data",
                                                  "ann_s8_relu64.dgsnann"))
    ap.add_argument("--ann-paper", default=os.path.join(
        os.path.dirname(os.path.abspath(__file__)), "paper_1906_04017_amd", "data",
        "ann_paper_tanh8.dgsnann"), help="paper-form per-octant network (version-2 artifact)")
    ap.add_argument("--per-direction-only", action="store_true",
                    help="only the per-direction paper-form networks on Problems 1-4 at 100^3 "
                         "and 128^3 S8 against GE")
    ap.add_argument("--paper-tables", action="store_true",
                    help="only reproduce the paper's Problem 1-4 grids (S2-S8 at 100^3, "
                         "10^3-100^3 at S8) with every local solver; prints one JSON line")
    ap.add_argument("--ann-only", action="store_true",
                    help="only run --steps sweeps of the BF16-MFMA network on the paper problems "
                         "(128^3, S8, 4 groups) after autotuning: the workload of the matrix-core "
                         "counter passes")
    ap.add_argument("--paper-solver", default="ann", choices=("ann", "ann_paper", "ge"),
                    help="local solver of --ann-only: the BF16-MFMA network (default), the "
                         "paper-form network or FP32 GE, for counters on the same workload")
    ap.add_argument("--aniso-only", action="store_true",
                    help="only time source iterations of the workload with P_L scattering, "
                         "in-group and with group-to-group matrices (P0, P1, P3): the workload "
                         "of the anisotropic kernel trace; prints one JSON line")
    ap.add_argument("--cpu-groups", type=int, default=8,
                    help="groups of the workload swept by the CPU oracle sample")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_calibration(mib):
    """Plain device copy of a known size, for scaling memory counters."""
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {mib} MiB (read {mib} MiB + write {mib} MiB each)")


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(groups, then directions, then KBA slabs would shard across GPUs)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1906_04017_amd import api, inputs

    if args.ann_only:
        ctx = api.Context(0)
        path = {"ann": args.ann, "ann_paper": args.ann_paper, "ge": None}[args.paper_solver]
        print(json.dumps(ann_sweeps(api, ctx, path, args.steps)), flush=True)
        return
    if args.paper_tables:
        ctx = api.Context(0)
        print(json.dumps(paper_tables(api, ctx, args.ann, args.ann_paper)), flush=True)
        return
    if args.per_direction_only:
        ctx = api.Context(0)
        rows = []
        for n in (100, 128):
            row = {"cells": f"{n}^3", "order": "S8"}
            row.update(per_direction_leg(api, ctx, n, None, None, 3))
            log(f"per-direction networks {n}^3 S8: " + json.dumps(row))
            rows.append(row)
        print(json.dumps({"table": "per_direction_networks", "rows": rows}), flush=True)
        return

    p = inputs.blocky_scatter(n=args.n, groups=args.groups, seed=2, order=args.order)
    log(f"workload {p['name']}")
    if args.aniso_only:
        ctx = api.Context(0)
        print(json.dumps(anisotropic_steps(api, ctx, p)), flush=True)
        return
    ctx = api.Context(0)
    om, w = api.quadrature_ls(p["order"])
    prob = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision="fp32")
    prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
    prob.set_inflow(p["psi_inc"])
    tile, sched, times = prob.autotune()
    log(f"autotune: tile {tile}, {sched} schedule (one sweep: " +
        ", ".join(f"{s} {b}^3 {m:.3f} ms" for (s, b), m in times.items()) + ")")
    st = prob.stats()
    solves = st["solves_per_sweep"]
    phi = torch.zeros((p["groups"], prob.ncell, 8), dtype=torch.float32, device="cuda")

    # the steps run as one source iteration of exactly K iterations (the
    # library overlaps each iteration's sweep with the previous residual
    # readback); warmup likewise
    prob.set_si_criterion("fixed")
    if args.warmup:
        phi, _ = prob.source_iterate(phi0=phi, tol=0.0, max_iter=args.warmup)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    prob.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, info = prob.source_iterate(phi0=phi, tol=0.0, max_iter=args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, kern_launches = prob.kernel_time()
    prob.set_timing(False)
    resid = info["resid"]
    assert info["iters"] == args.steps
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    value = solves * args.steps / wall
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, residual {resid:.3e}")

    # roofline of the sweep kernel: algorithmic bytes of one sweep over the
    # summed duration of that sweep's kernel launches
    sweep_kernel_ms = kern_ms / args.steps
    achieved = st["algo_bytes_per_sweep"] / (sweep_kernel_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(sched, tile, p["name"]),
            "kernel": (f"sweep_flow_ge<float, mass-inverse GE, {tile}x{tile}x{tile} tiles> "
                       "(one dataflow launch per sweep)" if sched == "dataflow" else
                       f"sweep_tile_ge<float, mass-inverse GE, {tile}x{tile}x{tile} tiles> "
                       "(one launch per tile hyperplane)"),
            "launches_per_sweep": kern_launches // args.steps,
            "kernel_ms_per_sweep": round(sweep_kernel_ms, 4),
            "avg_launch_us": round(1e3 * kern_ms / max(kern_launches, 1), 3),
            "algo_bytes_per_sweep": st["algo_bytes_per_sweep"]}
    roof["other_bounds"] = other_bounds(st, sched, tile, p["name"], p["groups"], prob.ncell,
                                        sweep_kernel_ms)

    fp64 = None if args.skip_extras else plain_fp64(api, ctx, p)
    conv = None if args.skip_extras else si_convergence(api, ctx, p)
    ann = None if args.skip_extras else ann_vs_ge(api, ctx, args.ann, args.ann_paper)
    adj = None if args.skip_extras else adjoint_box(api, ctx)
    aniso = None if args.skip_extras else anisotropic_steps(api, ctx, p)
    batch = None if args.skip_extras else uneven_batch(api, ctx, args.ann)

    cpu = err = None
    if not args.no_cpu_baseline:
        cpu, refs = cpu_baseline(p, args.cpu_groups)
        err = error_vs_oracle(api, ctx, prob, p, refs, args.cpu_groups)

    out = {
        "metric": "cell*dir*group solves/s (FP32 GE sweep, one source iteration per step)",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": p["name"], "cells": prob.ncell, "directions": prob.n_dirs,
                   "groups": p["groups"], "solver": "GE", "precision": "fp32",
                   "solves_per_step": solves, "last_residual": resid},
        "roofline": roof,
        "cpu_baseline": cpu,
        "error_vs_fp64_oracle": err,
        "fp64_ge": fp64,
        "si_convergence": conv,
        "ann_vs_ge": ann,
        "adjoint": adj,
        "anisotropic": aniso,
        "batch": batch,
    }
    print(json.dumps(out), flush=True)


def time_sweeps(prob, src, reps):
    import torch
    phi = prob.nodal_empty()
    prob.sweep(src, phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        prob.sweep(src, phi)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, phi


def plain_fp64(api, ctx, p, reps=10):
    """Plain (FP64) GE sweep throughput on the same workload, autotuned."""
    import torch
    om, w = api.quadrature_ls(p["order"])
    prob = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision="fp64")
    prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
    tile, sched, tune = prob.autotune()
    src = torch.tensor(np.repeat(p["q"][..., None], 8, axis=-1), dtype=torch.float64,
                       device="cuda")
    dt, _ = time_sweeps(prob, src, reps)
    solves = prob.stats()["solves_per_sweep"]
    log(f"fp64 GE sweep: {dt * 1e3:.3f} ms (tile {tile}, {sched} schedule; autotuner "
        + ", ".join(f"{k[0]} {k[1]}^3 {v:.3f} ms" for k, v in tune.items()) + ")")
    prob.close()
    return {"solves_per_s": solves / dt, "ms_per_sweep": dt * 1e3, "solver": "GE", "dtype": "f64",
            "tile": tile, "schedule": sched}


def si_convergence(api, ctx, p, tol=1e-8):
    """Source iteration of the benchmark workload to a 1e-8 max-norm
    residual with the plain FP64 GE, and with FP32 GE until its own floor:
    iterations, residuals, wall time, and the FP32 solution's norm-wise
    relative difference from the FP64 one per group."""
    import torch
    om, w = api.quadrature_ls(p["order"])
    out = {"workload": p["name"], "tol": tol}
    res = {}
    for prec in ("fp64", "fp32"):
        prob = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision=prec)
        prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
        prob.set_inflow(p["psi_inc"])
        prob.autotune()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi, info = prob.source_iterate(tol=tol, max_iter=2000, allow_notconv=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r, _ = prob.si_history()
        out[prec] = {"iterations": info["iters"], "residual": info["resid"],
                     "converged": info["converged"], "seconds": dt,
                     "rho_eff": api.spectral_radius(r)}
        res[prec] = phi.double()
        log(f"SI {prec}: {info['iters']} iterations to residual {info['resid']:.2e} "
            f"in {dt:.2f} s")
        prob.close()
    d = (res["fp32"] - res["fp64"]).abs().amax(dim=(1, 2)) / res["fp64"].abs().amax(dim=(1, 2))
    out["fp32_vs_fp64_rel_per_group"] = [float(v) for v in d.cpu()]
    log(f"SI fp32 vs fp64: max relative difference {float(d.max()):.2e}")
    return out


def ann_vs_ge(api, ctx, ann_path, pann_path, n=128, reps=3):
    """The paper's comparison on its four problems (one group each, 10 cm
    cube, psi_inc = 1 on three faces), 128^3, S8: one sweep of all groups with
    the FP32 GE solvers, with the BF16-MFMA ANN and with the paper-form
    per-octant network (vector ALUs), and each network's error eps_P
    (cell-average mean relative difference) against GE per group; group 4
    (c = 0.99) by source iteration to the paper's eps_S < 1e-4."""
    import torch
    from paper_1906_04017_amd import inputs
    p = inputs.paper_problems(n=n, groups=4, order=8)
    om, w = api.quadrature_ls(8)
    nets = {"ann": api.Ann(ctx, ann_path)}
    nets["ann_x2"] = api.Ann(ctx, ann_path)   # split-BF16 activations
    nets["ann_x2"].set_mode("bf16x2")
    if pann_path and os.path.exists(pann_path):
        nets["ann_paper"] = api.Ann(ctx, pann_path)
    S = torch.tensor(np.repeat(p["q"][..., None], 8, axis=-1), dtype=torch.float32, device="cuda")
    out = {"workload": p["name"], "ann_artifact": os.path.basename(ann_path),
           "ann_paper_artifact": os.path.basename(pann_path) if "ann_paper" in nets else None}
    res = {}
    for solver in ("ge", "ge_dense") + tuple(nets):
        prob = api.Problem(ctx, p["n"], p["length"], 4, om, w, precision="fp32",
                           solver="ann" if solver in nets else solver)
        prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
        prob.set_inflow(p["psi_inc"])
        if solver in nets:
            prob.set_ann(nets[solver])
        tile, sched, _ = prob.autotune()
        out[f"{solver}_schedule"] = f"{sched}, {tile}^3 tiles"
        dt, phi = time_sweeps(prob, S, reps)
        solves = prob.stats()["solves_per_sweep"]
        out[f"{solver}_solves_per_s"] = solves / dt
        out[f"{solver}_ms_per_sweep"] = dt * 1e3
        if solver == "ann":
            # the BF16 network's matrix-core rate by the method's 4096 flops
            # per solve (2 * (24 * 64 + 64 * 8)); the kernel issues 8192 after
            # padding K 24 -> 32 and the output rows 8 -> 32
            tf = 4096 * solves / dt / 1e12
            out["ann_mfma_roofline"] = {"bound": "mfma", "achieved": round(tf, 2),
                                        "peak": 2500.0, "unit": "TFLOP/s",
                                        "frac": round(tf / 2500.0, 5), "flops_per_solve": 4096,
                                        "issued_flops_per_solve": 8192}
        res[solver] = phi.double().mean(-1)        # cell averages [G, ncell]
        log(f"paper problems {solver}: {dt * 1e3:.3f} ms per sweep")
        prob.close()
    ref = res["ge"]
    for net in nets:
        out[f"{net}_over_ge_speed"] = out[f"{net}_solves_per_s"] / out["ge_solves_per_s"]
        out[f"{net}_over_ge_dense_speed"] = (out[f"{net}_solves_per_s"] /
                                             out["ge_dense_solves_per_s"])
        eps = ((res[net] - ref).abs() / (ref.abs() + 1e-8)).mean(-1).cpu().numpy()
        out[f"{net}_eps_p_percent_single_sweep"] = [round(100 * float(v), 3) for v in eps]
    # group 4: scattering, converged by SI with each solver (paper criterion)
    p4 = inputs.problem(p["n"], p["length"], 8, 1, p["sigma_t"][3:4], p["sigma_s"][3:4],
                        p["q"][3:4], p["psi_inc"], "problem4")
    si = {}
    for solver in ("ge",) + tuple(nets):
        prob = api.Problem(ctx, p4["n"], p4["length"], 1, om, w, precision="fp32",
                           solver="ann" if solver in nets else solver)
        prob.set_materials(p4["sigma_t"], p4["sigma_s"], p4["q"])
        prob.set_inflow(p4["psi_inc"])
        if solver in nets:
            prob.set_ann(nets[solver])
        prob.set_si_criterion("eps_s")
        phi, info = prob.source_iterate(tol=1e-4, max_iter=2000, allow_notconv=True)
        info["rho_eff"] = api.spectral_radius(prob.si_history()[0])
        si[solver] = (phi.double().mean(-1), info)
        log(f"problem 4 SI {solver}: {info['iters']} iterations, eps_S {info['eps_s']:.2e}")
        prob.close()
    for net in nets:
        e4 = ((si[net][0] - si["ge"][0]).abs() / (si["ge"][0].abs() + 1e-8)).mean().item()
        out[f"{net}_eps_p_percent_problem4_si"] = round(100 * e4, 3)
    out["problem4_si_iterations"] = {k: v[1]["iters"] for k, v in si.items()}
    out["problem4_rho_eff"] = {k: v[1]["rho_eff"] for k, v in si.items()}
    out["paper_context"] = ("paper, 100^3 S8, unstated hardware: ANN saves 68.4 % of the solve time "
                            "(3.16x); eps_P 1.59 / 2.45 / 0.45 / 0.87 % on Problems 1-4; SI "
                            "iterations GE / ANN 237 / 110 on Problem 4")
    for a in nets.values():
        a.close()
    return out


def ann_sweeps(api, ctx, ann_path, reps, n=128):
    """Sweeps of the paper problems (128^3, S8, 4 groups) with one local
    solver alone (a network artifact, or GE when ann_path is None), for the
    counters: the BF16 network's two layers issue 2 * 32 * 32 * 16 * 8 = 8192
    MFMA flops per solve (K padded 24 -> 32, the output rows 8 -> 32) for the
    method's 2 * (24 * 64 + 64 * 8) = 4096."""
    import torch
    from paper_1906_04017_amd import inputs
    p = inputs.paper_problems(n=n, groups=4, order=8)
    om, w = api.quadrature_ls(8)
    ann = api.Ann(ctx, ann_path) if ann_path else None
    prob = api.Problem(ctx, p["n"], p["length"], 4, om, w, precision="fp32",
                       solver="ann" if ann else "ge")
    prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
    prob.set_inflow(p["psi_inc"])
    if ann:
        prob.set_ann(ann)
    tile, sched, _ = prob.autotune()
    S = torch.tensor(np.repeat(p["q"][..., None], 8, axis=-1), dtype=torch.float32, device="cuda")
    dt, _ = time_sweeps(prob, S, reps)
    solves = prob.stats()["solves_per_sweep"]
    log(f"paper problems, one solver: {sched} schedule, {tile}^3 tiles, {dt * 1e3:.3f} ms per "
        "sweep")
    out = {"workload": p["name"], "solver": os.path.basename(ann_path) if ann else "GE",
           "schedule": sched, "tile": tile, "sweeps": reps + 1, "ms_per_sweep": dt * 1e3,
           "solves_per_sweep": solves, "method_flops_per_sweep": 4096 * solves,
           "method_tflops": 4096 * solves / dt / 1e12}
    prob.close()
    if ann:
        ann.close()
    return out


def paper_tables(api, ctx, ann_path, pann_path, reps=3):
    """The paper's evaluation grid (Sec. 4): Problems 1-4 in the 10 cm cube
    with psi_inc = 1 on the x = 0, y = 0 and z = 0 faces, at 100^3 cells with
    S2, S4, S6, S8 and at 10^3, 25^3, 50^3, 100^3 cells with S8.  For every
    configuration and local solver (FP32 GE, the BF16-MFMA network, the
    paper-form network): the time of one sweep of Problems 1-3 (no scattering,
    one sweep is the solution) and eps_P of each network against GE; for
    Problem 4 (c = 0.99) the source iterations to eps_S < 1e-4 and eps_P of the
    converged flux."""
    import torch
    from paper_1906_04017_amd import inputs
    nets = {"ann": api.Ann(ctx, ann_path)}
    # the same network with split-BF16 activations: its result is the
    # network's own to about 2^-16 (the parity tests bound its distance from
    # the FP64 forward of the artifact), so its eps_P is the network's
    # (training) error and the BF16 column's excess over it is rounding
    nets["ann_x2"] = api.Ann(ctx, ann_path)
    nets["ann_x2"].set_mode("bf16x2")
    if pann_path and os.path.exists(pann_path):
        nets["ann_paper"] = api.Ann(ctx, pann_path)
    solvers = ("ge",) + tuple(nets)
    configs = [(100, 2), (100, 4), (100, 6), (100, 8), (10, 8), (25, 8), (50, 8)]
    rows = []
    for n, order in configs:
        p = inputs.paper_problems(n=n, groups=4, order=order)
        om, w = api.quadrature_ls(order)
        S = torch.tensor(np.repeat(p["q"][..., None], 8, axis=-1), dtype=torch.float32,
                         device="cuda")
        row = {"cells": f"{n}^3", "order": f"S{order}", "directions": len(w)}
        avg = {}
        for sv in solvers:
            prob = api.Problem(ctx, p["n"], p["length"], 3, om, w, precision="fp32",
                               solver="ann" if sv in nets else "ge")
            prob.set_materials(p["sigma_t"][:3], p["sigma_s"][:3], p["q"][:3])
            prob.set_inflow(p["psi_inc"])
            if sv in nets:
                prob.set_ann(nets[sv])
            prob.autotune()
            dt, phi = time_sweeps(prob, S[:3], reps)
            row[f"{sv}_ms_per_sweep_p123"] = round(dt * 1e3, 4)
            avg[sv] = phi.double().mean(-1)
            prob.close()
        for sv in nets:
            eps = ((avg[sv] - avg["ge"]).abs() / (avg["ge"].abs() + 1e-8)).mean(-1).cpu().numpy()
            row[f"{sv}_eps_p_percent_p123"] = [round(100 * float(v), 3) for v in eps]
        p4 = inputs.problem(p["n"], p["length"], order, 1, p["sigma_t"][3:4], p["sigma_s"][3:4],
                            p["q"][3:4], p["psi_inc"], "problem4")
        si = {}
        for sv in solvers:
            prob = api.Problem(ctx, p4["n"], p4["length"], 1, om, w, precision="fp32",
                               solver="ann" if sv in nets else "ge")
            prob.set_materials(p4["sigma_t"], p4["sigma_s"], p4["q"])
            prob.set_inflow(p4["psi_inc"])
            if sv in nets:
                prob.set_ann(nets[sv])
            prob.autotune()
            prob.set_si_criterion("eps_s")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            phi, info = prob.source_iterate(tol=1e-4, max_iter=3000, allow_notconv=True)
            torch.cuda.synchronize()
            si[sv] = (phi.double().mean(-1), info, time.perf_counter() - t0)
            info["rho_eff"] = api.spectral_radius(prob.si_history()[0])
            prob.close()
        row["p4_si_iterations"] = {sv: si[sv][1]["iters"] for sv in solvers}
        row["p4_si_ms"] = {sv: round(1e3 * si[sv][2], 2) for sv in solvers}
        row["p4_rho_eff"] = {sv: (None if si[sv][1]["rho_eff"] is None else
                                  round(si[sv][1]["rho_eff"], 4)) for sv in solvers}
        # the paper's overall acceleration: time of the GE solution over the
        # network's (sweep speed and iteration count together)
        row["p4_overall_acceleration"] = {sv: round(si["ge"][2] / si[sv][2], 3) for sv in nets}
        for sv in nets:
            e4 = ((si[sv][0] - si["ge"][0]).abs() / (si["ge"][0].abs() + 1e-8)).mean().item()
            row[f"{sv}_eps_p_percent_p4"] = round(100 * e4, 3)
        if order == 8:
            row.update(per_direction_leg(api, ctx, n, avg["ge"], si["ge"][0], reps))
        log(f"paper tables {n}^3 S{order}: " + json.dumps(row))
        rows.append(row)
    # the per-direction networks also at the 128^3 cells of the network benchmark
    row = {"cells": "128^3", "order": "S8", "directions": 80}
    row.update(per_direction_leg(api, ctx, 128, None, None, reps))
    if len(row) > 3:
        log("paper tables 128^3 S8 (per-direction networks): " + json.dumps(row))
        rows.append(row)
    for a in nets.values():
        a.close()
    return {"table": "paper_problems_1_to_4", "rows": rows,
            "ann_artifact": os.path.basename(ann_path),
            "ann_paper_artifact": os.path.basename(pann_path) if "ann_paper" in nets else None,
            "paper_context": ("paper (unstated hardware): eps_P P1 0.11/1.30/1.78/1.59 %, "
                              "P2 0.07/1.09/2.57/2.45 %, P3 0.14/0.86/0.68/0.45 % at 100^3 "
                              "S2-S8; P4 SI iterations GE/ANN 211/101, 220/102, 228/104, "
                              "237/110 at 100^3 S2-S8 and 15/9, 42/20, 121/58 at 10^3, 25^3, "
                              "50^3 S8; effective spectral radius 0.957 (GE) / 0.859 (ANN); "
                              "overall acceleration on Problem 4 about 12")}


def per_direction_artifact(sigma_t, n, length=10.0, ranges=""):
    """Path of the shipped per-direction paper-form networks trained at
    sigma_t and the cell edge length / n (ranges: the suffix of networks
    trained on other inflow / source ranges), or None."""
    s = {10.0: "10", 0.001: "0.001"}.get(float(sigma_t))
    h = {100: "0.1", 128: "0.078125"}.get(int(n)) if length == 10.0 else None
    if s is None or h is None:
        return None
    path = os.path.join(ROOT, "paper_1906_04017_amd", "data",
                        f"ann_paper_dir_s8_sigma{s}_h{h}{ranges}.dgsnann")
    return path if os.path.exists(path) else None


def per_direction_leg(api, ctx, n, ge_avg, ge_p4, reps):
    """The paper-form networks held per quadrature direction, each Problem
    with the artifact trained at its sigma_t and cell size (S8): per Problem
    1-3 the time of one sweep (each Problem its own one-group problem) and
    eps_P against GE; Problem 4 the eps_S source iterations and eps_P of the
    converged flux.  ge_avg / ge_p4: GE cell averages from the caller (None:
    computed here with FP32 GE)."""
    import torch
    from paper_1906_04017_amd import inputs
    p = inputs.paper_problems(n=n, groups=4, order=8)
    paths = [per_direction_artifact(p["sigma_t"][g][0], n) for g in range(3)]
    # Problem 4's converged flux reaches 4 pi q / (sigma_t - sigma_s) = 126
    # (psi up to 10, sources up to 100): its networks are trained on those
    # ranges
    paths.append(per_direction_artifact(p["sigma_t"][3][0], n, ranges="_psi12_s120"))
    if any(x is None for x in paths):
        return {}
    om, w = api.quadrature_ls(8)
    out = {"ann_paper_dir_artifacts": [os.path.basename(x) for x in paths]}
    eps, ms, ms_ge = [], [], []
    for g in range(3):
        sl = slice(g, g + 1)
        S = torch.tensor(np.repeat(p["q"][sl][..., None], 8, axis=-1), dtype=torch.float32,
                         device="cuda")
        res = {}
        for sv in ("ge", "ann") if ge_avg is None else ("ann",):
            prob = api.Problem(ctx, p["n"], p["length"], 1, om, w, precision="fp32", solver=sv)
            prob.set_materials(p["sigma_t"][sl], p["sigma_s"][sl], p["q"][sl])
            prob.set_inflow(p["psi_inc"])
            if sv == "ann":
                ann = api.Ann(ctx, paths[g])
                prob.set_ann(ann)
            prob.autotune()
            dt, phi = time_sweeps(prob, S, reps)
            res[sv] = phi.double().mean(-1)[0]
            if sv == "ann":
                ms.append(round(dt * 1e3, 4))
                ann.close()
            else:
                ms_ge.append(round(dt * 1e3, 4))
            prob.close()
        ge = res["ge"] if ge_avg is None else ge_avg[g]
        eps.append(round(100 * float(((res["ann"] - ge).abs() / (ge.abs() + 1e-8)).mean()), 3))
    out["ann_paper_dir_eps_p_percent_p123"] = eps
    out["ann_paper_dir_ms_per_sweep_p123"] = ms
    if ms_ge:
        out["ge_ms_per_sweep_p123_one_group"] = ms_ge
    g = 3
    sl = slice(g, g + 1)
    res = {}
    for sv in ("ge", "ann") if ge_p4 is None else ("ann",):
        prob = api.Problem(ctx, p["n"], p["length"], 1, om, w, precision="fp32", solver=sv)
        prob.set_materials(p["sigma_t"][sl], p["sigma_s"][sl], p["q"][sl])
        prob.set_inflow(p["psi_inc"])
        if sv == "ann":
            ann = api.Ann(ctx, paths[g])
            prob.set_ann(ann)
        prob.autotune()
        prob.set_si_criterion("eps_s")
        phi, info = prob.source_iterate(tol=1e-4, max_iter=3000, allow_notconv=True)
        res[sv] = (phi.double().mean(-1), info["iters"])
        if sv == "ann":
            ann.close()
        prob.close()
    ge4 = res["ge"][0] if ge_p4 is None else ge_p4
    out["ann_paper_dir_p4_si_iterations"] = res["ann"][1]
    out["ann_paper_dir_eps_p_percent_p4"] = round(
        100 * float(((res["ann"][0] - ge4).abs() / (ge4.abs() + 1e-8)).mean()), 3)
    return out


def anisotropic_steps(api, ctx, p, iters=10):
    """Source iterations of the benchmark workload with P_L scattering, FP32
    GE, ms per iteration: in-group (sigma_{s,n} = (0.5, 0.25, 0.12)_n
    sigma_s) at L = 0, 1, 3, and with a group-to-group matrix per order
    (inputs.multigroup_orders: the same total scattering out of each group,
    spread over in-group, down- and some upscatter) at L = 0 (the P0 matrix
    alone), 1 and 3."""
    import torch
    from paper_1906_04017_amd import inputs
    om, w = api.quadrature_ls(p["order"])
    out = {"workload": p["name"], "iterations": iters}
    cases = [("P0", None), ("P1", None), ("P3", None), ("P0_gg", 0), ("P1_gg", 1), ("P3_gg", 3)]
    for name, gg in cases:
        prob = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision="fp32")
        prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
        prob.set_inflow(p["psi_inc"])
        prob.autotune()
        L = int(name[1])
        if gg is None and L:
            prob.set_anisotropy(inputs.anisotropic_orders(p["sigma_s"], L, seed=7))
        elif gg is not None:
            m = inputs.multigroup_orders(p["sigma_s"], L, seed=8)
            if L:
                prob.set_anisotropy_gg(m)
            else:
                prob.set_scattering(m[0])
            del m
        prob.source_iterate(tol=0.0, max_iter=2, allow_notconv=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob.source_iterate(tol=0.0, max_iter=iters, allow_notconv=True)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / iters
        out[f"{name}_ms_per_iteration"] = ms
        log(f"scattering {name}: {ms:.3f} ms per source iteration")
        prob.close()
    return out


def adjoint_box(api, ctx, n=32, cells=8, h=1e-6):
    """Gradient of the absorption in the central box (cells 12..19 of a 32^3
    cube, S4, 2 groups, c = 0.5) with respect to sigma_t and q through the
    FP32 forward and adjoint source iterations, checked at seeded cells against
    central differences of FP64 forward solves (sigma_s held fixed)."""
    import torch
    from paper_1906_04017_amd import inputs
    p = inputs.adjoint_box(n=n)
    om, w = api.quadrature_ls(p["order"])
    V = np.prod(np.array(p["length"]) / np.array(p["n"]))
    box = torch.tensor(p["box_mask"], device="cuda")

    def response(phi, st, ss):
        # J = sum_g sum_box (sigma_t - sigma_s) int phi, int phi = V/8 sum_nodes
        return (((st - ss) * box)[..., None] * phi).sum() * (V / 8)

    prob = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision="fp32",
                       store_psi=True)
    prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
    tile, sched, _ = prob.autotune()
    st = torch.tensor(p["sigma_t"], dtype=torch.float32, device="cuda", requires_grad=True)
    q = torch.tensor(p["q"], dtype=torch.float32, device="cuda", requires_grad=True)
    ss = torch.tensor(p["sigma_s"], dtype=torch.float32, device="cuda")
    # one untimed forward + adjoint solve first (first-use allocations)
    response(api.TransportSolve.apply(prob, st, q, ss, 1e-7, 500), st, ss).backward()
    st.grad = None
    q.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi = api.TransportSolve.apply(prob, st, q, ss, 1e-7, 500)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J = response(phi, st, ss)
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    gst = st.grad.double().cpu().numpy()
    gq = q.grad.double().cpu().numpy()
    # FP64 forward solves for central differences at seeded cells
    p64 = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision="fp64")
    rng = np.random.default_rng(44)
    sel = [(int(rng.integers(0, p["groups"])), int(rng.integers(0, n ** 3))) for _ in range(cells)]
    sel[0] = (0, int(np.flatnonzero(p["box_mask"])[7]))

    def J64(st_np, q_np):
        p64.set_materials(st_np, p["sigma_s"], q_np)
        ph, _ = p64.source_iterate(tol=1e-13, max_iter=2000)
        stt = torch.tensor(st_np, dtype=torch.float64, device="cuda")
        sst = torch.tensor(p["sigma_s"], dtype=torch.float64, device="cuda")
        return float(response(ph, stt, sst))

    err_t, err_q = [], []
    for g, c in sel:
        e = np.zeros_like(p["sigma_t"])
        e[g, c] = h
        fd_t = (J64(p["sigma_t"] + e, p["q"]) - J64(p["sigma_t"] - e, p["q"])) / (2 * h)
        fd_q = (J64(p["sigma_t"], p["q"] + e) - J64(p["sigma_t"], p["q"] - e)) / (2 * h)
        err_t.append(abs(gst[g, c] - fd_t) / max(abs(fd_t), 1e-300))
        err_q.append(abs(gq[g, c] - fd_q) / max(abs(fd_q), 1e-300))
    log(f"adjoint: forward SI {1e3 * (t1 - t0):.1f} ms, adjoint {1e3 * (t2 - t1):.1f} ms, "
        f"max rel err vs FD: sigma_t {max(err_t):.2e}, q {max(err_q):.2e}")
    prob.close()
    p64.close()
    fd64 = adjoint_fp64_vs_fd(api, ctx, p)
    log("adjoint FP64 vs FD: " + json.dumps(fd64))
    return {"workload": p["name"], "schedule": f"{sched}, {tile}^3 tiles",
            "forward_si_ms": 1e3 * (t1 - t0), "adjoint_ms": 1e3 * (t2 - t1),
            "fd_cells": len(sel), "fd_step": h, "max_rel_err_dsigma_t": max(err_t),
            "max_rel_err_dq": max(err_q), "precision": "fp32 adjoint vs fp64 central differences",
            "fp64_adjoint_vs_fd": fd64}


def adjoint_fp64_vs_fd(api, ctx, p, cells=64, h=1e-5, iters=100):
    """FP64 adjoint gradients of J = <g, phi> (g the box absorption weights
    of the unperturbed materials, held fixed) against central differences of
    FP64 source iterations that all run the same `iters` iterations (c = 0.5:
    converged to rounding), at `cells` seeded cells (half in the response box),
    norm-wise over the cells, and one directional derivative along a random
    relative sigma_t perturbation of every cell."""
    import torch
    om, w = api.quadrature_ls(p["order"])
    G, nc = p["sigma_t"].shape
    V = np.prod(np.array(p["length"]) / np.array(p["n"]))
    g = np.zeros((G, nc, 8))
    g[:, p["box_mask"], :] = ((p["sigma_t"] - p["sigma_s"])[:, p["box_mask"]] * V / 8)[..., None]
    prob = api.Problem(ctx, p["n"], p["length"], G, om, w, precision="fp64", store_psi=True)
    prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
    prob.autotune()
    prob.source_iterate(tol=1e-13, max_iter=2000)
    gst, gq, _ = prob.adjoint(torch.tensor(g, dtype=torch.float64, device="cuda"), tol=1e-13,
                              max_iter=2000)
    gst, gq = gst.cpu().numpy(), gq.cpu().numpy()
    fwd = api.Problem(ctx, p["n"], p["length"], G, om, w, precision="fp64")
    fwd.autotune()

    def J(st, q):
        fwd.set_materials(st, p["sigma_s"], q)
        phi, _ = fwd.source_iterate(tol=0.0, max_iter=iters, allow_notconv=True)
        return float((phi.cpu().numpy() * g).sum())

    rng = np.random.default_rng(47)
    box = np.flatnonzero(p["box_mask"])
    sel = [(int(rng.integers(0, G)), int(rng.choice(box))) for _ in range(cells // 2)]
    sel += [(int(rng.integers(0, G)), int(rng.integers(0, nc))) for _ in range(cells - cells // 2)]
    fd_t, fd_q, ad_t, ad_q = [], [], [], []
    for gg, c in sel:
        e = np.zeros((G, nc))
        e[gg, c] = h
        fd_t.append((J(p["sigma_t"] + e, p["q"]) - J(p["sigma_t"] - e, p["q"])) / (2 * h))
        fd_q.append((J(p["sigma_t"], p["q"] + e) - J(p["sigma_t"], p["q"] - e)) / (2 * h))
        ad_t.append(gst[gg, c])
        ad_q.append(gq[gg, c])
    fd_t, fd_q, ad_t, ad_q = map(np.array, (fd_t, fd_q, ad_t, ad_q))
    v = rng.uniform(-1.0, 1.0, size=(G, nc)) * p["sigma_t"]
    hd = 1e-7
    dd = (J(p["sigma_t"] + hd * v, p["q"]) - J(p["sigma_t"] - hd * v, p["q"])) / (2 * hd)
    prob.close()
    fwd.close()
    return {"cells": len(sel), "fd_step": h, "iterations_per_forward": iters,
            "rel_err_dsigma_t": float(np.abs(ad_t - fd_t).max() / np.abs(fd_t).max()),
            "rel_err_dq": float(np.abs(ad_q - fd_q).max() / np.abs(fd_q).max()),
            "rel_err_directional": float(abs((gst * v).sum() - dd) / abs(dd)),
            "norm": "max over the cells / max |FD| over the cells"}


def uneven_batch(api, ctx, ann_path, count=64):
    """64 independent problems (cubes of 16^3 to 96^3 cells, S4 to S12, 1 to
    8 groups, GE or ANN with probability 1/2, blocky random materials): one
    sweep of every problem in one graph launch; autotuned tiles; p50 / p99
    per-problem latency and aggregate solves per second."""
    import torch
    from paper_1906_04017_amd import inputs
    ps = inputs.uneven_batch(count=count)
    ann = api.Ann(ctx, ann_path)
    probs, srcs, phis = [], [], []
    solves = 0
    for p in ps:
        om, w = api.quadrature_ls(p["order"])
        prob = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision="fp32",
                           solver=p["solver"])
        prob.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
        if p["solver"] == "ann":
            prob.set_ann(ann)
        S = torch.tensor(np.repeat(p["q"][..., None], 8, axis=-1), dtype=torch.float32,
                         device="cuda")
        probs.append(prob)
        srcs.append(S)
        phis.append(torch.empty_like(S))
        solves += prob.stats()["solves_per_sweep"]
    batch = api.Batch(ctx, probs)
    for k in range(count):
        batch.set_io(k, srcs[k], phis[k])
    best_ms = batch.autotune()
    sched = batch.schedule()
    reps = 5

    def time_runs():
        batch.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            batch.run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    # the other schedule with the same tile assignment, for comparison
    other = "planes" if sched == "dataflow" else "dataflow"
    batch.set_schedule(other)
    dt_other = time_runs()
    lat_other = batch.latencies_us()
    batch.set_schedule(sched)
    dt = time_runs()
    lat = batch.latencies_us()
    log(f"batch: {other} schedule {1e3 * dt_other:.2f} ms per run, "
        f"p50 {np.percentile(lat_other, 50):.0f} us, p99 {np.percentile(lat_other, 99):.0f} us")
    log(f"batch: {count} problems, {solves} solves, {1e3 * dt:.2f} ms per run ({sched}), "
        f"p50 {np.percentile(lat, 50):.0f} us, p99 {np.percentile(lat, 99):.0f} us")
    # the sequential baseline: the same problems one after another, each
    # autotuned on its own and swept by its own call (sweep and octant
    # reduction), back to back on one stream
    for prob in probs:
        prob.autotune()
    for k in range(count):
        probs[k].sweep(srcs[k], phis[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for k in range(count):
            probs[k].sweep(srcs[k], phis[k])
    torch.cuda.synchronize()
    dt_seq = (time.perf_counter() - t0) / reps
    log(f"sequential: {1e3 * dt_seq:.2f} ms per run of the {count} problems one by one")
    out = {"problems": count, "solves_per_run": solves, "ms_per_run": 1e3 * dt,
           "solves_per_s": solves / dt, "autotune_best_ms": best_ms,
           "latency_us_p50": float(np.percentile(lat, 50)),
           "latency_us_p99": float(np.percentile(lat, 99)),
           "ann_problems": sum(1 for p in ps if p["solver"] == "ann"),
           "schedule": sched,
           "sequential": {"ms_per_run": 1e3 * dt_seq, "solves_per_s": solves / dt_seq,
                          "speedup_of_batch": dt_seq / dt,
                          "execution": "each problem autotuned alone, then one dgsn_sweep per "
                                       "problem back to back on one stream"},
           "other_schedule": {"schedule": other, "ms_per_run": 1e3 * dt_other,
                              "latency_us_p50": float(np.percentile(lat_other, 50)),
                              "latency_us_p99": float(np.percentile(lat_other, 99))},
           "execution": ("one HIP graph: one dataflow launch over a per-octant work queue of "
                         "all problems' tile blocks" if sched == "dataflow" else
                         "one HIP graph: one batched kernel per step over all problems")}
    batch.close()
    for prob in probs:
        prob.close()
    ann.close()
    return out


def _oracle_threads():
    cores = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        cores = min(cores, int(os.environ["OMP_NUM_THREADS"]))
    return cores


def _time_oracle_sweep(oracle, p, groups, threads, reps):
    """Median wall time of `reps` FP64 oracle sweeps of p restricted to
    `groups` (a slice), source S = q; returns (seconds, solves, phi)."""
    om, w = oracle.lq_n(p["order"])
    st = p["sigma_t"][groups]
    S = np.repeat(p["q"][groups, :, None], 8, axis=-1)
    mesh = (*p["n"], *p["length"])
    times, phi = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        phi = oracle.sweep(mesh, om, w, st, S, p["psi_inc"], nthreads=threads)
        times.append(time.perf_counter() - t0)
    solves = st.shape[1] * len(w) * st.shape[0]
    return float(np.median(times)), solves, phi


def cpu_baseline(p, groups):
    """The FP64 oracle timed on the host on bounded samples of the
    workloads: the benchmark workload (C2: one sweep of its first `groups`
    groups, median of 3, all cores; and one group on 1 core), the 8^3 S4
    absorber (C1, median of 3) and one group of the paper problems at 128^3
    S8 (C3 with GE: Problem 3, median of 3).  Returns the record and the
    oracle's fluxes of the C2 and C3 samples (S = q), against which the GPU
    results state their error."""
    import oracle
    from paper_1906_04017_amd import inputs
    cores = _oracle_threads()
    log(f"cpu baseline: oracle sweeps on {cores} threads and on 1 thread")
    dt, solves, phi_c2 = _time_oracle_sweep(oracle, p, slice(0, groups), cores, 3)
    dt1, solves1, _ = _time_oracle_sweep(oracle, p, slice(0, 1), 1, 1)
    c1 = inputs.absorber_cube()
    dtc1, solvesc1, _ = _time_oracle_sweep(oracle, c1, slice(0, 1), cores, 3)
    c3 = inputs.paper_problems(n=128, groups=4, order=8)
    dtc3, solvesc3, phi_c3 = _time_oracle_sweep(oracle, c3, slice(2, 3), cores, 3)
    rec = {"value": solves / dt, "unit": "solves/s", "cores": cores, "kind": "oracle",
           "sample": f"one FP64 sweep of {p['name']} restricted to {groups} group(s) "
                     f"({solves} solves), median of 3: {dt:.2f} s",
           "value_1core": solves1 / dt1,
           "sample_1core": f"one FP64 sweep of {p['name']} restricted to 1 group "
                           f"({solves1} solves) on 1 thread: {dt1:.2f} s",
           "absorber_cube_8^3_S4_G1": {"solves_per_s": solvesc1 / dtc1, "seconds": dtc1,
                                       "cores": cores, "reps": 3},
           "paper_problem3_128^3_S8_G1": {"solves_per_s": solvesc3 / dtc3, "seconds": dtc3,
                                          "cores": cores, "reps": 3}}
    log(f"cpu baseline: C2 {solves / dt:.3e} solves/s ({cores} threads), "
        f"{solves1 / dt1:.3e} (1 thread); C1 {solvesc1 / dtc1:.3e}; C3 {solvesc3 / dtc3:.3e}")
    return rec, {"c2": phi_c2, "c3_problem3": phi_c3}


def error_vs_oracle(api, ctx, prob, p, refs, groups):
    """Norm-wise relative error max|phi - phi_oracle| / max|phi_oracle| per
    group of one sweep with S = q: the FP32 GE benchmark problem as timed
    (autotuned), a FP64 GE problem on the same workload (autotuned), and the
    FP32 GE sweep of the paper's Problem 3 at 128^3 S8 (autotuned)."""
    import torch
    from paper_1906_04017_amd import inputs

    def per_group(phi, ref):
        phi = phi.double().cpu().numpy()[:ref.shape[0]]
        return [float(np.abs(phi[g] - ref[g]).max() / np.abs(ref[g]).max())
                for g in range(ref.shape[0])]

    S = np.repeat(p["q"][..., None], 8, axis=-1)
    out = {"reference": "FP64 oracle sweep, source S = q", "fp32_tolerance": 1e-5}
    out["fp32_ge_blocky_scatter_per_group"] = per_group(
        prob.sweep(torch.tensor(S, dtype=torch.float32, device="cuda")), refs["c2"])
    om, w = api.quadrature_ls(p["order"])
    p64 = api.Problem(ctx, p["n"], p["length"], p["groups"], om, w, precision="fp64")
    p64.set_materials(p["sigma_t"], p["sigma_s"], p["q"])
    p64.autotune()
    out["fp64_ge_blocky_scatter_per_group"] = per_group(
        p64.sweep(torch.tensor(S, dtype=torch.float64, device="cuda")), refs["c2"])
    p64.close()
    c3 = inputs.paper_problems(n=128, groups=4, order=8)
    om8, w8 = api.quadrature_ls(8)
    pc3 = api.Problem(ctx, c3["n"], c3["length"], 1, om8, w8, precision="fp32")
    pc3.set_materials(c3["sigma_t"][2:3], c3["sigma_s"][2:3], c3["q"][2:3])
    pc3.set_inflow(c3["psi_inc"])
    pc3.autotune()
    S3 = np.repeat(c3["q"][2:3, :, None], 8, axis=-1)
    out["fp32_ge_paper_problem3_128^3"] = per_group(
        pc3.sweep(torch.tensor(S3, dtype=torch.float32, device="cuda")), refs["c3_problem3"])[0]
    pc3.close()
    log("error vs FP64 oracle: fp32 %.2e, fp64 %.2e, fp32 problem 3 %.2e" % (
        max(out["fp32_ge_blocky_scatter_per_group"]),
        max(out["fp64_ge_blocky_scatter_per_group"]), out["fp32_ge_paper_problem3_128^3"]))
    return out


if __name__ == "__main__":
    main()
