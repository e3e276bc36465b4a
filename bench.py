#!/usr/bin/env python3
"""Benchmark of the AMR SIMP hot path on one MI355X.

Workload (default): the octree cantilever -- 16x8x8 base leaves refined up to
3 levels where a seeded smooth density field lies in its 0.1..0.9 band, 2:1
balanced (about 61k elements, 200k DOFs, hanging nodes).  One step is one pass
of the per-iteration hot path on that mesh:

    density -> coefficients + Jacobi diagonal -> K(rho) u = f solve to a
    1e-8 relative residual -> compliance + sensitivities -> sensitivity
    filter (r = 1.5) -> OC update

``value`` is the mean wall time of the solve inside the timed steps (ms,
lower is better) for the solver variant used (--solver; "best" takes the
fastest variant that reaches 1e-8 in an untimed survey).  Variants: plain
FP64 PCG; FP32 and BF16 inner solves with FP64 reliable updates; each of the
first two with the affine coarse space, whose set-up (k = 96 operator
applications on the new density) is counted inside the solve time.  Also
reported: the stiffness-apply roofline of the dominant kernel, the uniform
192x96x96 stiffness-apply bandwidth in FP64/FP32/BF16, the 50-iteration
adaptive SIMP run (plain vs coarse vs learned) and the CPU oracle on a bounded
sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "K(ρ)u=f solve ms to 1e-8 rel-res; stiffness-apply GB/s; learned+mixed vs FP64"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # FP64 vector: 256 CUs x 2.4 GHz x 128 flop/clk
APPLY_SOURCES = ("paper_1009_4975_amd/csrc/apply.hip", "paper_1009_4975_amd/csrc/kernels.h",
                 "paper_1009_4975_amd/csrc/internal.h")
PASS_SOURCES = APPLY_SOURCES + ("paper_1009_4975_amd/csrc/pcg.hip", "paper_1009_4975_amd/csrc/block3.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_octree_c2_traffic.txt")
PASS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "op_pass_octree_c2_fp32_coarse_block3_traffic.txt")
MG_SOURCES = APPLY_SOURCES + ("paper_1009_4975_amd/csrc/mg.hip",)
MG_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mg_level0_pass_octree_c2_traffic.txt")
MG_COARSE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mg_coarse_pass_octree_c2_traffic.txt")
MG_COARSE_BYTES_RULE = ("a coarse-level smoothing pass must move, per 3x3 block of the level's assembled operator, "
                        "its 9 FP64 values and its column index (76 B), and per node the row pointer (4 B), the "
                        "support flags (1 B), the direction d read, the iterate x and the residual r read and "
                        "written, the diagonal inverse read and the next direction written (168 B)")
MG_PASS_BYTES_RULE = ("the level-0 smoothing pass must move, per node that does not hang (hanging nodes carry no "
                      "values in the constrained form): the direction d read, the iterate x and the residual r "
                      "read and written, the diagonal inverse read, the next direction written (3 FP64 values "
                      "each, 168 B); plus c_e per element (8 B)")


def source_hash(sources=APPLY_SOURCES):
    h = hashlib.sha1()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def apply_source_hash():
    return source_hash(APPLY_SOURCES)


def measured_traffic(path=TRAFFIC_FILE, sources=APPLY_SOURCES):
    """HBM bytes per launch of a kernel from its committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the kernel's
    sources changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash(sources):
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(torch):
    """A plain device copy of 256 MiB (reads and writes 268,435,456 bytes
    each): the known traffic that scales FETCH_SIZE and WRITE_SIZE."""
    a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    ms_c = event_time(torch, lambda: c.copy_(a), 10)
    log(f"[bench] copy 256 MiB: {ms_c * 1e3:.1f} us ({2 * a.numel() * 8 / ms_c / 1e6:.0f} GB/s)")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_c2(binding, synth):
    case = synth.c2()
    fld = case.extra["field"]
    L = case.max_level
    t = binding.Octree(case.base, L)
    for _ in range(L):
        lv, an = t.leaves()
        t.refine(synth.band_marks(fld, lv, an, L))
    t.balance()
    mesh = t.build_mesh(case.fixed, case.load)
    lv, an = t.leaves()
    cen = an + 0.5 * (1 << (L - lv))[:, None]
    rho = fld(cen.astype(np.float64))
    return case, t, mesh, rho


def event_time(torch, fn, reps):
    """Average device time of fn() over reps launches, HIP events on the current stream."""
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


# solve variants: inner precision, then "+coarse" (affine coarse space) and/or
# "+block3" (3x3 node-block Jacobi in place of the scalar diagonal)
# multigrid options of the octree solves: two octree levels merged by the first
# coarsening, Chebyshev degree 1 on the analysis mesh and 2 on the coarse
# levels over [lambda_max / 50, 1.1 lambda_max]
MG_OPTS = dict(first=2, ratio=50.0, degree=1, coarse_degree=2, coarse_dofs=700, power_its=8, hi_factor=1.3)
# uniform bricks (C1, C5): degree 2 on every level over [lambda_max / 30, 1.1 lambda_max]
MG_OPTS_UNIFORM = dict(first=2, ratio=30.0, degree=2, coarse_degree=2, power_its=8, hi_factor=1.3, blocks0=True)

SOLVERS = ("fp64", "fp32", "bf16", "fp64+coarse", "fp32+coarse", "fp64+block3", "fp32+block3",
           "fp64+coarse+block3", "fp32+coarse+block3", "fp64+mg")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--solver", choices=[*SOLVERS, "best"],
                    default="best")
    ap.add_argument("--regions", default="3,2,2",
                    help="coarse-space regions rx,ry,rz of the octree solves (12 rx ry rz columns)")
    ap.add_argument("--c4-regions", default="3,2,2",
                    help="coarse-space regions of the adaptive SIMP run's coarse variants")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-c3", action="store_true", help="skip the uniform 192x96x96 apply measurement")
    ap.add_argument("--profile-only", action="store_true", help="only the timed steps (for profilers)")
    ap.add_argument("--c3-only", action="store_true", help="only the uniform 192x96x96 apply measurement")
    ap.add_argument("--no-c4", action="store_true", help="skip the 50-iteration adaptive SIMP run")
    ap.add_argument("--no-c15", action="store_true", help="skip the C1 and C5 solve lines")
    ap.add_argument("--no-amr-vs-uniform", action="store_true", help="skip the AMR against uniform comparison")
    ap.add_argument("--amr-vs-uniform-only", action="store_true", help="only the AMR against uniform comparison")
    ap.add_argument("--c4-only", action="store_true", help="only the 50-iteration adaptive SIMP run")
    ap.add_argument("--net-only", action="store_true",
                    help="only the network training rate at C4's sizes (9 pairs, 65x33x33, channels 4-16-16-16-3)")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2-D cantilever (Q4 quadtree) lines")
    ap.add_argument("--2d-only", dest="only_2d", action="store_true", help="only the 2-D cantilever lines")
    ap.add_argument("--mg-roofline-only", action="store_true",
                    help="only the multigrid level passes on C2 and a copy kernel of known size (for counter runs)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the C2 apply loop and a copy kernel of known size (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (--gpus 1); multi-GPU runs are not supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1009_4975_amd import binding

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    binding.load()
    dev = lambda a, dt=torch.float64: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    if args.c3_only:
        print(json.dumps(apply_uniform_bandwidth(torch, binding, synth, dev)), flush=True)
        copy_calibration(torch)
        return
    if args.net_only:
        print(json.dumps(net_training_rate(torch, binding)), flush=True)
        return
    if args.amr_vs_uniform_only:
        print(json.dumps({f"r{r}": amr_vs_uniform(torch, binding, synth, r) for r in (1.5, 3.0)}), flush=True)
        return
    if args.c4_only:
        print(json.dumps(c4_simp(torch, binding, synth, tuple(int(r) for r in args.c4_regions.split(",")))),
              flush=True)
        return
    if args.only_2d:
        print(json.dumps(plane_2d(torch, binding)), flush=True)
        return

    t0 = time.time()
    case, tree, mesh, rho_h = build_c2(binding, synth)
    log(f"[bench] C2 mesh: {mesh.n_elems} elements, {mesh.n_nodes} nodes, {3 * mesh.n_nodes} DOFs, "
        f"{len(mesh.hang_node)} hanging nodes ({time.time() - t0:.1f}s)")
    ctx = binding.Context(0)
    ctx.upload_mesh(mesh)
    info = ctx.info()
    rho = dev(rho_h)
    f = dev(mesh.f_load)
    b = torch.empty_like(f)
    u = torch.zeros_like(f)
    dc = torch.empty_like(rho)
    dcf = torch.empty_like(rho)
    rho_new = torch.empty_like(rho)
    ctx.set_density(rho)
    ctx.project_rhs(f, b)

    precs = {"fp64": binding.FP64, "fp32": binding.FP32, "bf16": binding.BF16}
    if args.mg_roofline_only:
        ctx.mg_setup(tree, **MG_OPTS)
        # the last dispatches of the level-0 operator and of the coarse-level
        # pass are these passes: 50 on level 0, then 50 on each smoothed coarse level
        lv_us = ctx.mg_pass_times(50)
        info = ctx.mg_info()
        log(f"[bench] C2 multigrid level passes (us): {', '.join(f'{t:.2f}' for t in lv_us)}; "
            f"DOFs {info['dofs']}, blocks {info['blocks']}")
        log(f"[bench] multigrid source hash {source_hash(MG_SOURCES)}")
        copy_calibration(torch)
        return
    if args.roofline_only:
        x = torch.randn_like(f)
        y = torch.empty_like(f)
        ms = event_time(torch, lambda: ctx.apply(x, y, binding.FP64), 50)
        log(f"[bench] C2 FP64 apply: {ms * 1e3:.2f} us/launch")
        name = args.solver if args.solver != "best" else "fp32+coarse+block3"
        op_us, up_us = pass_times(ctx, binding, b, u, name, tuple(int(r) for r in args.regions.split(",")), 50)
        log(f"[bench] C2 {name} operator pass {op_us:.2f} us, update {up_us:.2f} us per launch")
        log(f"[bench] pass source hash {source_hash(PASS_SOURCES)}")
        ctx.mg_setup(tree, **MG_OPTS)
        log(f"[bench] C2 multigrid level passes (us): {ctx.mg_pass_times(50)}")
        log(f"[bench] multigrid source hash {source_hash(MG_SOURCES)}")
        copy_calibration(torch)
        log(f"[bench] apply source hash {apply_source_hash()}")
        return

    c4_regions = tuple(int(r) for r in args.c4_regions.split(","))
    regions = tuple(int(r) for r in args.regions.split(","))

    mg_ready = [False]

    def solve(name, density_set=False):
        """One solve from zero; with "+coarse" the affine coarse space (--regions,
        12 columns per region) is built first and its set-up counts in ms; with
        "+block3" the 3x3 node-block Jacobi preconditioner (its inverse blocks
        are formed on the first solve after a density change, inside ms); with
        "+mg" multigrid-preconditioned CG (the hierarchy is built once per mesh,
        like the operator's chunk tables; its numeric set-up after the density
        change runs inside ms).  density_set: the caller has just set the
        density (the timed step), so the multigrid branch does not set it again."""
        u.zero_()
        if "+mg" in name:
            if not mg_ready[0]:
                ctx.mg_setup(tree, **MG_OPTS)
                mg_ready[0] = True
            if not density_set:
                ctx.set_density(rho)  # a fresh density: the solve rebuilds the coarse operators
                torch.cuda.synchronize()
            st = ctx.mg_pcg(b, u, rtol=1e-8, max_it=2000, check_every=2)
            st["setup_ms"] = 0.0
            return st
        prec = precs[name.split("+")[0]]
        t0 = time.perf_counter()
        coarse = "+coarse" in name
        if coarse:
            ctx.coarse_setup([], *regions, affine=True)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        pc = binding.BLOCK3 if "+block3" in name else binding.JACOBI
        st = ctx.pcg(b, u, rtol=1e-8, inner_prec=prec, inner_rtol=0.1, max_it=50000, precond=pc)
        st["ms"] += setup_ms
        st["setup_ms"] = setup_ms
        if coarse:
            ctx.coarse_clear()
        return st

    # --- solver variants (untimed survey, picks the fastest that reaches 1e-8)
    variants = {}
    if not args.profile_only:
        for name in SOLVERS:
            solve(name)
            runs = [solve(name) for _ in range(2)]
            ms = min(r["ms"] for r in runs)
            variants[name] = dict(ms=round(ms, 3), iters=runs[-1]["iters"], outer=runs[-1]["outer"],
                                  rel_res=runs[-1]["rel_res"], status=runs[-1]["status"],
                                  setup_ms=round(runs[-1]["setup_ms"], 3))
            log(f"[bench] solve {name}: {ms:.2f} ms, iters {runs[-1]['iters']}, outer {runs[-1]['outer']}, "
                f"rel_res {runs[-1]['rel_res']:.2e}")
    if args.solver == "best":
        ok = {k: v for k, v in variants.items() if v["rel_res"] <= 1e-8}
        solver = min(ok, key=lambda k: ok[k]["ms"]) if ok else "fp64"
    else:
        solver = args.solver

    def step():
        ctx.set_density(rho)
        st = solve(solver, density_set=True)
        c = ctx.compliance(u, f, rho, dc)
        ctx.filter(binding.FILTER_SENSITIVITY, 1.5, dc, dcf, rho=rho)
        ctx.oc_update(rho, dcf, rho_new, 0.25)
        return st, c

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    solve_ms, iters, rel = [], [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        st, c = step()
        solve_ms.append(st["ms"])
        iters.append(st["iters"])
        rel.append(st["rel_res"])
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t_start) * 1e3 / args.steps
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.2f} ms/step, solve {np.mean(solve_ms):.2f} ms "
        f"({solver}), compliance {c:.6e}")
    if args.profile_only:
        return

    # --- dominant kernel of the timed step, timed live: for the multigrid
    # solve the coarse-level smoothing pass (block rows with the Chebyshev
    # update; the level-0 pass is a second entry), otherwise the solver
    # variant's fused CG operator pass
    ne, nn = mesh.n_elems, mesh.n_nodes
    roofline_level0 = None
    if "+mg" in solver:
        lv_us = ctx.mg_pass_times(200)
        mgi = ctx.mg_info()
        op_us = lv_us[0]
        pb = 168.0 * (nn - len(mesh.hang_node)) + 8.0 * ne
        gbs = pb / (op_us * 1e-6) / 1e9
        # smoothed coarse levels (the last level is solved by its inverse); each
        # runs the same number of passes per V-cycle, so the launch-weighted
        # rate is total bytes over total time of one pass on each
        coarse = list(range(1, mgi["levels"] - 1))
        cb = [76.0 * mgi["blocks"][k] + 173.0 * (mgi["dofs"][k] // 3) + 4.0 for k in coarse]
        ct = [lv_us[k] for k in coarse]
        cgbs = sum(cb) / (sum(ct) * 1e-6) / 1e9
        log(f"[bench] C2 multigrid level passes (us): {', '.join(f'{t:.2f}' for t in lv_us)}; level 0 "
            f"{gbs:.0f} GB/s, coarse levels {cgbs:.0f} GB/s algorithmic")
        roofline = dict(bound="hbm", achieved=round(cgbs, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(cgbs / HBM_PEAK_GBS, 5),
                        traffic=measured_traffic(MG_COARSE_TRAFFIC_FILE, MG_SOURCES),
                        kernel="coarse-level smoothing pass of the multigrid V-cycle (k_mg_spmv<16>: product with "
                               "the level's 3x3 block rows and the Chebyshev update), one pass on each smoothed "
                               "coarse level (they run equally often)",
                        per_launch_us=round(sum(ct) / len(ct), 3), alg_bytes_per_launch=int(sum(cb) / len(cb)),
                        bytes_rule=MG_COARSE_BYTES_RULE,
                        levels=[dict(level=k, dofs=mgi["dofs"][k], blocks=mgi["blocks"][k], us=round(t, 3),
                                     alg_bytes=int(x), gbs=round(x / (t * 1e-6) / 1e9, 1))
                                for k, t, x in zip(coarse, ct, cb)],
                        traffic_unit="bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)")
        roofline_level0 = dict(bound="hbm", achieved=round(gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                               frac=round(gbs / HBM_PEAK_GBS, 5),
                               traffic=measured_traffic(MG_TRAFFIC_FILE, MG_SOURCES),
                               kernel="level-0 smoothing pass of the multigrid V-cycle (k_apply_chunks FP64: "
                                      "stiffness apply with the Chebyshev update of x, r and the next direction)",
                               per_launch_us=round(op_us, 3), alg_bytes_per_launch=int(pb),
                               bytes_rule=MG_PASS_BYTES_RULE,
                               traffic_unit="bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)")
    else:
        op_us, up_us = pass_times(ctx, binding, b, u, solver, regions, 200)
        pb = pass_bytes(solver, nn, ne)
        gbs = pb / (op_us * 1e-6) / 1e9
        log(f"[bench] C2 {solver} operator pass: {op_us:.2f} us/launch, {gbs:.0f} GB/s algorithmic; "
            f"update side {up_us:.2f} us")
        roofline = dict(bound="hbm", achieved=round(gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(gbs / HBM_PEAK_GBS, 5),
                        traffic=(measured_traffic(PASS_TRAFFIC_FILE, PASS_SOURCES)
                                 if solver == "fp32+coarse+block3" else None),
                        kernel=f"fused CG operator pass of the {solver} solve (k_apply_chunks: stiffness apply, "
                               "preconditioner, search direction, coarse-space partials)",
                        per_launch_us=round(op_us, 3), alg_bytes_per_launch=int(pb),
                        bytes_rule=PASS_BYTES_RULE, update_side_us=round(up_us, 3),
                        traffic_unit="bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)")
    # second entry: the plain FP64 stiffness apply on the same mesh
    x = torch.randn_like(f)
    y = torch.empty_like(f)
    apply_ms = event_time(torch, lambda: ctx.apply(x, y, binding.FP64), 200)
    ab = 48.0 * nn + 8.0 * ne
    log(f"[bench] C2 FP64 apply: {apply_ms * 1e3:.2f} us/launch ({ab / apply_ms / 1e6:.0f} GB/s algorithmic)")
    roofline_apply = dict(bound="hbm", achieved=round(ab / (apply_ms * 1e-3) / 1e9, 2), peak=HBM_PEAK_GBS,
                          unit="GB/s", frac=round(ab / (apply_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                          traffic=measured_traffic(), kernel="octree FP64 stiffness apply (k_apply_chunks, FP64)",
                          per_launch_us=round(apply_ms * 1e3, 3), alg_bytes_per_launch=int(ab),
                          bytes_rule="x read 24 B/node + y write 24 B/node + c_e 8 B/element",
                          traffic_unit="bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)")

    # --- C1 (one SIMP iteration on the uniform 24x12x12 cantilever) and C5
    # (1.6 M DOF bridge: solves and the adjoint sensitivities)
    c1 = None if args.no_c15 else solve_c1(torch, binding, synth, dev)
    c5 = None if args.no_c15 else solve_c5(torch, binding, synth, dev)

    # --- uniform 192x96x96 apply bandwidth
    c3 = None
    if not args.no_c3:
        c3 = apply_uniform_bandwidth(torch, binding, synth, dev)

    # --- 50-iteration adaptive SIMP run: plain vs coarse-corrected vs learned
    c4 = None
    if not args.no_c4:
        c4 = c4_simp(torch, binding, synth, c4_regions)

    # --- AMR against the uniform fine mesh (paper's trigger, design difference)
    avu = None if args.no_amr_vs_uniform else {f"r{r}": amr_vs_uniform(torch, binding, synth, r) for r in (1.5, 3.0)}
    net_rate = None if args.no_c4 else net_training_rate(torch, binding)

    # --- the 2-D variant: 256 x 128 Q4 cantilever, uniform and adaptive
    p2d = None if args.no_2d else plane_2d(torch, binding)

    # --- CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(synth, case, tree, mesh, rho_h, variants.get("fp64", {}).get("iters"))

    out = {
        "metric": METRIC, "value": round(float(np.mean(solve_ms)), 3), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16+f64"}[solver.split("+")[0]], "data": "synthetic",
        "config": {"workload": "octree cantilever 16x8x8 base leaves, 3 refinement levels, band-refined and "
                               "2:1 balanced", "elements": ne, "nodes": nn, "dofs": 3 * nn,
                   "hanging_nodes": int(len(mesh.hang_node)), "chunks": info["n_chunks"], "solver": solver,
                   "coarse_regions": list(regions) if "+coarse" in solver else None,
                   "multigrid": dict(MG_OPTS) if "+mg" in solver else None,
                   "rtol": 1e-8, "E0": 1.0, "Emin": 1e-9, "nu": 0.3, "p": 3.0},
        "solve_iters": int(np.median(iters)), "solve_rel_res": float(max(rel)),
        "solve_variants": variants, "roofline": roofline, "roofline_level0_pass": roofline_level0,
        "roofline_apply_fp64": roofline_apply,
        "c1_simp_iteration_24x12x12": c1, "c5_bridge_128x64x64": c5,
        "apply_uniform_192x96x96": c3, "simp_adaptive_bridge": c4, "network_training": net_rate, "amr_vs_uniform_cantilever": avu,
        "plane_2d_cantilever_256x128": p2d, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


PASS_BYTES_RULE = ("vectors the fused operator pass must move, per node: r read, preconditioner read (Jacobi "
                   "3 or node blocks 6 values), previous direction read, new direction and q written (3 values "
                   "each); plain passes read z instead of r and the preconditioner; plus c_e per element; "
                   "values of the inner precision (FP64 8 B, FP32 4 B)")


def pass_bytes(name, nn, ne):
    """Algorithmic bytes of one fused operator pass of solver variant `name`."""
    vb = 8 if name.startswith("fp64") else 4
    if "+coarse" in name:
        per_node = 3 + (6 if "+block3" in name else 3) + 3 + 3 + 3
    else:
        per_node = 3 + 3 + 3 + 3
    return per_node * vb * nn + vb * ne


def pass_times(ctx, binding, b, u, name, regions, reps):
    """Mean device time (us) of one operator pass and one update side of the
    solver variant `name` (amrto_pcg_pass_times, HIP events on the context
    stream); the coarse space is set up first for "+coarse" variants."""
    precs = {"fp64": binding.FP64, "fp32": binding.FP32, "bf16": binding.BF16}
    coarse = "+coarse" in name
    if coarse:
        ctx.coarse_setup([], *regions, affine=True)
    w = u.clone().zero_()
    op, up = ctx.pcg_pass_times(b, w, reps=reps, inner_prec=precs[name.split("+")[0]],
                                precond=binding.BLOCK3 if "+block3" in name else binding.JACOBI)
    if coarse:
        ctx.coarse_clear()
    return op, up


def best_ms(fn, n=3):
    out = [fn() for _ in range(n)]
    return min(out, key=lambda r: r["ms"]), out


def solve_c1(torch, binding, synth, dev):
    """One SIMP iteration on the uniform 24x12x12 cantilever (3,456 elements,
    12,675 DOFs): the seeded densities smoothed once by the r = 1.5 cone
    filter, then Jacobi-PCG (FP64) from zero to 1e-8, compliance and
    sensitivities, the Eq. (5) filter and the OC step; best of three."""
    case = synth.c1()
    tree = binding.Octree(case.dims, 0)
    mesh = binding.uniform_mesh(case.dims, case.fixed, case.load, tree=tree)
    ctx = binding.Context(0)
    ctx.upload_mesh(mesh)
    rho0 = dev(case.rho)
    rho = torch.empty_like(rho0)
    ctx.filter(binding.FILTER_DENSITY, case.smooth_radius, rho0, rho)
    f = dev(mesh.f_load)
    b = torch.empty_like(f)
    u = torch.zeros_like(f)
    dc, dcf, rho_new = (torch.empty_like(rho) for _ in range(3))

    def it(mg=False):
        t0 = time.perf_counter()
        ctx.set_density(rho)
        ctx.project_rhs(f, b)
        u.zero_()
        st = ctx.mg_pcg(b, u, rtol=1e-8, max_it=2000) if mg else ctx.pcg(b, u, rtol=1e-8)
        t1 = time.perf_counter()
        c = ctx.compliance(u, f, rho, dc)
        ctx.filter(binding.FILTER_SENSITIVITY, case.filter_radius, dc, dcf, rho=rho)
        ch, _ = ctx.oc_update(rho, dcf, rho_new, 0.3)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return dict(ms=(t2 - t0) * 1e3, solve_ms=st["ms"], design_ms=(t2 - t1) * 1e3, iters=st["iters"],
                    rel_res=st["rel_res"], compliance=c)

    it()
    r, _ = best_ms(it)
    log(f"[bench] C1 SIMP iteration: {r['ms']:.2f} ms (solve {r['solve_ms']:.2f} ms, {r['iters']} iterations, "
        f"rel_res {r['rel_res']:.2e}; compliance, sensitivities, filter, OC {r['design_ms']:.2f} ms)")
    ctx.mg_setup(tree, **MG_OPTS_UNIFORM)
    it(True)
    m, _ = best_ms(lambda: it(True))
    log(f"[bench] C1 SIMP iteration, multigrid: {m['ms']:.2f} ms (solve {m['solve_ms']:.2f} ms, {m['iters']} iterations, "
        f"rel_res {m['rel_res']:.2e})")
    return dict(iteration_ms=round(r["ms"], 3), solve_ms=round(r["solve_ms"], 3), design_ms=round(r["design_ms"], 3),
                iters=r["iters"], rel_res=r["rel_res"], compliance=r["compliance"], dofs=3 * mesh.n_nodes,
                solver="fp64 Jacobi-PCG from zero", rtol=1e-8,
                multigrid=dict(iteration_ms=round(m["ms"], 3), solve_ms=round(m["solve_ms"], 3), iters=m["iters"],
                               rel_res=m["rel_res"], compliance=m["compliance"], options=dict(MG_OPTS_UNIFORM)))


def solve_c5(torch, binding, synth, dev):
    """The 128x64x64 bridge (524,288 elements, 1,635,075 DOFs), rho ~ U[0.01, 1]:
    solves from zero to 1e-8 in FP64 and with FP32 inner solves (Jacobi and
    block-Jacobi), then compliance + adjoint sensitivities of the FP64
    solution; best of two per variant."""
    case = synth.c5()
    tree = binding.Octree(case.dims, 0)
    mesh = binding.uniform_mesh(case.dims, case.fixed, case.load, tree=tree)
    ctx = binding.Context(0)
    ctx.upload_mesh(mesh)
    rho = dev(case.rho)
    ctx.set_density(rho)
    f = dev(mesh.f_load)
    b = torch.empty_like(f)
    ctx.project_rhs(f, b)
    u = torch.zeros_like(f)
    dc = torch.empty_like(rho)
    out = {}
    for name, prec, pc in (("fp64", binding.FP64, binding.JACOBI), ("fp32", binding.FP32, binding.JACOBI),
                           ("fp64+block3", binding.FP64, binding.BLOCK3),
                           ("fp32+block3", binding.FP32, binding.BLOCK3)):
        def run():
            u.zero_()
            return ctx.pcg(b, u, rtol=1e-8, inner_prec=prec, inner_rtol=0.1, max_it=50000, precond=pc)
        r, _ = best_ms(run, 2)
        out[name] = dict(ms=round(r["ms"], 2), iters=r["iters"], outer=r["outer"], rel_res=r["rel_res"])
        log(f"[bench] C5 solve {name}: {r['ms']:.1f} ms, {r['iters']} iterations, rel_res {r['rel_res']:.2e}")
    ctx.mg_setup(tree, **MG_OPTS_UNIFORM)

    def run_mg():
        u.zero_()
        ctx.set_density(rho)  # the solve rebuilds the coarse operators
        torch.cuda.synchronize()
        return ctx.mg_pcg(b, u, rtol=1e-8, max_it=2000)
    r, _ = best_ms(run_mg, 2)
    out["fp64+mg"] = dict(ms=round(r["ms"], 2), iters=r["iters"], rel_res=r["rel_res"], options=dict(MG_OPTS_UNIFORM))
    log(f"[bench] C5 solve fp64+mg: {r['ms']:.1f} ms, {r['iters']} iterations, rel_res {r['rel_res']:.2e}")
    u.zero_()
    ctx.pcg(b, u, rtol=1e-8)
    ctx.compliance(u, f, rho, dc)
    sens_ms = event_time(torch, lambda: ctx.sensitivity(u, rho, dc), 20)
    out["adjoint_sensitivity_us"] = round(sens_ms * 1e3, 2)
    out["dofs"] = 3 * mesh.n_nodes
    log(f"[bench] C5 adjoint sensitivities: {sens_ms * 1e3:.1f} us per launch")
    return out


def amr_vs_uniform(torch, binding, synth, r=1.5):
    """The paper's AMR-against-uniform comparison on a synthetic cantilever:
    the same SIMP loop (multigrid-preconditioned CG to 1e-8 from the previous
    displacement, Eq. (5) filter, OC) on the fixed uniform 128x32x32 mesh and
    on an adaptive mesh started at 64x16x16 (one refinement level) adapted by
    the paper's trigger (CASE (i): largest design change < 0.01 after >= 5
    steps; CASE (ii): 10 steps), for the same number of design steps.  Both
    run the octree operator kernels and the same multigrid options.  Reports
    sizes, iterations, solve time, the first step whose design change fell
    below 0.01, the final compliances and the design difference D of
    Eq. (10) between the final designs (also every 50 steps).  r is the
    filter and refinement radius in finest cells."""
    from paper_1009_4975_amd.simp import AdaptiveSIMP
    case = synth.amr_vs_uniform(r=r)
    ex = case.extra
    sims, recs = {}, {"uniform": [], "amr": []}
    for name, base, L, rule in (("uniform", case.dims, 0, "never"), ("amr", case.base, case.max_level, "paper")):
        sims[name] = AdaptiveSIMP(base, L, case.fixed, case.load, volfrac=ex["volfrac"], rho_init=ex["rho_init"],
                                  rmin=ex["rmin"], rho_solid=ex["rho_solid"], r_amr=ex["r_amr"], adapt_rule=rule,
                                  min_steps=ex["min_steps"], max_steps=ex["max_steps"],
                                  change_tol=ex["change_tol"], rtol=1e-8, mg=MG_OPTS,
                                  p_continuation=ex.get("p_continuation"))
    trail = []
    t0 = time.perf_counter()
    for s in range(ex["steps"]):
        for name, sim in sims.items():
            recs[name].append(sim.step())
        if (s + 1) % 50 == 0:
            trail.append([s + 1, round(sims["uniform"].ctx.design_difference(
                sims["uniform"].rho, sims["amr"].ctx, sims["amr"].rho), 5)])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {}
    for name, rs in recs.items():
        conv = [i + 1 for i, x in enumerate(rs) if x["change"] < ex["change_tol"]]
        out[name] = dict(steps=len(rs), solve_ms=round(sum(x["solve_ms"] for x in rs), 1),
                         pcg_iters=int(sum(x["iters"] for x in rs)),
                         dofs_mean=int(np.mean([x["dofs"] for x in rs])), dofs_final=rs[-1]["dofs"],
                         elements_final=rs[-1]["n_elems"], adaptations=int(sum(x["adapted"] for x in rs)),
                         final_compliance=rs[-1]["compliance"], final_change=rs[-1]["change"],
                         first_step_change_below_tol=conv[0] if conv else None,
                         max_rel_res=max(x["rel_res"] for x in rs))
    su, sa = sims["uniform"], sims["amr"]
    D = su.ctx.design_difference(su.rho, sa.ctx, sa.rho)
    out["design_difference_D"] = D
    out["design_difference_every_50_steps"] = trail
    out["compliance_rel_diff_amr_vs_uniform"] = round(
        out["amr"]["final_compliance"] / out["uniform"]["final_compliance"] - 1.0, 5)
    out["solve_time_ratio_uniform_over_amr"] = round(out["uniform"]["solve_ms"] / out["amr"]["solve_ms"], 3)
    out["dofs_ratio_amr_over_uniform"] = round(out["amr"]["dofs_mean"] / out["uniform"]["dofs_mean"], 3)
    out["wall_s_both"] = round(wall, 2)
    out["config"] = dict(uniform=list(case.dims), amr_initial=list(case.base), levels=case.max_level,
                         volfrac=ex["volfrac"], rmin=ex["rmin"], r_amr=ex["r_amr"], steps=ex["steps"],
                         solver="fp64 multigrid-PCG, 1e-8", multigrid=dict(MG_OPTS),
                         p_continuation=ex.get("p_continuation"))
    log(f"[bench] AMR vs uniform (r = {r}, {ex['steps']} steps): uniform {out['uniform']['solve_ms']} ms solve, "
        f"{out['uniform']['pcg_iters']} its, {out['uniform']['dofs_mean']} DOFs mean, c {out['uniform']['final_compliance']:.4f}; "
        f"AMR {out['amr']['solve_ms']} ms, {out['amr']['pcg_iters']} its, {out['amr']['dofs_mean']} DOFs mean, "
        f"{out['amr']['adaptations']} adapts, c {out['amr']['final_compliance']:.4f}; "
        f"D = {100 * D:.3f} %, time ratio {out['solve_time_ratio_uniform_over_amr']}")
    return out


def net_training_rate(torch, binding, epochs=100):
    """Training epochs (forward, masked MSE, backward, Adam) of the warm-start
    network at the sizes C4 trains it on: 9 (density, displacement) pairs on
    the 65x33x33 grid of the 128x64x64 lattice (every second node), channels
    4-16-16-16-3, synthetic inputs (seed 0).  FLOPs count the convolutions'
    multiply-adds, forward once and backward twice."""
    ch, grid, B = [4, 16, 16, 16, 3], (65, 33, 33), 9
    net = binding.Net(ch, grid, max_batch=16, seed=0)
    g = torch.Generator(device="cuda").manual_seed(0)
    shape = (B, 4, grid[2], grid[1], grid[0])
    X = torch.randn(shape, device="cuda", generator=g)
    Y = torch.randn((B, 3) + shape[2:], device="cuda", generator=g)
    out, dout = torch.empty_like(Y), torch.empty_like(Y)

    def epoch(t):
        net.forward(X, out)
        net.mse(out, Y, dout)
        net.backward(dout)
        net.adam(1e-3, t)

    for t in range(1, 4):
        epoch(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(4, 4 + epochs):
        epoch(t)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / epochs
    V = grid[0] * grid[1] * grid[2]
    flop = 3 * sum(2 * B * V * a * c * 27 for a, c in zip(ch[:-1], ch[1:]))
    log(f"[bench] network training: {ms:.3f} ms per epoch ({flop / ms / 1e9:.1f} TFLOP/s of convolution work)")
    return dict(ms_per_epoch=round(ms, 4), tflops=round(flop / ms / 1e9, 2), pairs=B, grid=list(grid), channels=ch)


def apply_uniform_bandwidth(torch, binding, synth, dev):
    case = synth.c3()
    t0 = time.time()
    mesh = binding.uniform_mesh(case.dims, case.fixed, case.load)
    ctx = binding.Context(0)
    ctx.upload_mesh(mesh)
    ctx.set_density(dev(case.rho))
    nn, ne = mesh.n_nodes, mesh.n_elems
    log(f"[bench] C3 mesh {case.dims}: {ne} elements, {3 * nn} DOFs ({time.time() - t0:.1f}s)")
    xv = synth.random_vector(3 * nn, case.extra["vec_seed"])
    xv[mesh.dof_fixed.astype(bool)] = 0.0
    res = {}
    # rotate through enough buffers (> 256 MB Infinity Cache) so every launch reads from HBM
    for name, prec, dt, vb in (("fp64", binding.FP64, torch.float64, 8), ("fp32", binding.FP32, torch.float32, 4),
                               ("bf16", binding.BF16, torch.float32, 4)):
        nbuf = max(3, int(np.ceil(800e6 / (2 * 3 * nn * vb))))
        xs = [dev(xv, dt) for _ in range(nbuf)]
        ys = [torch.empty(3 * nn, dtype=dt, device="cuda") for _ in range(nbuf)]
        k = [0]

        def fn():
            i = k[0] % nbuf
            ctx.apply(xs[i], ys[i], prec)
            k[0] += 1

        ms = event_time(torch, fn, 60)
        cb = 8 if prec == binding.FP64 else 4
        alg_bytes = 2 * 3 * nn * vb + ne * cb + nn  # x read, y write, c_e, support mask
        gbs = alg_bytes / (ms * 1e-3) / 1e9
        res[name] = dict(us=round(ms * 1e3, 2), alg_bytes=alg_bytes, GBps=round(gbs, 1),
                         hbm_frac=round(gbs / HBM_PEAK_GBS, 4),
                         TFLOPs=round(1152.0 * ne / (ms * 1e-3) / 1e12, 2))
        log(f"[bench] C3 apply {name}: {ms * 1e3:.1f} us, {gbs:.0f} GB/s algorithmic "
            f"({100 * gbs / HBM_PEAK_GBS:.1f}% of HBM), {res[name]['TFLOPs']} TFLOP/s")
        del xs, ys
    return res


def c4_simp(torch, binding, synth, regions=(2, 2, 2)):
    """The adaptive bridge: 32x16x16 base leaves, 2 refinement levels (finest
    128x64x64), volume fraction 0.25, filter radius 1.5, OC, adapt every 5
    iterations, 50 iterations.  Variants differ only in how iterations 11-50
    solve: plain (previous solution as the start, Jacobi-PCG), plain with the
    3x3 node-block Jacobi preconditioner, the affine coarse space, and the
    learned start (network trained on iterations 1-10) with the coarse space;
    each in FP64 and with FP32 inner solves; recycled Krylov vectors;
    multigrid-preconditioned CG (its hierarchy rebuilt at every adaptation);
    and multigrid started from the network's prediction (the energy line
    search from u_prev along it), which isolates what the network gains."""
    from paper_1009_4975_amd.learned import LearnedWarmStart
    from paper_1009_4975_amd.simp import AdaptiveSIMP
    case = synth.c4()
    ex = case.extra
    n_train = ex["train_iters"]
    out = {}
    for name, prec, mode in (("plain_fp64", binding.FP64, None), ("plain_fp32", binding.FP32, None),
                             ("block3_fp64", binding.FP64, "block3"), ("block3_fp32", binding.FP32, "block3"),
                             ("coarse_fp64", binding.FP64, "coarse"), ("coarse_fp32", binding.FP32, "coarse"),
                             ("coarse_block3_fp64", binding.FP64, "coarse+block3"),
                             ("coarse_block3_fp32", binding.FP32, "coarse+block3"),
                             ("learned_coarse_fp64", binding.FP64, "learned"),
                             ("learned_coarse_fp32", binding.FP32, "learned"),
                             ("recycle_init_coarse_block3_fp64", binding.FP64, "recycle_init+coarse+block3"),
                             ("recycle_init_coarse_block3_fp32", binding.FP32, "recycle_init+coarse+block3"),
                             ("recycle_in_coarse_space_fp64", binding.FP64, "recycle_coarse"),
                             ("mg_fp64", binding.FP64, "mg"), ("learned_mg_fp64", binding.FP64, "learned_mg")):
        t0 = time.perf_counter()
        sim = AdaptiveSIMP(case.base, case.max_level, case.fixed, case.load, volfrac=ex["volfrac"],
                           rho_init=ex["rho_init"], rmin=ex["rmin"], rho_solid=ex["rho_solid"], r_amr=ex["r_amr"],
                           adapt_every=ex["adapt_every"], rtol=1e-8, inner_prec=prec, inner_rtol=0.1,
                           precond=binding.BLOCK3 if (mode or "").endswith("block3") else binding.JACOBI,
                           mg=MG_OPTS if mode in ("mg", "learned_mg") else None)
        if mode == "mg":
            mode = None  # every solve (iterations 1-50) is multigrid-preconditioned
        learned = mode in ("learned", "learned_mg")
        rec_from, rec_mode = None, None
        if (mode or "").startswith("recycle"):
            # from iteration 11 on: recorded solves whose Ritz vectors start
            # the next solve ("init", with the solver of the coarse+block3
            # variant) or join the affine coarse space ("coarse")
            rec_mode = "init" if mode.startswith("recycle_init") else "coarse"
            mode = "coarse" if rec_mode == "init" else None
            rec_from = n_train
        # the node-block preconditioner changes nothing else in a run
        mode = {"block3": None, "coarse+block3": "coarse"}.get(mode, mode)
        ws = LearnedWarmStart(case.dims, cell=2, hidden=8, layers=3, epochs=100, seed=ex["net_seed"],
                              regions=tuple(regions)) if mode else None
        recs, train_ms = [], 0.0
        for k in range(ex["iters"]):
            if rec_from is not None and k == rec_from:
                sim.recycle = dict(mode=rec_mode, m=64, k=4, keep=4, regions=tuple(regions), affine=True)
                sim.ctx.recycle_setup(64)
            if learned and k < n_train:
                r = sim.step(warm_start=ws.collect_before, after_solve=ws.collect_after)
            elif mode and k >= n_train:
                if learned and not ws.trained:
                    ws.train()
                    train_ms = ws.train_ms
                # with multigrid the network's start is the only change (no coarse space)
                r = sim.step(warm_start=(lambda s: ws.warm_start(s, use_net=learned,
                                                                 coarse=False if mode == "learned_mg" else None)))
            else:
                r = sim.step()
            recs.append(r)
        torch.cuda.synchronize()
        late = recs[n_train:]
        out[name] = dict(
            iters_11_50=int(sum(r["iters"] for r in late)),
            solve_ms_11_50=round(sum(r["solve_ms"] for r in late), 1),
            warm_and_coarse_setup_ms_11_50=round(sum(r["warm_ms"] for r in late), 1),
            train_ms=round(train_ms, 1),
            step_ms_total=round(sum(r["step_ms"] for r in recs), 1),
            wall_s=round(time.perf_counter() - t0, 2),
            final_compliance=recs[-1]["compliance"], max_rel_res=max(r["rel_res"] for r in recs),
            dofs_min_max=[min(r["dofs"] for r in recs), max(r["dofs"] for r in recs)],
            elements_final=recs[-1]["n_elems"])
        log(f"[bench] C4 {name}: iterations 11-50 {out[name]['iters_11_50']} PCG its, "
            f"{out[name]['solve_ms_11_50']} ms solve + {out[name]['warm_and_coarse_setup_ms_11_50']} ms set-up, "
            f"train {train_ms:.0f} ms, compliance {recs[-1]['compliance']:.6e}, DOFs {out[name]['dofs_min_max']}")
    base = out["plain_fp64"]
    for k, v in out.items():
        v["time_vs_plain_fp64"] = round((v["solve_ms_11_50"] + v["warm_and_coarse_setup_ms_11_50"] + v["train_ms"]) /
                                        (base["solve_ms_11_50"] + base["warm_and_coarse_setup_ms_11_50"]), 4)
    return out


PLANE_BYTES_RULE = ("per CG iteration, per node: z and the previous direction read, the new direction written; "
                    "the direction read and q written by the operator; x, r, the direction, q and the inverse "
                    "diagonal read and x, r, z written by the update (2 FP64 values each, 208 B); plus the "
                    "element modulus (8 B per element)")


def plane_2d(torch, binding):
    """The 2-D variant on the 256 x 128 cantilever (left edge clamped, unit
    point load at the middle of the right edge, volume fraction 0.5, rmin 1.5):
    one design iteration on the uniform grid (solve from zero to 1e-8 on a
    seeded smooth density), and 40 adaptive iterations from 32 x 16 base
    leaves with 3 levels (adapt every 10) against the same 40 on the uniform
    grid."""
    from paper_1009_4975_amd.plane_simp import PlaneSIMP
    out = {}
    sim = PlaneSIMP((32, 16), 3, uniform=True, volfrac=0.5, rmin=1.5, adapt_every=0, check_every=64)
    lv, an = sim.leaves()
    cen = an + 0.5 * (1 << (3 - lv))[:, None]
    rng = np.random.default_rng(2024)
    rho_h = np.clip(0.5 + 0.35 * np.sin(cen[:, 0] / 17.0 + rng.uniform(0, 6.28)) *
                    np.cos(cen[:, 1] / 11.0 + rng.uniform(0, 6.28)), 0.05, 1.0)
    rho = torch.tensor(rho_h, dtype=torch.float64, device="cuda")
    sim.ctx.set_density(rho)
    u = torch.zeros_like(sim.f)
    runs = []
    for _ in range(3):
        u.zero_()
        torch.cuda.synchronize()
        runs.append(sim.ctx.pcg(sim.b, u, rtol=1e-8, max_it=100000, check_every=64))
    best = min(runs, key=lambda r: r["ms"])
    nn, ne = sim.mesh.n_nodes, sim.mesh.n_elems
    us_it = best["ms"] * 1e3 / max(1, best["iters"])
    alg = 208.0 * nn + 8.0 * ne
    out["uniform_solve"] = dict(elements=ne, dofs=2 * nn, solve_ms=round(best["ms"], 3), iters=best["iters"],
                                outer=best["outer"], rel_res=best["rel_res"], us_per_iter=round(us_it, 3),
                                alg_bytes_per_iter=int(alg), gbs=round(alg / (us_it * 1e-6) / 1e9, 2),
                                bytes_rule=PLANE_BYTES_RULE)
    log(f"[bench] 2-D uniform 256x128 solve: {best['ms']:.2f} ms, {best['iters']} iters, {us_it:.2f} us/iter")
    for name, kw in (("uniform", dict(uniform=True, adapt_every=0)), ("amr", dict(uniform=False, adapt_every=10))):
        s = PlaneSIMP((32, 16), 3, volfrac=0.5, rmin=1.5, check_every=64, **kw)
        recs = [s.step() for _ in range(40)]
        out[name + "_40_iterations"] = dict(
            solve_ms_total=round(sum(r["solve_ms"] for r in recs), 2),
            step_ms_total=round(sum(r["step_ms"] for r in recs), 2),
            iters_total=int(sum(r["iters"] for r in recs)), dofs_mean=round(float(np.mean([r["dofs"] for r in recs])), 1),
            dofs_last=recs[-1]["dofs"], compliance_last=recs[-1]["compliance"], adapts=sum(r["adapted"] for r in recs))
        log(f"[bench] 2-D {name} 40 iterations: solve {out[name + '_40_iterations']['solve_ms_total']:.1f} ms, "
            f"compliance {recs[-1]['compliance']:.4f}, dofs {recs[-1]['dofs']}")
    out["config"] = dict(lattice=[256, 128], base=[32, 16], levels=3, load="unit point load at (256, 64), -y",
                         support="x = 0", volfrac=0.5, rmin=1.5, rtol=1e-8, p=3.0)
    return out


def cpu_baseline(synth, case, tree, mesh, rho_h, gpu_iters):
    """The oracle's Jacobi-PCG on the same C2 system, single thread: one full
    solve to a relative residual of 1e-8 (about 10 s of CPU work), timed as
    it stands; the assembly before it is reported, not counted."""
    from threadpoolctl import threadpool_limits

    from oracle import mesh as om, system as osys
    with threadpool_limits(1):
        t0 = time.perf_counter()
        lv, an = tree.leaves()
        m = om.build_mesh(lv, an, case.max_level, case.dims)
        key = {tuple(c): i for i, c in enumerate(m.coords.tolist())}
        okey = {(int(l), *map(int, a)): e for e, (l, a) in enumerate(zip(m.level, m.anchor))}
        eperm = np.array([okey[(int(l), *map(int, a))] for l, a in zip(lv, an)])
        rho_o = np.empty(m.n_elems)
        rho_o[eperm] = rho_h
        s = osys.build_system(m, osys.elem_coeff(m, rho_o), om.fixed_dofs(m, case.fixed), om.load_vector(m, case.load))
        setup = time.perf_counter() - t0
        r = osys.pcg_jacobi(s.A, s.b, rtol=1e-8, max_it=20000)
        per_it = r.seconds / max(1, r.iters)
    log(f"[bench] CPU oracle: setup {setup:.1f}s, full solve {r.seconds:.1f}s: {r.iters} iterations "
        f"({per_it * 1e3:.2f} ms each; the FP64 GPU solve took {gpu_iters}), true rel. residual {r.rel_res:.2e}")
    return dict(value=round(r.seconds * 1e3, 1), unit="ms", cores=1, kind="oracle",
                sample=f"oracle Jacobi-PCG on the same assembled system, one full solve to 1e-8: {r.iters} "
                       f"iterations in {r.seconds:.1f}s; assembly/setup {setup:.1f}s not included",
                host=host_info(), threads="1 (threadpoolctl limit on BLAS/OpenMP; SciPy CSR matvec is serial)")


def host_info():
    """CPU model, logical CPUs and thread settings of the host the oracle runs on."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return dict(cpu_model=model, os_cpu_count=os.cpu_count(), affinity_cpus=affinity,
                OMP_NUM_THREADS=os.environ.get("OMP_NUM_THREADS"))


if __name__ == "__main__":
    main()
