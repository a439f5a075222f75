"""Benchmark of the generalized-Stokes hot path on one MI355X.

Workload (default): the 128^3 warped box with log-uniform viscosity per 8^3
block (contrast up to 1e6), Q2-Q1, 6 levels down to 4^3, 50.9M velocity +
2.1M pressure dofs.

One timed step = one pass of the whole hot path on that workload:
  * R applications of the FP64 matrix-free operator A (the dominant kernel;
    every colour launch timed with HIP events on the library stream);
  * geometry + coefficient upload and preconditioner setup (ALE Jacobians,
    coefficient packing, diag(A), diag(B diag(A)^-1 B^T), Lanczos bounds,
    dense coarse inverse, V-cycle graphs);
  * three solves from a zero guess to relative residual 1e-8: the plain FP64
    path (FP64 V-cycle launched kernel by kernel, separate Chebyshev/residual
    vector kernels, default launch shapes), the same FP64 solve with every
    optimisation (captured graph, fused last-touch epilogues, tuned launches),
    and the mixed-precision solve (FP32 V-cycle, FP64 FGMRES / residuals /
    Schur block) with the same optimisations.
Inputs are resident in HBM before the timed region.  `value` is the FP64
vmult throughput N_vel / t_apply in GDoF/s; the solve times, their ratio
and the mixed-vs-FP64 velocity difference are reported beside it.

After the timed steps (not part of them): the pseudo-elastic extension solve
on the same mesh (flexible CG + multigrid on A with c_m = 0, eta = mu_A / 2,
to 1e-6), FP64 and FP32 V-cycle, reported under "extension"; the corrector
mode (convection and streamline terms): its Stokes apply on the same mesh and
its solve on the 64^3 box, reported under "corrector".

Prints one JSON line (N = 1 only: the library runs the hot path on one GPU).
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
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def cell_kernel_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_2305_08986_amd", "csrc", "kernels_cell.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def algorithmic_bytes_per_cell(dim: int, elem: int) -> int:
    """Bytes one cell of the A-apply must move: per quadrature point 9 (4) values of
    det(J) w J^-1 plus 2 coefficients, the unique velocity dofs of the cell read
    and written once (2^dim nodes x dim components), and the int32 cell->node map."""
    q = 3 ** dim
    geo = (dim * dim + 2) * q * elem
    vec = 2 * (2 ** dim) * dim * elem
    cmap = 4 * q
    return geo + vec + cmap


def kernel_bytes_per_cell(dim: int, elem: int) -> int:
    """Bytes the A-only kernel itself must move per cell: it reads K' = sqrt(cvisc) K
    and cmass, (dim^2 + 1) values per point instead of (dim^2 + 2)."""
    q = 3 ** dim
    return (dim * dim + 1) * q * elem + 2 * (2 ** dim) * dim * elem + 4 * q


def load_counter_profile(workload: str, form: str = "phased"):
    """HBM traffic of the FP64 A apply from the committed rocprofv3 counter summary:
    per processing-phase launch of the default phased form, or per apply (the single
    launch and its initialisation kernel) of the atomic form."""
    tag = "" if form == "phased" else "atomic_"
    path = os.path.join(ROOT, "profiles", f"counters_cell3d_A_fp64_{tag}{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != cell_kernel_source_hash():
        return None
    return d


def extension_measure(name, mesh, d_disp, fsi, W, np, torch, rtol: float = 1e-6, reps: int = 3):
    """The pseudo-elastic extension on the same warped mesh (mu_A law, seeded wall data):
    flexible CG + multigrid to rtol 1e-6 (the paper's extension criterion), FP64 and FP32
    V-cycle, each after one untimed solve; median of ``reps`` timed solves."""
    ext = W.make_extension_inputs(name, mesh)
    ectx = fsi.Context.from_mesh(mesh)
    ectx.set_displacement(d_disp)
    for j in range(ectx.n_levels):
        mu = torch.from_numpy(ext.mu[j]).cuda()
        ectx.set_coefficients(j, torch.zeros_like(mu), 0.5 * mu)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ectx.setup()
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t0)
    g = torch.from_numpy(ext.g).cuda()
    res = {}
    sol = {}
    for label, prec in (("fp64", 0), ("mixed", 1)):
        ectx.set_mg_params(precision=prec)
        ectx.solve_extension(g, rtol=rtol, max_iter=200)
        times = []
        for _ in range(reps):
            u, info = ectx.solve_extension(g, rtol=rtol, max_iter=200)
            times.append(info["time_ms"])
        sol[label] = u
        res[label] = dict(ms=round(float(np.median(times)), 2), iters=info["iters"], rel_res=info["rel_res"],
                          status=info["status"])
    diff = float(torch.linalg.vector_norm(sol["mixed"] - sol["fp64"]) / torch.linalg.vector_norm(sol["fp64"]))
    return {"rtol": rtol, "setup_ms": round(setup_ms, 1), "fp64": res["fp64"], "mixed": res["mixed"],
            "speedup_mixed_vs_fp64": round(res["fp64"]["ms"] / res["mixed"]["ms"], 3),
            "rel_diff_mixed_vs_fp64": diff,
            "first_solve_builds_coarse_inverse": True}


def corrector_measure(name, ctx, W, np, torch, fsi, solve_workload: str = "C2", rtol: float = 1e-8):
    """Corrector mode (convection and streamline terms, Sec. 3.1.1 and 3.2): the Stokes
    apply with the terms on the bench workload's finest level (FP64 and FP32, median of
    timed applications), and the corrector solve (k_A = 6, BiCGStab Schur step) on the
    64^3 box to rtol 1e-8: plain FP64 path, optimised FP64 and mixed precision (the last
    two: the median of three solves)."""
    J = ctx.n_levels - 1
    sz = ctx.sizes(J)
    wl = W.make_workload(name, levels=[J])
    c = W.make_convection_inputs(name, wl.mesh, J, wl.eta[J])
    ctx.set_convection(J, c.vconv, c.r, c.rho)
    del wl
    n = sz["n_vel"] + sz["n_p"]
    _, o64, _ = ctx.time_operator(J, precision=0, mode=39, reps=10)
    _, o32, _ = ctx.time_operator(J, precision=1, mode=39, reps=10)
    _, op7, _ = ctx.time_operator(J, precision=0, mode=7, reps=10)
    out = {"apply": {"workload": name, "fp64_us": round(o64, 1), "fp64_gdofs": round(n / (o64 * 1e-6) / 1e9, 3),
                     "fp32_us": round(o32, 1), "fp32_gdofs": round(n / (o32 * 1e-6) / 1e9, 3),
                     "predictor_fp64_us": round(op7, 1),
                     "streamline_active_cells": float((c.r[:, 0] > 0).mean())}}
    wl = W.make_workload(solve_workload)
    cctx = fsi.Context.from_mesh(wl.mesh)
    fsi.setup_workload(cctx, wl)
    for j in range(cctx.n_levels):
        cj = W.make_convection_inputs(solve_workload, wl.mesh, j, wl.eta[j])
        cctx.set_convection(j, cj.vconv, cj.r, cj.rho)
    cctx.setup()
    cctx.autotune()
    cctx.set_mg_params(corrector=1, k_A=6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cctx.setup()
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t0)
    gu = torch.from_numpy(wl.g_u).cuda()
    gp = torch.from_numpy(wl.g_p).cuda()
    res = {}
    sol = {}
    # the tuned paths may add with atomics on some levels, and the mixed corrector
    # preconditioner's iteration count moves with rounding: median of three solves
    for label, prm, runs in (("plain_fp64", dict(precision=0, use_graph=0, fused=0, tuned=0), 1),
                             ("fp64", dict(precision=0), 3), ("mixed", dict(precision=1), 3)):
        cctx.set_mg_params(corrector=1, k_A=6, **prm)
        got = []
        for _ in range(runs):
            u, p, info = cctx.solve(gu, gp, rtol=rtol, max_iter=300)
            got.append((info["time_ms"], info, u))
        got.sort(key=lambda g: g[0])
        ms, info, u = got[len(got) // 2]
        sol[label] = u
        res[label] = dict(ms=round(ms, 1), iters=info["iters"], rel_res=info["rel_res"], status=info["status"])
        if runs > 1:
            res[label]["runs_ms"] = [round(g[0], 1) for g in got]
            res[label]["runs_iters"] = [g[1]["iters"] for g in got]
    du = float(torch.linalg.vector_norm(sol["mixed"] - sol["fp64"]) / torch.linalg.vector_norm(sol["fp64"]))
    out["solve"] = {"workload": solve_workload, "rtol": rtol, "k_A": 6, "setup_ms": round(setup_ms, 1), **res,
                    "speedup_mixed_vs_plain_fp64": round(res["plain_fp64"]["ms"] / res["mixed"]["ms"], 3),
                    "velocity_rel_diff_mixed_vs_fp64": du}
    return out


def cpu_baseline(seconds: float = 12.0):
    """The CPU oracle's A-apply (CSR SpMV, scipy) timed on a bounded sample."""
    import numpy as np
    from oracle import fem
    from paper_2305_08986_amd import workloads as W

    wl = W.make_workload("T3_16", levels=[2])
    box = fem.level_box(wl.mesh, 2)
    ref = fem.Reference(3)
    t0 = time.perf_counter()
    J = fem.jacobians_q1(box, wl.disp, ref)
    op = fem.assemble(box, J, wl.c_mass[2], wl.eta[2], ref)
    t_asm = time.perf_counter() - t0
    u = np.random.default_rng(0).uniform(-1, 1, box.n_vel)
    reps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        op.A @ u
        reps += 1
    dt = time.perf_counter() - t0
    gdofs = box.n_vel * reps / dt / 1e9
    return {
        "value": gdofs, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
        "sample": (f"FP64 CSR SpMV y = A u (scipy, single thread) of the oracle-assembled Q2 velocity block on a "
                   f"16^3 warped box with the same viscosity law (n_vel={box.n_vel}, nnz={op.A.nnz}); "
                   f"{reps} products in {dt:.1f} s; assembly {t_asm:.1f} s not included"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extension", action="store_true", help="skip the extension-solve measurement")
    ap.add_argument("--no-corrector", action="store_true", help="skip the corrector-mode measurement")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs the hot path on one GPU only (no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2305_08986_amd import fsi
    from paper_2305_08986_amd import workloads as W

    torch.cuda.set_device(0)
    name = args.workload
    _log(f"[bench] generating workload {name}")
    wl = W.make_workload(name)
    mesh = wl.mesh
    ctx = fsi.Context.from_mesh(mesh)
    J = ctx.n_levels - 1
    sz = ctx.sizes(J)
    nv, npr, nc = sz["n_vel"], sz["n_p"], sz["n_cells"]
    # inputs resident in HBM before timing
    d_disp = torch.from_numpy(wl.disp).cuda()
    d_cm = [torch.from_numpy(a).cuda() for a in wl.c_mass]
    d_eta = [torch.from_numpy(a).cuda() for a in wl.eta]
    gu = torch.from_numpy(wl.g_u).cuda()
    gp = torch.from_numpy(wl.g_p).cuda()
    del wl
    torch.cuda.synchronize()

    def do_setup():
        ctx.set_displacement(d_disp)
        for j in range(ctx.n_levels):
            ctx.set_coefficients(j, d_cm[j], d_eta[j])
        ctx.setup()

    _log("[bench] setup + autotune")
    do_setup()
    ctx.autotune()
    tuning = {f"L{j}": [ctx.tuning(j, 0)[0], ctx.tuning(j, 1)[0]] for j in range(ctx.n_levels)}

    def one_step(record):
        t0 = time.perf_counter()
        # the FP64 A apply in its default launch shape (one wavefront per row, streaming
        # geometry loads, four phase launches) and in the form the autotuner chose (on
        # the large 3D levels usually the single atomic launch)
        ctx.set_mg_params(tuned=0)
        k0_us, op0_us, nl0 = ctx.time_operator(J, precision=0, mode=1, reps=args.apply_reps)
        ctx.set_mg_params(tuned=1)
        k_us, op_us, nl = ctx.time_operator(J, precision=0, mode=1, reps=args.apply_reps)
        k32_us, op32_us, _ = ctx.time_operator(J, precision=1, mode=1, reps=max(4, args.apply_reps // 2))
        ks_us, ops_us, _ = ctx.time_operator(J, precision=0, mode=7, reps=max(4, args.apply_reps // 2))
        # FP32 A with the geometry formed from the vertex displacements in the kernel
        ctx.set_mg_params(vertex_geometry=1)
        kv_us, opv_us, _ = ctx.time_operator(J, precision=1, mode=1, reps=max(4, args.apply_reps // 2))
        ctx.set_mg_params(vertex_geometry=0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        do_setup()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # plain FP64: per-launch V-cycle, separate vector kernels, default launch shapes
        ctx.set_mg_params(precision=0, use_graph=0, fused=0, tuned=0)
        u64, p64, i64 = ctx.solve(gu, gp, rtol=args.rtol, max_iter=300, restart=100)
        # FP64 with every optimisation of the mixed path (graph, fused epilogues, tuned launches)
        ctx.set_mg_params(precision=0, use_graph=1, fused=1, tuned=1)
        uft, pft, ift = ctx.solve(gu, gp, rtol=args.rtol, max_iter=300, restart=100)
        ctx.set_mg_params(precision=1, use_graph=1, fused=1, tuned=1)
        umx, pmx, imx = ctx.solve(gu, gp, rtol=args.rtol, max_iter=300, restart=100)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        du = float(torch.linalg.vector_norm(umx - u64) / torch.linalg.vector_norm(u64))
        rec = dict(k_us=k_us, op_us=op_us, n_launch=nl, k0_us=k0_us, op0_us=op0_us, n_launch0=nl0, k32_us=k32_us, op32_us=op32_us, ks_us=ks_us, ops_us=ops_us,
                   opv_us=opv_us,
                   apply_s=t1 - t0, setup_s=t2 - t1, solve_s=t3 - t2, fp64=i64, fp64_opt=ift, mixed=imx, du=du,
                   step_s=t3 - t0)
        record.append(rec)
        _log(f"[bench] step: A-apply {op_us:.0f} us (cell kernel {k_us:.1f} us in {nl} launches), "
             f"setup {1e3*(t2-t1):.0f} ms, "
             f"plain fp64 solve {i64['time_ms']:.0f} ms/{i64['iters']} it ({i64['status']}), "
             f"optimised fp64 {ift['time_ms']:.0f} ms/{ift['iters']} it ({ift['status']}), "
             f"mixed {imx['time_ms']:.0f} ms/{imx['iters']} it ({imx['status']}), du {du:.2e}")

    warm = []
    for _ in range(args.warmup):
        one_step(warm)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    def mean(key, sub=None):
        vals = [r[key][sub] if sub else r[key] for r in recs]
        return float(np.mean(vals))

    op_us = mean("op_us")
    k_us = mean("k_us")
    gdofs = nv / (op_us * 1e-6) / 1e9
    n_launch = recs[-1]["n_launch"]
    tuned_var = tuning[f"L{J}"][0]
    atomic = tuned_var >= fsi.N_LAUNCH_VARIANTS
    op0_us, k0_us, n_launch0 = mean("op0_us"), mean("k0_us"), recs[-1]["n_launch0"]
    bpc = algorithmic_bytes_per_cell(mesh.dim, 8)
    # algorithmic bytes per launch / mean launch duration (k_us = all launches of one
    # apply; the atomic form: its one launch and the initialisation kernel)
    achieved = bpc * nc / (k_us * 1e-6) / 1e9
    kbpc = kernel_bytes_per_cell(mesh.dim, 8)
    # the counter summary must cover the measured form: the atomic one, or the default
    # phased variant
    prof = load_counter_profile(name, "atomic") if atomic else (load_counter_profile(name) if tuned_var == 0 else None)
    traffic = None
    flops = None
    if prof is not None:
        traffic = prof["hbm_bytes_per_launch"]
        if prof.get("fp64_flops_per_launch"):
            tf = prof["fp64_flops_per_launch"] / (k_us / n_launch * 1e-6) / 1e12
            flops = {"fp64_tflops": round(tf, 2), "peak": FP64_PEAK_TFLOPS, "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                     "source": "rocprofv3 SQ_INSTS_VALU_FMA/ADD/MUL_F64 per launch (profiles/)"}
    fp64_ms = mean("fp64", "time_ms")
    ft_ms = mean("fp64_opt", "time_ms")
    mx_ms = mean("mixed", "time_ms")
    out = {
        "metric": "Q2 matrix-free vmult GDoF/s; Stokes solve time to rel.res 1e-8, FP64 vs mixed",
        "value": round(gdofs, 4),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{name}: {W.CONFIGS[name]['desc']}, Q2-Q1, {ctx.n_levels} levels",
            "cells": nc, "n_vel": nv, "n_p": npr, "rtol": args.rtol,
            "mg": "FGMRES(100) + 1 V-cycle, k_A=4, m=2, k_S=n_S=1",
        },
        "apply": {
            "fp64_A_gdofs": round(gdofs, 4),
            "fp64_A_us": round(op_us, 1),
            "fp64_A_kernel_us": round(k_us, 2),
            "fp64_A_launches": n_launch,
            "fp64_A_mean_launch_us": round(k_us / n_launch, 2),
            "fp64_A_form": (f"single atomic launch over all phases (variant {tuned_var}) + output initialisation"
                            if atomic else f"phased, variant {tuned_var}"),
            "fp64_A_phased_default_gdofs": round(nv / (op0_us * 1e-6) / 1e9, 4),
            "fp64_A_phased_default_us": round(op0_us, 1),
            "fp64_A_phased_default_mean_launch_us": round(k0_us / n_launch0, 2),
            "fp64_A_phased_default_roofline_frac": round(bpc * nc / (k0_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "fp32_A_gdofs": round(nv / (mean("op32_us") * 1e-6) / 1e9, 4),
            "fp64_stokes_gdofs": round((nv + npr) / (mean("ops_us") * 1e-6) / 1e9, 4),
            "fp32_A_vertex_geometry_gdofs": round(nv / (mean("opv_us") * 1e-6) / 1e9, 4),
            "algorithmic_bytes_per_cell": bpc,
            "kernel_bytes_per_cell": kbpc,
        },
        "solve": {
            "fp64_plain_ms": round(fp64_ms, 1), "fp64_plain_iters": recs[-1]["fp64"]["iters"],
            "fp64_plain_rel_res": recs[-1]["fp64"]["rel_res"], "fp64_plain_status": recs[-1]["fp64"]["status"],
            "fp64_optimised_ms": round(ft_ms, 1), "fp64_optimised_iters": recs[-1]["fp64_opt"]["iters"],
            "mixed_graph_ms": round(mx_ms, 1), "mixed_iters": recs[-1]["mixed"]["iters"],
            "mixed_rel_res": recs[-1]["mixed"]["rel_res"], "mixed_status": recs[-1]["mixed"]["status"],
            "speedup_mixed_vs_plain_fp64": round(fp64_ms / mx_ms, 3),
            "speedup_mixed_vs_optimised_fp64": round(ft_ms / mx_ms, 3),
            "velocity_rel_diff_mixed_vs_fp64": recs[-1]["du"],
            "setup_ms": round(1e3 * mean("setup_s"), 1),
        },
        "tuning_variant": tuning,
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "achieved_kernel_bytes": round(kbpc * nc / (k_us * 1e-6) / 1e9, 1),
            "kernel": (("cell3d<double, A> as one atomic launch over all phases plus its output "
                        f"initialisation, autotuned; median apply {k_us:.1f} us (both kernels); traffic per apply")
                       if atomic else
                       (("cell3d<double, A>" if mesh.dim == 3 else "cell2d<double, A>")
                        + f" launch variant {tuned_var}, {n_launch} launches (processing phases) per apply, "
                        + f"median apply {k_us / n_launch:.1f} us per launch; traffic per launch")),
        },
        "flops": flops,
    }
    if not args.no_extension:
        _log("[bench] extension solve")
        out["extension"] = extension_measure(name, mesh, d_disp, fsi, W, np, torch)
    if not args.no_corrector:
        _log("[bench] corrector mode")
        out["corrector"] = corrector_measure(name, ctx, W, np, torch, fsi)
    if not args.no_cpu_baseline:
        _log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
