"""Benchmark of the generalized-Stokes hot path on one MI355X.

Workload (default): the 128^3 warped box with log-uniform viscosity per 8^3
block (contrast up to 1e6), Q2-Q1, 6 levels down to 4^3, 50.9M velocity +
2.1M pressure dofs.

Before the W warm-up steps, applies run untimed for 0.3 s (reported as
config.prewarm): the GPU's clocks take tens of milliseconds of sustained load to
settle after the set-up's host-side pauses.

Timed region: K steps, each one application of the FP64 matrix-free operator
v = A u on the finest level (the hot-path kernel of every Krylov iteration and
smoothing step), in the launch form the autotuner chose for that level, with
u and v resident in HBM.  One pair of HIP events on the library stream (the
context is created on torch's current stream) brackets the K steps, and device
synchronisations bracket the loop.  `value` = N_vel * K / wall time, in GDoF/s;
the roofline's `achieved` divides the algorithmic bytes of one apply by the
events' mean apply time.

After the timed loop (reported, not timed as steps), each once and in a fixed
budget:
  * the same apply in its default phased launch form, FP32 A, the FP64 Stokes
    apply and the FP32 and FP64 applies with geometry formed from the vertices;
  * geometry + coefficient upload and preconditioner setup;
  * three solves from a zero guess to relative residual 1e-8: the plain FP64
    path (FP64 V-cycle launched kernel by kernel, separate Chebyshev/residual
    vector kernels, default launch shapes), the same FP64 solve with every
    optimisation (captured graph, fused epilogues where faster, tuned launch
    shapes), and the mixed-precision solve (FP32 V-cycle, FP64 FGMRES /
    residuals / Schur block; median of five, its iteration count moves with
    the order of the atomic adds);
  * the pseudo-elastic extension solve on the same mesh;
  * the corrector mode: its Stokes apply on the same mesh and its solve on the
    64^3 box;
  * the CPU oracle's element-by-element apply on a bounded sample of the same
    workload's cells, on every host core the box gives this job (run first, in
    a child process, before the GPU is touched).

Prints one JSON line (one GPU only: the library runs the hot path on one GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# untimed applies before the warm-up steps (seconds of sustained load)
PREWARM_S = 0.3
# worker processes of the CPU leg: the host cores a one-GPU job gets on the box
CPU_WORKERS_MAX = 16


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def cell_kernel_source_hash() -> str:
    """Hash of the sources of the kernels the counter summaries measure: the cell kernels
    and the initialisation (zero fill) of the atomic form."""
    h = hashlib.sha256()
    for name in ("kernels_cell.hip", "kernels_aux.hip"):
        with open(os.path.join(ROOT, "paper_2305_08986_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


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


def load_counter_profile(workload: str, form: str = "phased", prec: str = "fp64", variant=None):
    """HBM traffic of the A apply (FP64 or FP32) from the committed rocprofv3 counter
    summary: per processing-phase launch of the default phased form, or per apply (the
    single launch and its initialisation kernel) of the atomic form.  With `variant`,
    only a summary taken in that launch variant (the file of the form, or the one named
    for the variant)."""
    tag = "" if form == "phased" else "atomic_"
    names = [f"counters_cell3d_A_{prec}_{tag}{workload}.json"]
    if variant is not None:
        names.insert(0, f"counters_cell3d_A_{prec}_{tag}v{variant}_{workload}.json")
    for name in names:
        path = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(path):
            continue
        with open(path) as f:
            d = json.load(f)
        if d.get("kernel_source_sha256_16") != cell_kernel_source_hash():
            continue
        if variant is not None and d.get("variant") != variant:
            continue
        return d
    return None


# ---------------------------------------------------------------- CPU leg (oracle)
_CPU = {}


def _cpu_block(c0: int, c1: int):
    """One block of the oracle's element-by-element apply (a worker of the CPU leg)."""
    import numpy as np
    from oracle import fem
    g = _CPU
    d, v = fem.apply_ebe(g["box"], g["disp"], g["cm"], g["eta"], g["ref"], g["u"], np.arange(c0, c1))
    return c1 - c0, float(v @ g["u"][d])


def cpu_leg(name: str, seconds: float, block: int) -> dict:
    """The CPU oracle's A apply (fem.apply_ebe: element matrices by quadrature, local
    products, scatter) over consecutive blocks of the workload's finest-level cells,
    on a pool of worker processes, until the time budget is spent.  Runs in a process
    that never touches the GPU."""
    import multiprocessing as mp

    import numpy as np
    from oracle import fem
    from paper_2305_08986_amd import workloads as W

    mesh = W.make_mesh(name)
    J = mesh.n_levels - 1
    wl = W.make_workload(name, levels=[J])
    box = fem.level_box(wl.mesh, J)
    _CPU.update(box=box, disp=wl.disp, cm=wl.c_mass[J], eta=wl.eta[J], ref=fem.Reference(mesh.dim),
                u=np.random.default_rng(7).uniform(-1.0, 1.0, box.n_vel))
    ncell = box.n_cells
    workers = max(1, min(CPU_WORKERS_MAX, os.cpu_count() or 1))
    done = 0
    chk = 0.0
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        pending = []
        nxt = 0
        while True:
            while nxt < ncell and len(pending) < 2 * workers and time.perf_counter() - t0 < seconds:
                pending.append(pool.apply_async(_cpu_block, (nxt, min(ncell, nxt + block))))
                nxt += block
            if not pending:
                break
            n, c = pending.pop(0).get()
            done += n
            chk += c
        dt = time.perf_counter() - t0
    dof_per_cell = box.n_vel / ncell
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": done * dof_per_cell / dt / 1e9, "unit": "GDoF/s", "cores": workers, "kind": "oracle",
        "sample": (f"oracle element-by-element FP64 A apply (fem.apply_ebe: Gauss-quadrature element matrices, "
                   f"local products, scatter) on the first {done} of the {ncell} finest-level cells of the {name} "
                   f"workload, blocks of {block} cells over {workers} worker processes, {dt:.1f} s; GDoF/s = "
                   f"cells/s x N_vel/N_cells ({dof_per_cell:.2f})"),
        "nproc": os.cpu_count(), "cpu_model": model, "cells": done, "seconds": round(dt, 2),
        "checksum": chk,
    }


def run_cpu_leg_child(name: str, seconds: float) -> dict:
    """The CPU leg in a child process (single-threaded numpy per worker)."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", "--workload", name,
                        "--cpu-seconds", str(seconds)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=seconds + 240)
    if r.returncode != 0:
        raise RuntimeError(f"CPU leg failed: {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


# ---------------------------------------------------------------- GPU legs
def extension_measure(name, mesh, d_disp, fsi, W, np, torch, rtol: float = 1e-6):
    """The pseudo-elastic extension on the same warped mesh (mu_A law, seeded wall data):
    flexible CG + multigrid to rtol 1e-6 (the paper's extension criterion), FP64 and FP32
    V-cycle; the first solve of each builds the graphs, the second is timed."""
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
        u, info = ectx.solve_extension(g, rtol=rtol, max_iter=200)
        sol[label] = u
        res[label] = dict(ms=round(info["time_ms"], 2), iters=info["iters"], rel_res=info["rel_res"],
                          status=info["status"])
    diff = float(torch.linalg.vector_norm(sol["mixed"] - sol["fp64"]) / torch.linalg.vector_norm(sol["fp64"]))
    ectx.close()
    return {"rtol": rtol, "setup_ms": round(setup_ms, 1), "fp64": res["fp64"], "mixed": res["mixed"],
            "speedup_mixed_vs_fp64": round(res["fp64"]["ms"] / res["mixed"]["ms"], 3),
            "rel_diff_mixed_vs_fp64": diff}


def corrector_measure(name, ctx, W, np, torch, fsi, solve_workload: str = "C2", rtol: float = 1e-8):
    """Corrector mode (convection and streamline terms, Sec. 3.1.1 and 3.2): the Stokes
    apply with the terms on the bench workload's finest level (FP64 and FP32, median of
    timed applications), and the corrector solve (k_A = 6, BiCGStab Schur step) on the
    64^3 box to rtol 1e-8: plain FP64 path, optimised FP64 and mixed precision (the
    mixed one: median of three)."""
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
    # the 64^3 level's FP64 A apply in its autotuned form (the 64^3 row of the measurement plan)
    Jc = cctx.n_levels - 1
    _, a64_us, _ = cctx.time_operator(Jc, precision=0, mode=1, reps=20)
    nvc, ncc = cctx.sizes(Jc)["n_vel"], cctx.sizes(Jc)["n_cells"]
    out["apply_64cube"] = {"workload": solve_workload, "fp64_A_us": round(a64_us, 1),
                           "fp64_A_gdofs": round(nvc / (a64_us * 1e-6) / 1e9, 3),
                           "roofline_frac": round(algorithmic_bytes_per_cell(3, 8) * ncc / (a64_us * 1e-6) / 8e12, 4)}
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
    for label, prm, runs in (("plain_fp64", dict(precision=0, use_graph=0, fused=0, tuned=0), 1),
                             ("fp64", dict(precision=0), 1), ("mixed", dict(precision=1), 3)):
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
    du = float(torch.linalg.vector_norm(sol["mixed"] - sol["plain_fp64"]) /
               torch.linalg.vector_norm(sol["plain_fp64"]))
    cctx.close()
    out["solve"] = {"workload": solve_workload, "rtol": rtol, "k_A": 6, "setup_ms": round(setup_ms, 1), **res,
                    "speedup_mixed_vs_plain_fp64": round(res["plain_fp64"]["ms"] / res["mixed"]["ms"], 3),
                    "velocity_rel_diff_mixed_vs_fp64": du}
    return out


def gcsi_measure(W, torch, fsi, name: str = "G2", rtol: float = 1e-8, ext_rtol: float = 1e-6, steps: int = 5):
    """One GCSI_2(P, C) time step (Algorithm 1) on the channel with an elastic strip
    (128 x 32 x 32 cells, or its 1024 x 256 2D section for G2_2D), driven by an inflow
    profile of peak 1 (the FSI2-type inflow of Sec. 5) and gravity: explicit displacement,
    new geometry, coefficients, set-up,
    right-hand side, FGMRES (mixed precision) and the extension per stage, then the
    displacement recovery.  A first step tunes the launches and captures the graphs; then
    five steps are run from the same initial history, each moving the history back by one
    step, and the median step is reported."""
    from paper_2305_08986_amd import gcsi
    g = W.make_gcsi_inputs(name, inflow=1.0)
    S = gcsi.Stepper(g, precision=fsi.PREC_MIXED, autotune=True)
    dev = lambda x: torch.from_numpy(x).cuda()
    args = ([dev(x) for x in g.u], [dev(x) for x in g.v], [dev(x) for x in g.w], dev(g.p))
    S.step(*args, rtol=rtol, ext_rtol=ext_rtol)
    *_, recs = S.run(*args, steps, rtol=rtol, ext_rtol=ext_rtol)
    S.close()
    r = sorted(recs, key=lambda x: x["step_ms"])[len(recs) // 2]
    stages = [{k: (round(v, 2) if k.endswith("_ms") else v) for k, v in st.items() if k != "u_hash"}
              for st in r["stages"]]
    cells = g.mesh.n_cells(g.mesh.n_levels - 1)
    return {"workload": f"{name} channel with strip {'x'.join(map(str, g.mesh.n_fine))}, inflow peak 1", "cells": cells,
            "scheme": "GCSI_2(P,C)", "precision": "mixed", "rtol": rtol, "ext_rtol": ext_rtol, "steps": steps,
            "step_ms": round(r["step_ms"], 1), "steps_ms": [round(x["step_ms"], 1) for x in recs],
            "steps_iters": [[st["iters"] for st in x["stages"]] for x in recs], "median_step_stages": stages}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--mixed-runs", type=int, default=5, help="mixed solves (the median is reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solves", action="store_true", help="skip the three solves")
    ap.add_argument("--no-extension", action="store_true", help="skip the extension-solve measurement")
    ap.add_argument("--no-corrector", action="store_true", help="skip the corrector-mode measurement")
    ap.add_argument("--no-gcsi", action="store_true", help="skip the time-step (GCSI) measurement")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-block", type=int, default=512)
    ap.add_argument("--cpu-leg", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.cpu_leg:
        print(json.dumps(cpu_leg(args.workload, args.cpu_seconds, args.cpu_block)), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs the hot path on one GPU only (no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu_baseline:
        _log(f"[bench] CPU oracle baseline ({args.cpu_seconds:.0f} s budget, before any GPU work)")
        cpu = run_cpu_leg_child(args.workload, args.cpu_seconds)
        _log(f"[bench] CPU oracle: {cpu['value']:.5f} GDoF/s on {cpu['cores']} processes, {cpu['cells']} cells")

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
    t0 = time.perf_counter()
    do_setup()
    ctx.autotune()
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    tuning = {f"L{j}": [ctx.tuning(j, 0)[0], ctx.tuning(j, 1)[0]] for j in range(ctx.n_levels)}
    tuned_var = tuning[f"L{J}"][0]
    atomic = tuned_var >= fsi.N_LAUNCH_VARIANTS

    # ---------------- timed loop: K applications of v = A u (FP64, autotuned form)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    u = torch.rand(nv, dtype=torch.float64, device="cuda", generator=gen) * 2.0 - 1.0
    v = torch.empty_like(u)
    stream = torch.cuda.current_stream()
    assert stream.cuda_stream == ctx.stream.cuda_stream
    # the GPU's clocks take some tens of milliseconds of sustained load to settle after the
    # host-side pauses of the set-up (per-apply times fall by about 4% over the first
    # 50 ms): applies run for PREWARM_S before the warm-up steps, untimed, so that the
    # timed steps see the sustained state a solve runs in
    t0 = time.perf_counter()
    prewarm = 0
    while time.perf_counter() - t0 < PREWARM_S:
        for _ in range(10):
            ctx.apply_A(J, u, out=v)
        torch.cuda.synchronize()
        prewarm += 10
    prewarm_ms = 1e3 * (time.perf_counter() - t0)
    _log(f"[bench] timed loop: {prewarm} pre-warm applies ({prewarm_ms:.0f} ms), {args.warmup} warm-up + "
         f"{args.steps} FP64 A applies on {nc} cells")
    for _ in range(args.warmup):
        ctx.apply_A(J, u, out=v)
    torch.cuda.synchronize()
    # one HIP event pair on the library stream around the K steps: the average apply over
    # the timed region, without an event record between steps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for k in range(args.steps):
        ctx.apply_A(J, u, out=v)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    apply_us = 1e3 * e0.elapsed_time(e1) / args.steps
    gdofs = nv * args.steps / wall / 1e9
    _log(f"[bench] FP64 A apply: {apply_us:.1f} us mean (events), {1e3 * wall / args.steps:.3f} ms per step (wall), "
         f"{gdofs:.3f} GDoF/s")

    # ---------------- the other forms and operators (fsi_time_operator: medians)
    ctx.set_mg_params(tuned=0)
    k0_us, op0_us, nl0 = ctx.time_operator(J, precision=0, mode=1, reps=10)
    ctx.set_mg_params(tuned=1)
    k_us, op_us, nl = ctx.time_operator(J, precision=0, mode=1, reps=10)
    _, op32_us, _ = ctx.time_operator(J, precision=1, mode=1, reps=10)
    _, ops_us, _ = ctx.time_operator(J, precision=0, mode=7, reps=10)
    ctx.set_mg_params(vertex_geometry=3)
    _, opv_us, _ = ctx.time_operator(J, precision=1, mode=1, reps=10)
    _, opv64_us, _ = ctx.time_operator(J, precision=0, mode=1, reps=10)
    ctx.set_mg_params(vertex_geometry=0)

    bpc = algorithmic_bytes_per_cell(mesh.dim, 8)
    kbpc = kernel_bytes_per_cell(mesh.dim, 8)
    # algorithmic bytes of one apply / its mean duration over the timed steps (HIP events on
    # the library stream; the atomic form is its output zero fill plus one cell launch)
    achieved = bpc * nc / (apply_us * 1e-6) / 1e9
    prof = load_counter_profile(name, "atomic", "fp64", tuned_var) if atomic else load_counter_profile(name, "phased", "fp64", tuned_var)
    traffic = None
    flops = None
    if prof is not None:
        traffic = prof["hbm_bytes_per_launch"]
        if prof.get("fp64_flops_per_launch"):
            per = apply_us if atomic else apply_us / max(1, nl)
            tf = prof["fp64_flops_per_launch"] / (per * 1e-6) / 1e12
            flops = {"fp64_tflops": round(tf, 2), "peak": FP64_PEAK_TFLOPS, "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                     "source": "rocprofv3 SQ_INSTS_VALU_FMA/ADD/MUL_F64 per launch (profiles/)"}
    # the FP32 A apply of the V-cycle (median of timed applies in its tuned form): its own
    # roofline and, where the committed counter summary matches the tuned variant and the
    # kernel source, its HBM traffic and FP32 FLOP rate
    bpc32 = algorithmic_bytes_per_cell(mesh.dim, 4)
    var32 = tuning[f"L{J}"][1]
    prof32 = load_counter_profile(name, "atomic", "fp32", var32) if var32 >= fsi.N_LAUNCH_VARIANTS else None
    fp32_roof = {
        "bound": "hbm", "achieved": round(bpc32 * nc / (op32_us * 1e-6) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(bpc32 * nc / (op32_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_cell": bpc32,
        "apply_us": round(op32_us, 1), "variant": var32,
        "traffic": prof32["hbm_bytes_per_launch"] if prof32 else None,
        "fp32_tflops": (round(prof32["fp32_flops_per_launch"] / (op32_us * 1e-6) / 1e12, 2) if prof32 else None),
        "fp32_peak_tflops": FP32_PEAK_TFLOPS,
    }
    out = {
        "metric": "Q2 matrix-free vmult GDoF/s; Stokes solve time to rel.res 1e-8, FP64 vs mixed",
        "value": round(gdofs, 4),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{name}: {W.CONFIGS[name]['desc']}, Q2-Q1, {ctx.n_levels} levels",
            "step": "one FP64 matrix-free apply v = A u on the finest level (autotuned launch form)",
            "prewarm": {"applies": prewarm, "ms": round(prewarm_ms, 1),
                        "note": "untimed applies before the warm-up steps, until the clocks settle"},
            "cells": nc, "n_vel": nv, "n_p": npr, "rtol": args.rtol,
            "mg": "FGMRES(100) + 1 V-cycle, k_A=4, m=2, k_S=n_S=1",
        },
        "apply": {
            "fp64_A_gdofs": round(gdofs, 4),
            "fp64_A_event_us_mean": round(apply_us, 2),
            "fp64_A_form": (f"output initialisation + one atomic cell launch over all phases (variant {tuned_var})"
                            if atomic else f"phased, variant {tuned_var}, {nl} launches"),
            "fp64_A_timeop_kernel_us": round(k_us, 2),
            "fp64_A_timeop_us": round(op_us, 2),
            "fp64_A_phased_default_gdofs": round(nv / (op0_us * 1e-6) / 1e9, 4),
            "fp64_A_phased_default_us": round(op0_us, 1),
            "fp64_A_phased_default_mean_launch_us": round(k0_us / max(1, nl0), 2),
            "fp64_A_phased_default_roofline_frac": round(bpc * nc / (k0_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "fp32_A_gdofs": round(nv / (op32_us * 1e-6) / 1e9, 4),
            "fp32_A_roofline": fp32_roof,
            "fp64_stokes_gdofs": round((nv + npr) / (ops_us * 1e-6) / 1e9, 4),
            "fp32_A_vertex_geometry_gdofs": round(nv / (opv_us * 1e-6) / 1e9, 4),
            "fp64_A_vertex_geometry_gdofs": round(nv / (opv64_us * 1e-6) / 1e9, 4),
            "algorithmic_bytes_per_cell": bpc,
            "kernel_bytes_per_cell": kbpc,
        },
        "tuning_variant": tuning,
        "setup_autotune_s": round(tune_s, 2),
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "achieved_kernel_bytes": round(kbpc * nc / (apply_us * 1e-6) / 1e9, 1),
            "frac_kernel_bytes": round(kbpc * nc / (apply_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "kernel": (("cell3d<double, A> as one atomic launch over all phases, with its output initialisation, "
                        f"autotuned; mean apply {apply_us:.1f} us over the timed steps; traffic per apply")
                       if atomic else
                       (("cell3d<double, A>" if mesh.dim == 3 else "cell2d<double, A>")
                        + f" launch variant {tuned_var}, {nl} launches per apply, mean apply {apply_us:.1f} us")),
        },
        "flops": flops,
    }
    print(json.dumps({"partial": "timed loop done", "value": out["value"], "roofline_frac": out["roofline"]["frac"]}),
          file=sys.stderr, flush=True)

    if not args.no_solves:
        _log("[bench] setup (timed once)")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        do_setup()
        torch.cuda.synchronize()
        setup_ms = 1e3 * (time.perf_counter() - t1)
        solves = {}
        _log("[bench] plain FP64 solve")
        ctx.set_mg_params(precision=0, use_graph=0, fused=0, tuned=0)
        u64, p64, i64 = ctx.solve(gu, gp, rtol=args.rtol, max_iter=300, restart=100)
        _log(f"[bench]   {i64['time_ms']:.0f} ms, {i64['iters']} it, {i64['status']}")
        _log("[bench] optimised FP64 solve")
        ctx.set_mg_params(precision=0, use_graph=1, fused=1, tuned=1)
        uft, pft, ift = ctx.solve(gu, gp, rtol=args.rtol, max_iter=300, restart=100)
        _log(f"[bench]   {ift['time_ms']:.0f} ms, {ift['iters']} it, {ift['status']}")
        ctx.set_mg_params(precision=1, use_graph=1, fused=1, tuned=1)
        mixed = []
        for r in range(max(1, args.mixed_runs)):
            _log(f"[bench] mixed solve {r + 1}/{args.mixed_runs}")
            umx, pmx, imx = ctx.solve(gu, gp, rtol=args.rtol, max_iter=300, restart=100)
            du = float(torch.linalg.vector_norm(umx - u64) / torch.linalg.vector_norm(u64))
            dp = float(torch.linalg.vector_norm(pmx - p64) / torch.linalg.vector_norm(p64))
            mixed.append((imx["time_ms"], imx, du, dp))
            _log(f"[bench]   {imx['time_ms']:.0f} ms, {imx['iters']} it, {imx['status']}, du {du:.2e}")
        mixed.sort(key=lambda m: m[0])
        mx_ms, imx, du, dp = mixed[len(mixed) // 2]
        solves = {
            "fp64_plain_ms": round(i64["time_ms"], 1), "fp64_plain_iters": i64["iters"],
            "fp64_plain_rel_res": i64["rel_res"], "fp64_plain_status": i64["status"],
            "fp64_optimised_ms": round(ift["time_ms"], 1), "fp64_optimised_iters": ift["iters"],
            "fp64_optimised_rel_res": ift["rel_res"],
            "mixed_graph_ms": round(mx_ms, 1), "mixed_iters": imx["iters"],
            "mixed_rel_res": imx["rel_res"], "mixed_status": imx["status"],
            "mixed_runs_ms": [round(m[0], 1) for m in mixed], "mixed_runs_iters": [m[1]["iters"] for m in mixed],
            "speedup_mixed_vs_plain_fp64": round(i64["time_ms"] / mx_ms, 3),
            "speedup_mixed_vs_optimised_fp64": round(ift["time_ms"] / mx_ms, 3),
            "velocity_rel_diff_mixed_vs_fp64": du,
            "velocity_rel_diff_mixed_vs_fp64_max": max(m[2] for m in mixed),
            "pressure_rel_diff_mixed_vs_fp64": dp,
            "setup_ms": round(setup_ms, 1),
        }
        out["solve"] = solves
        del u64, p64, uft, pft, umx, pmx
    if not args.no_extension:
        _log("[bench] extension solve")
        out["extension"] = extension_measure(name, mesh, d_disp, fsi, W, np, torch)
    if not args.no_corrector:
        _log("[bench] corrector mode")
        out["corrector"] = corrector_measure(name, ctx, W, np, torch, fsi)
        out["apply_64cube"] = out["corrector"].pop("apply_64cube")
    if not args.no_gcsi:
        _log("[bench] GCSI_2(P,C) time step")
        out["gcsi_step"] = gcsi_measure(W, torch, fsi)
        out["gcsi_step_2d"] = gcsi_measure(W, torch, fsi, name="G2_2D")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
