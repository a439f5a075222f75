"""Micro-benchmark of the matrix-free level operators (one workload, one level).

    python -m paper_2305_08986_amd.opbench --workload C3 --mode A --prec fp64 --reps 20

Times the fused cell kernel with HIP events (fsi_time_operator) and prints one
JSON line per (precision, launch variant) pair: --prec and --variant take
comma-separated lists, and a pinned --variant overrides the autotuner.  With --copy-calibration it also runs a plain elementwise copy kernel
(y = 1.0 * x, 2 GiB each way) first, which profiler counter runs use to scale
HBM byte counters.
"""
from __future__ import annotations

import argparse
import json
import sys

MODES = {"A": 1, "BT": 2, "B": 4, "stokes": 7, "cheb": 9, "res": 23, "convA": 33, "conv": 39}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--mode", default="A", choices=sorted(MODES))
    ap.add_argument("--prec", default="fp64", help="fp64, fp32 or a comma-separated list")
    ap.add_argument("--variant", default="", help="launch variant(s) 0..15 to pin, comma-separated")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--level", type=int, default=-1)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch variant")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--vertex-geometry", type=int, default=0,
                    help="fsi_mg_params.vertex_geometry: bit 0 FP32 kernels, bit 1 FP64 kernels")
    a = ap.parse_args(argv)

    import torch

    from . import fsi
    from . import workloads as W

    torch.cuda.set_device(0)
    out = {}
    if a.copy_calibration:
        n = 1 << 28                     # 2 GiB of doubles
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.mul(x, 1.0, out=y)        # an elementwise kernel: reads x once, writes y once
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out["copy_bytes_read"] = 8 * n
        out["copy_bytes_written"] = 8 * n
        out["copy_GBps"] = 16 * n / (ms * 1e-3) / 1e9
        del x, y
    wl = W.make_workload(a.workload)
    ctx = fsi.Context.from_mesh(wl.mesh)
    fsi.setup_workload(ctx, wl)
    lev = ctx.n_levels - 1 if a.level < 0 else a.level
    if MODES[a.mode] & 32:
        c = W.make_convection_inputs(a.workload, wl.mesh, lev, wl.eta[lev])
        ctx.set_convection(lev, c.vconv, c.r, c.rho)
    if a.vertex_geometry:
        ctx.set_mg_params(vertex_geometry=a.vertex_geometry)
    precs = [{"fp64": 0, "fp32": 1}[x] for x in a.prec.split(",")]
    variants = [int(v) for v in a.variant.split(",")] if a.variant else [None]
    if not a.no_autotune and variants == [None]:
        ctx.autotune()
    s = ctx.sizes(lev)
    for p in precs:
        for var in variants:
            if var is not None:
                ctx.set_tuning(lev, p, var)
            k_us, op_us, nl = ctx.time_operator(lev, precision=p, mode=MODES[a.mode], reps=a.reps)
            out.update(dict(workload=a.workload, level=lev, mode=a.mode, prec=["fp64", "fp32"][p], reps=a.reps,
                            vertex_geometry=a.vertex_geometry,
                            variant=ctx.tuning(lev, p)[0], n_cells=s["n_cells"], n_vel=s["n_vel"],
                            kernel_us=k_us, launches=nl, mean_launch_us=k_us / nl, operator_us=op_us,
                            gdofs=s["n_vel"] / (op_us * 1e-6) / 1e9))
            print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
