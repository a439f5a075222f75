"""Time-step sequence of generalized-Stokes solves on a moving mesh (Sec. 3, Alg. 1).

    python -m paper_2305_08986_amd.sequence --workload C4 --steps 20

Every step advances the ALE displacement by a fresh smooth increment, redraws
the viscosity field and the right-hand side, recomputes geometry and
coefficients on all levels, rebuilds the preconditioner and solves to the
relative residual tolerance, starting from the previous step's solution.  Two
paths run on the same inputs, each warm-started from its own previous solution:

  * plain:  FP64 V-cycle launched kernel by kernel, separate vector kernels,
            default launch shapes;
  * mixed:  FP32 V-cycle as a captured HIP graph, fused epilogues where the
            autotuner measured them faster, tuned launch shapes.

The preconditioner setup is the same computation for both paths (it prepares
the FP64 and FP32 data at once); its time is counted in both totals.  Inputs are
generated on the host and copied to the device before the timed region of each
step.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def run(workload: str = "C4", steps: int = 20, rtol: float = 1e-8, restart: int = 100, max_iter: int = 400,
        log=None, keep_final: bool = False):
    """Run the sequence; with keep_final the last step's solutions of both paths are
    returned as host arrays under out["final"][path] = (u, p)."""
    import numpy as np
    import torch

    from . import fsi
    from . import workloads as W

    log = log or (lambda m: None)
    torch.cuda.set_device(0)
    disp = None
    ctx = None
    state = {}
    rec = []
    tune_s = None
    for n in range(1, steps + 1):
        wl = W.make_workload(workload, step=n, prev_disp=disp)
        disp = wl.disp
        if ctx is None:
            ctx = fsi.Context.from_mesh(wl.mesh)
        d_disp = torch.from_numpy(wl.disp).cuda()
        d_cm = [torch.from_numpy(a).cuda() for a in wl.c_mass]
        d_eta = [torch.from_numpy(a).cuda() for a in wl.eta]
        gu = torch.from_numpy(wl.g_u).cuda()
        gp = torch.from_numpy(wl.g_p).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.set_displacement(d_disp)
        for j in range(ctx.n_levels):
            ctx.set_coefficients(j, d_cm[j], d_eta[j])
        ctx.setup()
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        if tune_s is None:
            t0 = time.perf_counter()
            ctx.autotune()
            tune_s = time.perf_counter() - t0
        step = dict(step=n, setup_ms=1e3 * setup_s, eta_contrast=wl.info.get("eta_contrast"))
        for path, prm in (("plain", dict(precision=0, use_graph=0, fused=0, tuned=0)),
                          ("mixed", dict(precision=1, use_graph=1, fused=1, tuned=1))):
            ctx.set_mg_params(**prm)
            if path not in state:
                state[path] = (torch.zeros_like(gu), torch.zeros_like(gp))
            u, p = state[path]
            _, _, info = ctx.solve(gu, gp, u, p, rtol=rtol, max_iter=max_iter, restart=restart)
            step[path] = dict(iters=info["iters"], solve_ms=info["time_ms"], rel_res=info["rel_res"],
                              status=info["status"])
        du = float(torch.linalg.vector_norm(state["mixed"][0] - state["plain"][0])
                   / torch.linalg.vector_norm(state["plain"][0]))
        step["velocity_rel_diff"] = du
        rec.append(step)
        log(f"[sequence] step {n}: setup {step['setup_ms']:.0f} ms, plain {step['plain']['solve_ms']:.0f} ms/"
            f"{step['plain']['iters']} it, mixed {step['mixed']['solve_ms']:.0f} ms/{step['mixed']['iters']} it, "
            f"du {du:.2e}")
        del d_disp, d_cm, d_eta, wl

    def total(path):
        return sum(r["setup_ms"] + r[path]["solve_ms"] for r in rec)

    out = dict(workload=workload, steps=steps, rtol=rtol, restart=restart,
               n_vel=ctx.sizes(ctx.n_levels - 1)["n_vel"], n_p=ctx.sizes(ctx.n_levels - 1)["n_p"],
               autotune_ms=1e3 * tune_s,
               plain_total_ms=total("plain"), mixed_total_ms=total("mixed"),
               speedup_total=total("plain") / total("mixed"),
               setup_mean_ms=float(np.mean([r["setup_ms"] for r in rec])),
               plain_solve_mean_ms=float(np.mean([r["plain"]["solve_ms"] for r in rec])),
               mixed_solve_mean_ms=float(np.mean([r["mixed"]["solve_ms"] for r in rec])),
               plain_iters=[r["plain"]["iters"] for r in rec], mixed_iters=[r["mixed"]["iters"] for r in rec],
               max_velocity_rel_diff=max(r["velocity_rel_diff"] for r in rec),
               all_converged=all(r[p]["status"] == "OK" for r in rec for p in ("plain", "mixed")),
               per_step=rec)
    if keep_final:
        out["final"] = {k: (v[0].cpu().numpy(), v[1].cpu().numpy()) for k, v in state.items()}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="C4")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--rtol", type=float, default=1e-8)
    a = ap.parse_args(argv)
    out = run(a.workload, a.steps, a.rtol, log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(out), flush=True)
    return 0 if out["all_converged"] else 1


if __name__ == "__main__":
    sys.exit(main())
