"""Solver runs for kernel traces: one FGMRES solve per configuration, or one GCSI time step.

    python -m paper_2305_08986_amd.solvebench --workload C3 --configs mixed,fp64,plain
    python -m paper_2305_08986_amd.solvebench --gcsi G2 [--inflow 1.0]

Before each timed solve (or the timed second step) a float32 torch fill of 2^23
elements runs alone on the device: in a kernel trace, the dispatches between two such
markers belong to one solve.  Prints one JSON line per solve.
"""
from __future__ import annotations

import argparse
import json
import sys

CONFIGS = {
    "mixed": dict(precision=1),
    "fp64": dict(precision=0),
    "plain": dict(precision=0, use_graph=0, fused=0, tuned=0),
}


def _marker(torch):
    torch.cuda.synchronize()
    torch.full((1 << 23,), 1.0, device="cuda", dtype=torch.float32)
    torch.cuda.synchronize()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--configs", default="mixed,fp64,plain")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--gcsi", default="", help="time one GCSI_2(P,C) step of this channel case instead")
    ap.add_argument("--inflow", type=float, default=1.0, help="inflow peak of the channel case")
    a = ap.parse_args(argv)

    import torch

    from . import fsi
    from . import workloads as W

    torch.cuda.set_device(0)
    if a.gcsi:
        from . import gcsi
        g = W.make_gcsi_inputs(a.gcsi, inflow=a.inflow)
        S = gcsi.Stepper(g, precision=fsi.PREC_MIXED, autotune=True)
        dev = lambda x: torch.from_numpy(x).cuda()
        args = ([dev(x) for x in g.u], [dev(x) for x in g.v], [dev(x) for x in g.w], dev(g.p))
        S.step(*args, rtol=a.rtol)
        _marker(torch)
        r = S.step(*args, rtol=a.rtol)
        print(json.dumps({"gcsi": a.gcsi, "step_ms": r["step_ms"],
                          "stages": [{k: v for k, v in s.items() if k != "u_hash"} for s in r["stages"]]}), flush=True)
        return
    wl = W.make_workload(a.workload)
    ctx = fsi.Context.from_mesh(wl.mesh)
    fsi.setup_workload(ctx, wl)
    ctx.setup()
    ctx.autotune()
    gu = torch.from_numpy(wl.g_u).cuda()
    gp = torch.from_numpy(wl.g_p).cuda()
    for name in a.configs.split(","):
        ctx.set_mg_params(**CONFIGS[name])
        u = torch.zeros_like(gu)
        p = torch.zeros_like(gp)
        _marker(torch)
        _, _, info = ctx.solve(gu, gp, u, p, rtol=a.rtol, max_iter=400)
        print(json.dumps({"workload": a.workload, "config": name, "iters": info["iters"],
                          "time_ms": info["time_ms"], "rel_res": info["rel_res"]}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
