"""Failure handling through the C ABI, forced from host-side inputs (every
kernel still runs to completion)."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2305_08986_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx(name="T3_4"):
    from paper_2305_08986_amd import fsi
    wl = W.make_workload(name)
    return wl, fsi.Context.from_mesh(wl.mesh), fsi


def test_inverted_cell_is_reported():
    wl, ctx, fsi = _ctx()
    d = wl.disp.copy()
    # fold one interior vertex across its neighbour: det J < 0 in the adjacent cells
    pn = wl.mesh.p_nodes(ctx.n_levels - 1)
    v = 2 + pn[0] * (2 + pn[1] * 2)
    h = wl.mesh.extent[0] / wl.mesh.n_fine[0]
    d[0, v] += 2.5 * h
    with pytest.raises(fsi.FSIError) as e:
        ctx.set_displacement(d)
    assert e.value.status == fsi.FSI_ERR_INVERTED_CELL


def test_state_errors_before_setup():
    wl, ctx, fsi = _ctx()
    J = ctx.n_levels - 1
    u = torch.zeros(ctx.sizes(J)["n_vel"], dtype=torch.float64, device="cuda")
    with pytest.raises(fsi.FSIError) as e:
        ctx.apply_A(J, u)                      # no geometry yet
    assert e.value.status == fsi.FSI_ERR_STATE
    ctx.set_displacement(wl.disp)
    with pytest.raises(fsi.FSIError) as e:
        ctx.apply_A(J, u)                      # no coefficients yet
    assert e.value.status == fsi.FSI_ERR_STATE
    with pytest.raises(fsi.FSIError) as e:
        ctx.setup()
    assert e.value.status == fsi.FSI_ERR_STATE
    p = torch.zeros(ctx.sizes(J)["n_p"], dtype=torch.float64, device="cuda")
    with pytest.raises(fsi.FSIError) as e:
        ctx.solve(u, p)
    assert e.value.status == fsi.FSI_ERR_STATE


def test_argument_errors():
    wl, ctx, fsi = _ctx()
    assert ctx.raw_status("fsi_apply_A", 99, None, None) == fsi.FSI_ERR_ARG
    with pytest.raises(fsi.FSIError) as e:
        ctx.set_mg_params(k_S=2)
    assert e.value.status == fsi.FSI_ERR_ARG
    s = fsi.Sizes()
    assert ctx.lib.fsi_get_sizes(ctx.h, ctx.n_levels, ctypes.byref(s)) == fsi.FSI_ERR_ARG
    # launch variants and solve options out of range
    for lev, prec, var in ((ctx.n_levels, 0, 0), (0, 2, 0), (0, 0, fsi.N_LAUNCH_VARIANTS + len(fsi.ATOMIC_VARIANTS)), (0, 1, -1)):
        assert ctx.lib.fsi_set_tuning(ctx.h, lev, prec, var) == fsi.FSI_ERR_ARG
    # 2D levels have two atomic shapes
    c2 = fsi.Context.from_mesh(W.make_workload("T2_R").mesh)
    assert c2.lib.fsi_set_tuning(c2.h, 0, 0, fsi.N_LAUNCH_VARIANTS + len(fsi.ATOMIC_VARIANTS_2D)) == fsi.FSI_ERR_ARG
    assert c2.lib.fsi_set_tuning(c2.h, 0, 0, fsi.ATOMIC_VARIANTS_2D[-1]) == fsi.FSI_OK
    c2.close()
    fsi.setup_workload(ctx, wl)
    ctx.setup()
    gu = torch.from_numpy(wl.g_u).cuda()
    gp = torch.from_numpy(wl.g_p).cuda()
    for bad in (dict(reorth=3), dict(reorth=-1), dict(restart=0)):
        with pytest.raises(fsi.FSIError) as e:
            ctx.solve(gu, gp, **bad)
        assert e.value.status == fsi.FSI_ERR_ARG


def test_nonfinite_inputs_are_rejected():
    wl, ctx, fsi = _ctx()
    fsi.setup_workload(ctx, wl)
    J = ctx.n_levels - 1
    eta = wl.eta[J].copy()
    eta[3, 4] = np.nan
    with pytest.raises(fsi.FSIError) as e:
        ctx.set_coefficients(J, wl.c_mass[J], eta)
    assert e.value.status == fsi.FSI_ERR_NONFINITE
    ctx.set_coefficients(J, wl.c_mass[J], wl.eta[J])
    ctx.setup()
    g = torch.from_numpy(wl.g_u).cuda()
    g[5] = float("inf")
    with pytest.raises(fsi.FSIError) as e:
        ctx.solve(g, torch.from_numpy(wl.g_p).cuda())
    assert e.value.status == fsi.FSI_ERR_NONFINITE


def test_max_iter_returns_not_converged_with_iterate():
    wl, ctx, fsi = _ctx()
    fsi.setup_workload(ctx, wl)
    ctx.setup()
    gu = torch.from_numpy(wl.g_u).cuda()
    gp = torch.from_numpy(wl.g_p).cuda()
    u, p, info = ctx.solve(gu, gp, rtol=1e-12, max_iter=1)
    assert info["status"] == "NOT_CONVERGED" and info["iters"] == 1
    assert 0 < info["rel_res"] < 1.0
    assert torch.isfinite(u).all() and float(u.abs().max()) > 0
    # the returned rel_res is the true residual of the returned iterate
    v, q = ctx.apply_stokes(ctx.n_levels - 1, u, p)
    r = torch.cat([gu - v, gp - q])
    rr = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(torch.cat([gu, gp])))
    assert abs(rr - info["rel_res"]) <= 1e-10 + 1e-8 * rr


def test_zero_rhs_gives_zero_solution():
    wl, ctx, fsi = _ctx()
    fsi.setup_workload(ctx, wl)
    ctx.setup()
    gu = torch.zeros(len(wl.g_u), dtype=torch.float64, device="cuda")
    gp = torch.zeros(len(wl.g_p), dtype=torch.float64, device="cuda")
    u, p, info = ctx.solve(gu, gp, u=torch.ones_like(gu), p=torch.ones_like(gp))
    assert info["status"] == "OK" and info["iters"] == 0
    assert float(u.abs().max()) == 0.0 and float(p.abs().max()) == 0.0


def test_library_loaded_before_any_gpu_work_gives_a_working_context():
    """A fresh process that loads the library before torch has touched the GPU: the
    binding imports torch first, so both bind to torch's HIP runtime and the context
    is created (loaded the other way round, creation failed with FSI_ERR_HIP)."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_2305_08986_amd import fsi, workloads as W\n"
            "fsi.load_library()\n"
            "ctx = fsi.Context.from_mesh(W.make_workload('T3_4').mesh)\n"
            "print('create ok', ctx.n_levels, flush=True)\n")
    env = dict(os.environ, PYTHONPATH=root + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "create ok" in r.stdout, (r.returncode, r.stdout[-1000:], r.stderr[-2000:])
