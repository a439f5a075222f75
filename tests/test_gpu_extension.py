"""GPU extension solve (the pseudo-elastic extension Ext of Sec. 2) against the
oracle, through the C ABI.

* Small meshes: the flexible-CG + multigrid solution equals the oracle's direct
  solution of the boundary-value problem (FP64 V-cycle and FP32 V-cycle).
* Affine boundary data with constant mu on a warped mesh: the GPU solution is the
  affine field at every node (the discrete space holds it exactly).
* 96^3 with the mu_A law: converges in both precisions; sampled interior rows of the
  unconstrained operator vanish on the solution (oracle, cell by cell).
* Degenerate and error cases.
"""
import numpy as np
import pytest

from oracle import fem, solvers
from paper_2305_08986_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ext_ctx(name, faces=None, constant_mu=None, boundary_field=None, precision=0):
    from paper_2305_08986_amd import fsi
    wl = W.make_workload(name, dirichlet_faces=faces, levels=[])
    ext = W.make_extension_inputs(name, wl.mesh, constant_mu=constant_mu, boundary_field=boundary_field)
    ctx = fsi.Context.from_mesh(wl.mesh)
    ctx.set_displacement(wl.disp)
    for j in range(ctx.n_levels):
        ctx.set_coefficients(j, np.zeros_like(ext.mu[j]), 0.5 * ext.mu[j])
    ctx.set_mg_params(precision=precision)
    ctx.setup()
    return wl, ext, ctx


def _oracle(wl, ext):
    J = wl.mesh.n_levels - 1
    box = fem.level_box(wl.mesh, J)
    ref = fem.Reference(wl.mesh.dim)
    Jq = fem.jacobians_q1(box, wl.disp, ref)
    return solvers.extension_solve(box, Jq, ext.mu[J], ref, ext.g), box


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", ["T3_R", "T2_R", "T3_8"])
def test_extension_matches_oracle_direct_solve(name, prec):
    wl, ext, ctx = _ext_ctx(name, precision=prec)
    want, box = _oracle(wl, ext)
    g = torch.from_numpy(ext.g).cuda()
    u, info = ctx.solve_extension(g, rtol=1e-10, max_iter=200)
    print(name, prec, info["iters"], info["rel_res"])
    assert info["status"] == "OK" and info["rel_res"] <= 1e-10
    got = u.cpu().numpy()
    dm = box.dirichlet_vel_dofs()
    assert np.array_equal(got[dm], ext.g[dm])
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err <= 1e-8, err
    # the history starts at the zero-guess residual and ends at the reported value
    assert info["history"][0] == pytest.approx(1.0) and len(info["history"]) == info["iters"] + 1


def test_extension_reproduces_affine_field_on_warped_mesh():
    from tests.test_oracle_pins import _q2_node_displacement
    rng = np.random.default_rng(47)
    Bm = rng.uniform(-0.02, 0.02, (3, 3))
    c = rng.uniform(-0.01, 0.01, 3)
    wl0 = W.make_workload("T3_R", dirichlet_faces=63, levels=[])
    field = lambda X: Bm @ (X + _q2_node_displacement(wl0.mesh, wl0.disp)) + c[:, None]
    wl, ext, ctx = _ext_ctx("T3_R", faces=63, constant_mu=2.5, boundary_field=field)
    u, info = ctx.solve_extension(torch.from_numpy(ext.g).cuda(), rtol=1e-12, max_iter=200)
    want = field(W.velocity_node_coords(wl.mesh, wl.mesh.n_levels - 1)).ravel()
    err = np.abs(u.cpu().numpy() - want).max() / np.abs(want).max()
    assert info["status"] == "OK" and err <= 1e-9, (err, info["iters"])


def test_extension_full_size_96cube():
    """96^3 warped box, mu_A law, seeded boundary data: FP64 and mixed converge to 1e-6 and
    agree; sampled interior rows of A u (unconstrained operator) vanish relative to the
    boundary lifting."""
    wl, ext, ctx = _ext_ctx("C4")
    g = torch.from_numpy(ext.g).cuda()
    u64, i64 = ctx.solve_extension(g, rtol=1e-6, max_iter=100)
    ctx.set_mg_params(precision=1)
    u32, i32 = ctx.solve_extension(g, rtol=1e-6, max_iter=100)
    print("96^3 extension", i64["iters"], i64["time_ms"], i32["iters"], i32["time_ms"])
    assert i64["status"] == "OK" and i32["status"] == "OK"
    assert float(torch.linalg.vector_norm(u32 - u64) / torch.linalg.vector_norm(u64)) <= 1e-5
    J = wl.mesh.n_levels - 1
    box = fem.level_box(wl.mesh, J)
    free = fem.Box(box.dim, box.cells, box.extent, 0)       # no Dirichlet rows: A of the form
    rng = np.random.default_rng(53)
    dm = box.dirichlet_vel_dofs()
    # random interior rows, and rows of nodes next to the z = 0 wall (where the lifting acts)
    nx, ny, _ = box.vel_nodes
    ix = rng.integers(1, nx - 1, 30)
    iy = rng.integers(1, ny - 1, 30)
    comp = rng.integers(0, 3, 30)
    near = comp * box.n_vel_nodes + ix + nx * (iy + ny * 1)
    rows = np.unique(np.concatenate([rng.choice(np.nonzero(~dm)[0], 30, replace=False), near]))
    assert not dm[rows].any()
    u = u64.cpu().numpy()
    zero = np.zeros_like(ext.mu[J])
    ref = fem.Reference(3)
    au, _ = fem.apply_rows(free, wl.disp, zero, 0.5 * ext.mu[J], ref, u, None, rows, [])
    gw = np.where(dm, ext.g, 0.0)
    ag, _ = fem.apply_rows(free, wl.disp, zero, 0.5 * ext.mu[J], ref, gw, None, rows, [])
    assert np.abs(au).max() <= 1e-5 * np.abs(ag).max(), (np.abs(au).max(), np.abs(ag).max())


def test_extension_degenerate_and_error_cases():
    from paper_2305_08986_amd import fsi
    wl, ext, ctx = _ext_ctx("T3_4")
    n = len(ext.g)
    # zero boundary data: the extension vanishes, whatever the initial guess
    u, info = ctx.solve_extension(torch.zeros(n, dtype=torch.float64, device="cuda"),
                                  u=torch.ones(n, dtype=torch.float64, device="cuda"))
    assert info["status"] == "OK" and info["iters"] == 0 and float(u.abs().max()) == 0.0
    # max_iter 0 returns the initial guess with its residual
    u, info = ctx.solve_extension(torch.from_numpy(ext.g).cuda(), max_iter=0)
    assert info["status"] == "NOT_CONVERGED" and info["iters"] == 0 and info["rel_res"] == pytest.approx(1.0)
    g = torch.from_numpy(ext.g).cuda()
    bad = g.clone()
    bad[int(np.nonzero(ext.g)[0][0])] = float("nan")
    o = fsi.SolveOpts(rtol=1e-6, max_iter=10, restart=1, reorth=0)
    import ctypes as C
    st = ctx.raw_status("fsi_solve_extension", C.c_void_p(bad.data_ptr()), C.c_void_p(g.clone().data_ptr()),
                        C.byref(o), None)
    assert st == fsi.FSI_ERR_NONFINITE
    o.rtol = -1.0
    st = ctx.raw_status("fsi_solve_extension", C.c_void_p(g.data_ptr()), C.c_void_p(g.clone().data_ptr()),
                        C.byref(o), None)
    assert st == fsi.FSI_ERR_ARG
    ctx2 = fsi.Context.from_mesh(wl.mesh)
    o.rtol = 1e-6
    st = ctx2.raw_status("fsi_solve_extension", C.c_void_p(g.data_ptr()), C.c_void_p(g.clone().data_ptr()),
                         C.byref(o), None)
    assert st == fsi.FSI_ERR_STATE


def test_extension_graph_replays_equal_eager():
    """The captured extension preconditioner replayed over several solves, with eager
    work in between, gives the eager solve's result in both precisions."""
    wl, ext, ctx = _ext_ctx("T3_R")
    g = torch.from_numpy(ext.g).cuda()
    for prec in (0, 1):
        ctx.set_mg_params(precision=prec, use_graph=0)
        ue, ie = ctx.solve_extension(g, rtol=1e-10)
        ctx.set_mg_params(use_graph=1)
        for rep in range(3):
            ug, ig = ctx.solve_extension(g, rtol=1e-10)
            ctx.apply_A(ctx.n_levels - 1, ug)          # eager work between the replays
            torch.cuda.synchronize()
            assert ig["iters"] == ie["iters"], (prec, rep)
            assert float((ug - ue).abs().max()) <= 1e-14 * float(ue.abs().max()), (prec, rep)
