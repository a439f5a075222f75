"""GPU parity of one GCSI_k(M_1, .., M_S) time step (Algorithm 1, Sec. 3.1.1) on the
channel-with-strip case G1 (16 x 4 x 4 cells, two levels) against the oracle's step
(oracle/gcsi.py: assembled operators, direct solves).

* the explicit displacement and its vertex values (rounding of one BDF combination);
* the right-hand sides g_vM and g_p of both modes, componentwise against the sum of
  magnitudes of every quadrature term: |g - g*|_i <= 64 u (|terms|)_i;
* the corrector-mode operator built from v# and w# (convective velocity at the Gauss
  points and the Peclet law on the finest and the next level), componentwise;
* the extension with the solid's cells fixed, against the direct solve;
* whole GCSI_2(P, C) and GCSI_1(P) steps, FP64 and mixed-precision V-cycles, against
  the oracle's step: every stage's velocity, mesh velocity and pressure and the
  recovered displacement.
"""
import numpy as np
import pytest

from oracle import fem
from oracle import gcsi as og
from paper_2305_08986_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
C_BOUND = 64


def _dev(x, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda", dtype=dtype or torch.float64).contiguous()


@pytest.fixture(scope="module")
def case():
    g = W.make_gcsi_inputs("G1")
    J = g.mesh.n_levels - 1
    ref = fem.Reference(3)
    pb = og.Problem(box=fem.level_box(g.mesh, J), ext_box=fem.level_box(g.ext_mesh, J),
                    solid_q=g.solid_q[J].astype(bool), solid_cells=g.solid_cells.astype(bool), mu_A=g.mu_A[J],
                    prm=og.Params(**g.material))
    st = og.State(u=g.u, v=g.v, w=g.w, p=g.p)
    out = og.step(pb, st, ("P", "C"), ref)
    return g, pb, st, ref, out


def _within(got, want, scale, what):
    err = np.abs(got - want)
    bound = C_BOUND * U64 * scale
    bad = err > bound
    worst = float(np.max(err / np.maximum(scale * U64, 1e-300)))
    print(f"{what}: worst |err| / (u scale) = {worst:.1f}")
    assert not np.any(bad), (what, int(bad.sum()), worst)


def _ctx(mesh):
    from paper_2305_08986_amd import fsi
    return fsi, fsi.Context.from_mesh(mesh)


def test_explicit_displacement_and_vertex_values(case):
    g, pb, st, ref, out = case
    fsi, ctx = _ctx(g.mesh)
    prm = fsi.GcsiParams.of(**g.material)
    J = g.mesh.n_levels - 1
    nvert = ctx.sizes(J)["n_vert"]
    u_out = torch.empty(pb.box.n_vel, device="cuda", dtype=torch.float64)
    disp = torch.empty(3 * nvert, device="cuda", dtype=torch.float64)
    ctx.gcsi_displacement(prm, _dev(g.w[0]), _dev(g.u[0]), _dev(g.u[1]), out=u_out, disp=disp)
    torch.cuda.synchronize()
    want = og.explicit_displacement(pb.prm, g.w[0], g.u)
    scale = pb.prm.gamma * pb.prm.tau * np.abs(g.w[0]) + sum(abs(a) * np.abs(x) for a, x in zip(pb.prm.alpha, g.u))
    _within(u_out.cpu().numpy(), want, scale, "u#")
    assert np.array_equal(disp.cpu().numpy().reshape(3, -1), og.vertex_values(pb.box, u_out.cpu().numpy()))
    ctx.close()


@pytest.mark.parametrize("mode", ["P", "C"])
def test_right_hand_side_matches_oracle(case, mode):
    g, pb, st, ref, out = case
    fsi, ctx = _ctx(g.mesh)
    prm = fsi.GcsiParams.of(**g.material)
    J = g.mesh.n_levels - 1
    uh = out["stages"][0 if mode == "P" else 1]["u_hash"]
    disp = og.vertex_values(pb.box, uh)
    want_u, want_p = og.rhs(pb.box, ref, pb.prm, mode, pb.solid_q, disp, uh, st)
    abs_u, abs_p = og.rhs(pb.box, ref, pb.prm, mode, pb.solid_q, disp, uh, st, absolute=True)
    g_u = torch.full((pb.box.n_vel,), np.nan, device="cuda", dtype=torch.float64)
    g_p = torch.full((pb.box.n_p,), np.nan, device="cuda", dtype=torch.float64)
    f = [_dev(x) for x in (g.u[0], g.u[1], g.v[0], g.v[1], g.w[0], g.w[1])]
    ctx.gcsi_rhs(prm, fsi.GCSI_PREDICTOR if mode == "P" else fsi.GCSI_CORRECTOR,
                 _dev(g.solid_q[J], torch.uint8), _dev(disp.ravel()), _dev(uh), *f, g_u, g_p)
    torch.cuda.synchronize()
    assert np.abs(want_p).max() > 0 and np.abs(want_u).max() > 0
    _within(g_u.cpu().numpy(), want_u, abs_u, f"g_u ({mode})")
    _within(g_p.cpu().numpy(), want_p, abs_p, f"g_p ({mode})")
    ctx.close()


def _inject(mesh, f, level):
    """Nodal values of a fine Q2 field at the nodes of ``level`` (same positions)."""
    J = mesh.n_levels - 1
    s = 1 << (J - level)
    nn = mesh.vel_nodes(J)
    return np.ascontiguousarray(f.reshape(3, nn[2], nn[1], nn[0])[:, ::s, ::s, ::s].reshape(-1))


def test_corrector_operator_from_the_step_fields_matches_oracle(case):
    g, pb, st, ref, out = case
    fsi, ctx = _ctx(g.mesh)
    prm = fsi.GcsiParams.of(**g.material)
    J = g.mesh.n_levels - 1
    uh = out["stages"][1]["u_hash"]
    vh, wh = out["stages"][0]["v"], out["stages"][0]["w"]
    disp = og.vertex_values(pb.box, uh)
    ctx.set_displacement(disp.ravel())
    ctx.gcsi_set_coefficients(prm, [_dev(x, torch.uint8) for x in g.solid_q])
    ctx.gcsi_set_convection(prm, _dev(vh), _dev(wh))
    rng = np.random.default_rng(17)
    for j in (J, J - 1):
        box = fem.level_box(g.mesh, j)
        dj = W.inject_displacement(g.mesh, disp, j)
        Jq = fem.jacobians_q1(box, dj, ref)
        cm, eta = og.coefficients(pb.prm, g.solid_q[j].astype(bool))
        vq, r = og.convection_inputs(box, ref, _inject(g.mesh, vh, j), _inject(g.mesh, wh, j), eta)
        op = fem.assemble(box, Jq, cm, eta, ref)
        A = op.A + fem.assemble_convection(box, Jq, vq, pb.prm.rho_f, r, ref)
        opa = fem.assemble(box, Jq, cm, eta, ref, absolute=True)
        Aa = opa.A + fem.assemble_convection(box, Jq, vq, pb.prm.rho_f, r, ref, absolute=True)
        x = rng.uniform(-1, 1, box.n_vel)
        x[op.dir_mask] = rng.uniform(-1, 1, int(op.dir_mask.sum()))
        y = rng.uniform(-1, 1, box.n_p)
        v, q = ctx.apply_corrector(j, _dev(x), _dev(y))
        torch.cuda.synchronize()
        _within(v.cpu().numpy(), A @ x + op.B.T @ y, Aa @ np.abs(x) + np.abs(opa.B.T) @ np.abs(y), f"(A+N+S) x level {j}")
        _within(q.cpu().numpy(), op.B @ x, np.abs(opa.B) @ np.abs(x), f"B x level {j}")
    ctx.close()


@pytest.mark.parametrize("launch", ["phased", 16, 17, 18, 19, 20])
def test_extension_with_fixed_solid_cells_matches_direct_solve(case, launch):
    """Also with the single atomic launch (every shape) pinned on every level: with fixed
    cells it reads the per-node wall mask, so the fixed nodes stay constrained."""
    g, pb, st, ref, out = case
    fsi, ctx = _ctx(g.ext_mesh)
    J = g.mesh.n_levels - 1
    ctx.set_fixed_cells(g.solid_cells)
    ctx.set_displacement(np.zeros(3 * ctx.sizes(J)["n_vert"]))
    for j in range(ctx.n_levels):
        ctx.set_coefficients(j, np.zeros_like(g.mu_A[j]), 0.5 * g.mu_A[j])
    ctx.setup()
    if launch != "phased":
        ctx.set_mg_params(tuned=1, atomics=1)
        for j in range(ctx.n_levels):
            for prec in (0, 1):
                ctx.set_tuning(j, prec, launch)
    v = np.random.default_rng(5).uniform(-1, 1, pb.box.n_vel)
    gv = torch.empty(pb.box.n_vel, device="cuda", dtype=torch.float64)
    ctx.fixed_values(_dev(v), gv)
    w, info = ctx.solve_extension(gv, rtol=1e-12, max_iter=300)
    torch.cuda.synchronize()
    want = og.extension(pb.ext_box, ref, pb.mu_A, v, og.fixed_nodes(pb.ext_box, pb.solid_cells))
    got = w.cpu().numpy()
    print("extension", info["iters"], info["rel_res"])
    assert info["status"] == "OK"
    fixed = np.tile(og.fixed_nodes(pb.ext_box, pb.solid_cells), 3)
    assert np.array_equal(got[fixed], v[fixed])
    assert np.linalg.norm(got - want) <= 1e-9 * np.linalg.norm(want)
    ctx.close()


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_gcsi2_pc_step_matches_oracle_step(case, precision):
    g, pb, st, ref, out = case
    from paper_2305_08986_amd import gcsi
    S = gcsi.Stepper(g, precision=precision)
    res = S.step([_dev(x) for x in g.u], [_dev(x) for x in g.v], [_dev(x) for x in g.w], _dev(g.p),
                 ("P", "C"), rtol=1e-12, ext_rtol=1e-12)
    for k, rec in enumerate(res["stages"]):
        print({a: b for a, b in rec.items() if a != "u_hash"})
        assert rec["status"] == "OK" and rec["ext_status"] == "OK"
    # per stage: the predictor's fields set the corrector's geometry and convection
    for k, (mode, want) in enumerate(zip(("P", "C"), out["stages"])):
        rec = res["stages"][k]
        assert _rel(rec["u_hash"].cpu().numpy(), want["u_hash"]) <= 1e-9, mode
    errs = {key: _rel(res[key].cpu().numpy(), out[key]) for key in ("u", "v", "w", "p")}
    print("relative max-norm differences", errs)
    for key, e in errs.items():
        assert e <= 1e-8, (key, e)
    S.close()


def test_gcsi1_predictor_step_matches_oracle_step(case):
    g, pb, st, ref, _ = case
    from paper_2305_08986_amd import gcsi
    mat = dict(g.material, k=1)
    pb1 = og.Problem(box=pb.box, ext_box=pb.ext_box, solid_q=pb.solid_q, solid_cells=pb.solid_cells, mu_A=pb.mu_A,
                     prm=og.Params(**mat))
    st1 = og.State(u=g.u[:1], v=g.v[:1], w=g.w[:1], p=g.p)
    want = og.step(pb1, st1, ("P",), ref)
    g1 = W.GcsiInputs(**{**g.__dict__, "material": mat})
    S = gcsi.Stepper(g1)
    res = S.step([_dev(g.u[0])], [_dev(g.v[0])], [_dev(g.w[0])], _dev(g.p), ("P",), rtol=1e-12, ext_rtol=1e-12)
    errs = {key: _rel(res[key].cpu().numpy(), want[key]) for key in ("u", "v", "w", "p")}
    print("GCSI_1(P)", errs)
    for key, e in errs.items():
        assert e <= 1e-8, (key, e)
    S.close()


def test_gcsi2_step_at_128x32x32_converges_and_keeps_its_invariants():
    """At the measured size (the oracle's direct solves do not reach it): every stage
    converges, the mesh velocity equals the velocity on the solid's nodes and vanishes on
    the other walls, no-slip rows stay zero, the displacement is the recovery formula of
    the final mesh velocity, and the mixed-precision step agrees with the FP64 one."""
    from paper_2305_08986_amd import gcsi
    g = W.make_gcsi_inputs("G2")
    J = g.mesh.n_levels - 1
    args = ([_dev(x) for x in g.u], [_dev(x) for x in g.v], [_dev(x) for x in g.w], _dev(g.p))
    res = {}
    for label, prec in (("fp64", 0), ("mixed", 1)):
        S = gcsi.Stepper(g, precision=prec, autotune=True)
        res[label] = S.step(*args, rtol=1e-10, ext_rtol=1e-10)
        S.close()
        for rec in res[label]["stages"]:
            print(label, {a: b for a, b in rec.items() if a != "u_hash"})
            assert rec["status"] == "OK" and rec["ext_status"] == "OK", rec
            assert rec["rel_res"] <= 1e-10 and rec["ext_rel_res"] <= 1e-10
    box, ebox = fem.level_box(g.mesh, J), fem.level_box(g.ext_mesh, J)
    fixed = np.tile(og.fixed_nodes(ebox, g.solid_cells.astype(bool)), 3)
    prm = og.Params(**g.material)
    for label, r in res.items():
        v, w, u = (r[k].cpu().numpy() for k in ("v", "w", "u"))
        assert np.array_equal(w[fixed], v[fixed]), label
        assert not np.any(w[ebox.dirichlet_vel_dofs() & ~fixed]), label
        assert not np.any(v[box.dirichlet_vel_dofs()]), label
        want = og.explicit_displacement(prm, w, g.u)
        scale = prm.gamma * prm.tau * np.abs(w) + sum(abs(a) * np.abs(x) for a, x in zip(prm.alpha, g.u))
        _within(u, want, scale, f"u^n ({label})")
    for key in ("v", "w", "u", "p"):
        a, b = res["mixed"][key].cpu().numpy(), res["fp64"][key].cpu().numpy()
        e = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        print("mixed vs fp64", key, e)
        assert e <= 1e-7, (key, e)


def test_time_step_entry_points_reject_bad_input(case):
    """Argument and state errors of the time-step and fixed-cell entry points (host-side
    checks; no kernel sees a bad input)."""
    import ctypes as C
    g, pb, st, ref, out = case
    fsi, ctx = _ctx(g.mesh)
    prm = fsi.GcsiParams.of(**g.material)
    z = torch.zeros(pb.box.n_vel, device="cuda", dtype=torch.float64)
    zp = torch.zeros(pb.box.n_p, device="cuda", dtype=torch.float64)
    sq = _dev(g.solid_q[-1], torch.uint8)
    vp = lambda t: C.c_void_p(None if t is None else t.data_ptr())
    for bad in (dict(k=3), dict(tau=0.0), dict(eta_f=0.0), dict(rho_s=-1.0), dict(mu_s=float("nan"))):
        b = fsi.GcsiParams.of(**{**g.material, **bad})
        assert ctx.raw_status("fsi_gcsi_displacement", C.byref(b), vp(z), vp(z), vp(z), vp(z), None) == fsi.FSI_ERR_ARG
    # k = 2 needs u^{n-2}; at least one output
    assert ctx.raw_status("fsi_gcsi_displacement", C.byref(prm), vp(z), vp(z), None, vp(z), None) == fsi.FSI_ERR_ARG
    assert ctx.raw_status("fsi_gcsi_displacement", C.byref(prm), vp(z), vp(z), vp(z), None, None) == fsi.FSI_ERR_ARG
    args = [vp(sq), vp(z), vp(z), vp(z), vp(z), vp(z), vp(z), vp(z), vp(z), vp(z), vp(zp)]
    assert ctx.raw_status("fsi_gcsi_rhs", C.byref(prm), 7, *args) == fsi.FSI_ERR_ARG           # mode
    bad = list(args)
    bad[7] = C.c_void_p(None)                                                                    # w1
    assert ctx.raw_status("fsi_gcsi_rhs", C.byref(prm), fsi.GCSI_PREDICTOR, *bad) == fsi.FSI_ERR_ARG
    assert ctx.raw_status("fsi_gcsi_rhs", C.byref(prm), fsi.GCSI_CORRECTOR, *bad) == fsi.FSI_OK   # w unused
    # the convection needs the time-step coefficients; fixed values need fixed cells
    assert ctx.raw_status("fsi_gcsi_set_convection", C.byref(prm), vp(z), vp(z)) == fsi.FSI_ERR_STATE
    assert ctx.raw_status("fsi_fixed_values", vp(z), vp(z)) == fsi.FSI_ERR_STATE
    # the lifting needs geometry and coefficients, the corrector terms in the corrector mode,
    # and finite data on the Dirichlet nodes
    assert ctx.raw_status("fsi_lift_dirichlet", vp(z), vp(z), vp(zp)) == fsi.FSI_ERR_STATE
    J = g.mesh.n_levels - 1
    ctx.set_displacement(np.zeros(3 * ctx.sizes(J)["n_vert"]))
    ctx.gcsi_set_coefficients(prm, [_dev(x, torch.uint8) for x in g.solid_q])
    bad_d = torch.zeros_like(z)
    bad_d[0] = float("nan")                      # node 0 is a wall node (corner)
    assert ctx.raw_status("fsi_lift_dirichlet", vp(bad_d), vp(z), vp(zp)) == fsi.FSI_ERR_NONFINITE
    assert ctx.raw_status("fsi_lift_dirichlet", vp(z), vp(z), vp(zp)) == fsi.FSI_OK
    ctx.set_mg_params(corrector=1, k_A=6)
    assert ctx.raw_status("fsi_lift_dirichlet", vp(z), vp(z), vp(zp)) == fsi.FSI_ERR_STATE
    torch.cuda.synchronize()
    ctx.close()
    # fixed cells: once, before the set-up; the block solve is refused when its coarse
    # matrix is singular
    fsi, ext = _ctx(g.ext_mesh)
    ext.set_fixed_cells(g.solid_cells)
    with pytest.raises(fsi.FSIError) as e:
        ext.set_fixed_cells(g.solid_cells)
    assert e.value.status == fsi.FSI_ERR_STATE
    ext.set_displacement(np.zeros(3 * ext.sizes(ext.n_levels - 1)["n_vert"]))
    for j in range(ext.n_levels):
        ext.set_coefficients(j, np.zeros_like(g.mu_A[j]), 0.5 * g.mu_A[j])
    ext.setup()
    with pytest.raises(fsi.FSIError) as e:
        ext.solve(z, zp)
    assert e.value.status == fsi.FSI_ERR_STATE
    # the single atomic launch reads the fixed nodes' wall bits: allowed with fixed cells
    assert ext.raw_status("fsi_set_tuning", ext.n_levels - 1, 0, 16) == fsi.FSI_OK
    ext.close()


@pytest.mark.parametrize("mode", ["P", "C"])
def test_lifted_right_hand_side_with_inflow_matches_oracle(case, mode):
    """fsi_gcsi_rhs followed by fsi_lift_dirichlet (inflow profile on x = 0) against the
    oracle's right-hand side and lifting, componentwise; the Dirichlet rows equal the data."""
    g0, pb, st, ref, out = case
    g = W.make_gcsi_inputs("G1", inflow=1.0)
    fsi, ctx = _ctx(g.mesh)
    prm = fsi.GcsiParams.of(**g.material)
    J = g.mesh.n_levels - 1
    st = og.State(u=g.u, v=g.v, w=g.w, p=g.p)
    uh = out["stages"][0 if mode == "P" else 1]["u_hash"]
    disp = og.vertex_values(pb.box, uh)
    ctx.set_displacement(disp.ravel())
    ctx.gcsi_set_coefficients(prm, [_dev(x, torch.uint8) for x in g.solid_q])
    Jq = fem.jacobians_q1(pb.box, disp, ref)
    cm, eta = og.coefficients(pb.prm, pb.solid_q)
    conv = None
    box0 = fem.Box(3, pb.box.cells, pb.box.extent, 0)
    if mode == "C":
        vh, wh = out["stages"][0]["v"], out["stages"][0]["w"]
        ctx.gcsi_set_convection(prm, _dev(vh), _dev(wh))
        ctx.set_mg_params(corrector=1, k_A=6)
        vq, r = og.convection_inputs(pb.box, ref, vh, wh, eta)
        conv = (vq, pb.prm.rho_f, r)
    want_u, want_p = og.rhs(pb.box, ref, pb.prm, mode, pb.solid_q, disp, uh, st)
    abs_u, abs_p = og.rhs(pb.box, ref, pb.prm, mode, pb.solid_q, disp, uh, st, absolute=True)
    want_u, want_p = og.lift_dirichlet(pb.box, ref, Jq, cm, eta, g.dirichlet, want_u, want_p, conv)
    dm = pb.box.dirichlet_vel_dofs()
    dw = np.abs(np.where(dm, g.dirichlet, 0.0))
    opa = fem.assemble(box0, Jq, cm, eta, ref, absolute=True)
    Aa = opa.A if conv is None else opa.A + fem.assemble_convection(box0, Jq, conv[0], conv[1], conv[2], ref,
                                                                      absolute=True)
    scale_u = abs_u + Aa @ dw + np.abs(want_u)
    scale_p = abs_p + opa.B @ dw + np.abs(want_p)
    g_u = torch.empty(pb.box.n_vel, device="cuda", dtype=torch.float64)
    g_p = torch.empty(pb.box.n_p, device="cuda", dtype=torch.float64)
    f = [_dev(x) for x in (g.u[0], g.u[1], g.v[0], g.v[1], g.w[0], g.w[1])]
    ctx.gcsi_rhs(prm, fsi.GCSI_PREDICTOR if mode == "P" else fsi.GCSI_CORRECTOR,
                 _dev(g.solid_q[J], torch.uint8), _dev(disp.ravel()), _dev(uh), *f, g_u, g_p)
    ctx.lift_dirichlet(_dev(g.dirichlet), g_u, g_p)
    torch.cuda.synchronize()
    gu = g_u.cpu().numpy()
    assert np.array_equal(gu[dm], g.dirichlet[dm])
    _within(gu, want_u, scale_u, f"lifted g_u ({mode})")
    _within(g_p.cpu().numpy(), want_p, scale_p, f"lifted g_p ({mode})")
    ctx.close()


def test_gcsi2_step_with_inflow_matches_oracle_step(case):
    """The channel driven by an inflow profile (and gravity): GCSI_2(P,C) on the GPU
    against the oracle's step with the same Dirichlet data."""
    g0, pb0, _, ref, _ = case
    from paper_2305_08986_amd import gcsi
    g = W.make_gcsi_inputs("G1", inflow=1.0)
    pb = og.Problem(box=pb0.box, ext_box=pb0.ext_box, solid_q=pb0.solid_q, solid_cells=pb0.solid_cells,
                    mu_A=pb0.mu_A, prm=og.Params(**g.material), dirichlet=g.dirichlet)
    want = og.step(pb, og.State(u=g.u, v=g.v, w=g.w, p=g.p), ("P", "C"), ref)
    S = gcsi.Stepper(g, precision=1)
    res = S.step([_dev(x) for x in g.u], [_dev(x) for x in g.v], [_dev(x) for x in g.w], _dev(g.p),
                 ("P", "C"), rtol=1e-12, ext_rtol=1e-12)
    S.close()
    v = res["v"].cpu().numpy()
    dm = pb.box.dirichlet_vel_dofs()
    assert np.allclose(v[dm], g.dirichlet[dm], rtol=0, atol=1e-9)
    errs = {key: _rel(res[key].cpu().numpy(), want[key]) for key in ("u", "v", "w", "p")}
    print("GCSI_2(P,C) with inflow", errs, [r["iters"] for r in res["stages"]])
    for key, e in errs.items():
        assert e <= 1e-8, (key, e)


def test_three_steps_with_inflow_match_the_oracle_run(case):
    """Three GCSI_2(P,C) steps with the history moved back after each (Algorithm 1's data),
    inflow and gravity, against the oracle's run."""
    g0, pb0, _, ref, _ = case
    from paper_2305_08986_amd import gcsi
    g = W.make_gcsi_inputs("G1", inflow=1.0)
    pb = og.Problem(box=pb0.box, ext_box=pb0.ext_box, solid_q=pb0.solid_q, solid_cells=pb0.solid_cells,
                    mu_A=pb0.mu_A, prm=og.Params(**g.material), dirichlet=g.dirichlet)
    st, _ = og.run(pb, og.State(u=g.u, v=g.v, w=g.w, p=g.p), 3, ("P", "C"), ref)
    S = gcsi.Stepper(g, precision=1)
    u, v, w, p, recs = S.run([_dev(x) for x in g.u], [_dev(x) for x in g.v], [_dev(x) for x in g.w], _dev(g.p),
                             3, rtol=1e-12, ext_rtol=1e-12)
    S.close()
    for i in range(2):
        errs = {key: _rel(got.cpu().numpy(), want) for key, got, want in
                (("u", u[i], st.u[i]), ("v", v[i], st.v[i]), ("w", w[i], st.w[i]))}
        print("history", i, errs)
        for key, e in errs.items():
            assert e <= 1e-8, (i, key, e)
    assert _rel(p.cpu().numpy(), st.p) <= 1e-8
    print("iterations", [[s["iters"] for s in r["stages"]] for r in recs])


@pytest.mark.parametrize("mode", ["P", "C"])
def test_right_hand_side_at_128x32x32_sampled_rows(mode):
    """The measured size: sampled rows of g_vM and g_p (nodes in the solid, on its boundary,
    next to the walls and the inflow face, and random ones) against the oracle summed over
    the cells around them, componentwise."""
    g = W.make_gcsi_inputs("G2", inflow=1.0)
    J = g.mesh.n_levels - 1
    box = fem.level_box(g.mesh, J)
    ref = fem.Reference(3)
    prm = og.Params(**g.material)
    st = og.State(u=g.u, v=g.v, w=g.w, p=g.p)
    uh = og.explicit_displacement(prm, g.w[0], g.u)
    disp = og.vertex_values(box, uh)
    sq = g.solid_q[J].astype(bool)
    rng = np.random.default_rng(23)
    vn = box.vel_nodes
    lex = lambda i, j, k: i + vn[0] * (j + vn[1] * k)
    solid_nodes = np.nonzero(og.fixed_nodes(box, g.solid_cells.astype(bool)))[0]
    nodes = np.unique(np.concatenate([
        rng.choice(box.n_vel_nodes, 24, replace=False), rng.choice(solid_nodes, 12, replace=False),
        [lex(1, 1, 1), lex(1, vn[1] // 2, vn[2] // 2), lex(vn[0] - 1, vn[1] // 2, vn[2] // 2),
         lex(vn[0] // 2, 1, vn[2] - 2), lex(vn[0] // 2, vn[1] - 2, 1)]]))
    pn = rng.choice(box.n_p, 16, replace=False)
    cells = np.unique(np.concatenate([box.cells_of_vel_node(int(n)) for n in nodes] +
                                     [box.cells_of_p_node(int(k)) for k in pn]))
    want_u, want_p = og.rhs(box, ref, prm, mode, sq, disp, uh, st, cells=cells)
    abs_u, abs_p = og.rhs(box, ref, prm, mode, sq, disp, uh, st, absolute=True, cells=cells)
    fsi, ctx = _ctx(g.mesh)
    gp_ = fsi.GcsiParams.of(**g.material)
    g_u = torch.empty(box.n_vel, device="cuda", dtype=torch.float64)
    g_p = torch.empty(box.n_p, device="cuda", dtype=torch.float64)
    f = [_dev(x) for x in (g.u[0], g.u[1], g.v[0], g.v[1], g.w[0], g.w[1])]
    ctx.gcsi_rhs(gp_, fsi.GCSI_PREDICTOR if mode == "P" else fsi.GCSI_CORRECTOR, _dev(g.solid_q[J], torch.uint8),
                 _dev(disp.ravel()), _dev(uh), *f, g_u, g_p)
    torch.cuda.synchronize()
    rows = np.concatenate([nodes + a * box.n_vel_nodes for a in range(3)])
    assert np.abs(want_u[rows]).max() > 0 and np.abs(want_p[pn]).max() > 0
    _within(g_u.cpu().numpy()[rows], want_u[rows], abs_u[rows], f"g_u rows ({mode}, 128x32x32)")
    _within(g_p.cpu().numpy()[pn], want_p[pn], abs_p[pn], f"g_p rows ({mode}, 128x32x32)")
    ctx.close()
