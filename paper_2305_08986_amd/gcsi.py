"""One GCSI_k(M_1, .., M_S) time step (Algorithm 1, Sec. 3.1.1) through the C ABI.

Per stage M (predictor P or corrector C) the library is called in the order of the
algorithm: the explicit displacement u# = gamma tau w# - sum_i alpha_i u^{n-i}
(fsi_gcsi_displacement, which also gives the vertex displacement of the new geometry),
the new geometry (fsi_set_displacement) and the coefficients of the stress splitting
(fsi_gcsi_set_coefficients), in the corrector stage the convective velocity
v° = v# - w# with the streamline parameter (fsi_gcsi_set_convection), the set-up of the
block V-cycle (fsi_setup), the right-hand side g_vM, g_p (fsi_gcsi_rhs, with nonzero
Dirichlet data such as an inflow profile lifted by fsi_lift_dirichlet), the FGMRES solve
from the last velocity and pressure (fsi_solve), and the extension w = Ext(v) on
a second context that fixes the solid's nodes (fsi_fixed_values, fsi_solve_extension);
then w# := w.  After the stages the displacement is recovered with the same splitting
from w^n.  This module orders the calls and holds the device buffers; every arithmetic
step runs in the HIP library.
"""
from __future__ import annotations

import time
from typing import Optional, Sequence

from . import fsi


class Stepper:
    """Two library contexts on one mesh: the generalized-Stokes system (walls and the
    outflow of the channel) and the extension (every face fixed, the solid's cells fixed,
    reference geometry, c_m = 0 and eta = mu_A / 2, set up once)."""

    def __init__(self, inputs, precision: int = fsi.PREC_FP64, autotune: bool = False, ext_precision=None,
                 reorth: int = 0, corrector_mg: Optional[dict] = None, **mg):
        import torch
        self.torch = torch
        self.inputs = inputs
        self.prm = fsi.GcsiParams.of(**inputs.material)
        self.mg = dict(precision=precision, **mg)
        # multigrid parameters of the corrector stage on top of those: Table 4's corrector
        # column (k_A = 6), and a wider Chebyshev interval, 2 lambda instead of 1.2 lambda: the
        # Lanczos estimate of the nonsymmetric corrector operator falls short of its spectrum
        # on the channel step (median corrector iterations 35 -> 17 over six advancing steps)
        self.corrector_mg = {**dict(k_A=6, cheb_upper=2.0), **(corrector_mg or {})}
        self.stokes = fsi.Context.from_mesh(inputs.mesh)
        self.ext = fsi.Context.from_mesh(inputs.ext_mesh)
        self.ext.set_fixed_cells(inputs.solid_cells)
        J = self.stokes.n_levels - 1
        self.J = J
        sz = self.stokes.sizes(J)
        self.nv, self.np, self.nvert = sz["n_vel"], sz["n_p"], sz["n_vert"]
        self.dim = inputs.mesh.dim
        dev = dict(device="cuda", dtype=torch.float64)
        self.ext.set_displacement(torch.zeros(self.dim * self.nvert, **dev))
        for j in range(self.ext.n_levels):
            mu = torch.as_tensor(inputs.mu_A[j], **dev)
            self.ext.set_coefficients(j, torch.zeros_like(mu), 0.5 * mu)
        self.ext.set_mg_params(precision=precision if ext_precision is None else ext_precision)
        self.ext.setup()
        if autotune:   # the extension's reference geometry never changes: tune its launches once
            self.ext.autotune()
        self.solid_q = [torch.as_tensor(x, device="cuda", dtype=torch.uint8).contiguous() for x in inputs.solid_q]
        # velocity data on the Dirichlet nodes of the Stokes system (an inflow profile), or none
        d = getattr(inputs, "dirichlet", None)
        self.dirichlet = None if d is None else torch.as_tensor(d, **dev).contiguous()
        self.u_hash = torch.empty(self.nv, **dev)
        self.disp = torch.empty(self.dim * self.nvert, **dev)
        self.g_u = torch.empty(self.nv, **dev)
        self.g_p = torch.empty(self.np, **dev)
        self.g_ext = torch.empty(self.nv, **dev)
        self.autotune = autotune
        self._tuned = set()
        self.reorth = reorth     # FGMRES Gram-Schmidt passes (fsi_solve_opts.reorth)

    def close(self):
        self.stokes.close()
        self.ext.close()

    def stage(self, mode: str, u1, u2, v1, v2, w1, w2, v_hash, w_hash, v0, p0, rtol, ext_rtol, max_iter):
        t = self.torch
        S, prm = self.stokes, self.prm
        S.gcsi_displacement(prm, w_hash, u1, u2, out=self.u_hash, disp=self.disp)
        S.set_displacement(self.disp)
        S.gcsi_set_coefficients(prm, self.solid_q)
        corr = mode == "C"
        S.set_mg_params(**{**self.mg, **(dict(corrector=1, **self.corrector_mg) if corr else dict(corrector=0))})
        if corr:
            S.gcsi_set_convection(prm, v_hash, w_hash)
        S.setup()
        if self.autotune and mode not in self._tuned:   # the corrector classes are tuned once their terms are set
            S.autotune()
            self._tuned.add(mode)
        S.gcsi_rhs(prm, fsi.GCSI_CORRECTOR if corr else fsi.GCSI_PREDICTOR, self.solid_q[self.J], self.disp,
                   self.u_hash, u1, u2, v1, v2, w1, w2, self.g_u, self.g_p)
        if self.dirichlet is not None:
            S.lift_dirichlet(self.dirichlet, self.g_u, self.g_p)
        v, p = v0.clone(), p0.clone()
        _, _, info = S.solve(self.g_u, self.g_p, v, p, rtol=rtol, max_iter=max_iter, reorth=self.reorth)
        self.ext.fixed_values(v, self.g_ext)
        w = w_hash.clone()
        _, einfo = self.ext.solve_extension(self.g_ext, w, rtol=ext_rtol, max_iter=max_iter)
        return v, p, w, dict(mode=mode, iters=info["iters"], rel_res=info["rel_res"], status=info["status"],
                             solve_ms=info["time_ms"], ext_iters=einfo["iters"], ext_rel_res=einfo["rel_res"],
                             ext_status=einfo["status"], ext_ms=einfo["time_ms"], u_hash=self.u_hash.clone())

    def step(self, u, v, w, p, modes: Sequence[str] = ("P", "C"), rtol: float = 1e-8, ext_rtol: float = 1e-6,
             max_iter: int = 300) -> dict:
        """u, v, w: [field at n-1, field at n-2] (device FP64, component-major); p: the last
        pressure.  Returns u^n, v^n, w^n, p^n and per-stage solver records."""
        t0 = time.perf_counter()
        u1, u2 = u[0], (u[1] if self.prm.k == 2 else None)
        v1, v2 = v[0], (v[1] if self.prm.k == 2 else None)
        w1, w2 = w[0], (w[1] if self.prm.k == 2 else None)
        w_hash, v_hash = w1, v1
        v_cur, p_cur = v1, p
        stages = []
        for mode in modes:
            v_cur, p_cur, w_hash, rec = self.stage(mode, u1, u2, v1, v2, w1, w2, v_hash, w_hash, v_cur, p_cur,
                                                   rtol, ext_rtol, max_iter)
            v_hash = v_cur
            stages.append(rec)
        u_new = self.torch.empty_like(u1)
        self.stokes.gcsi_displacement(self.prm, w_hash, u1, u2, out=u_new)
        self.torch.cuda.synchronize()
        return dict(u=u_new, v=v_cur, w=w_hash, p=p_cur, stages=stages,
                    step_ms=1e3 * (time.perf_counter() - t0))

    def run(self, u, v, w, p, n_steps: int, modes: Sequence[str] = ("P", "C"), rtol: float = 1e-8,
            ext_rtol: float = 1e-6, max_iter: int = 300):
        """n_steps steps; after each the history moves back by one step (u^{n-2} := u^{n-1},
        u^{n-1} := u^n, likewise v and w).  Returns the final (u, v, w, p) lists/tensor and the
        per-step records."""
        k = self.prm.k
        u, v, w = list(u)[:k], list(v)[:k], list(w)[:k]
        recs = []
        for _ in range(n_steps):
            r = self.step(u, v, w, p, modes, rtol, ext_rtol, max_iter)
            u = [r["u"]] + u[:k - 1]
            v = [r["v"]] + v[:k - 1]
            w = [r["w"]] + w[:k - 1]
            p = r["p"]
            recs.append(dict(step_ms=r["step_ms"], stages=r["stages"]))
        return u, v, w, p, recs
