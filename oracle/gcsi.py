"""ORACLE -- test infrastructure only (tests and the smoke check).  Never imported by
the product path.

Plain FP64 CPU version of one time step of the GCSI_k(M_1, .., M_S) scheme
(Algorithm 1, Sec. 3.1.1) on the structured box mesh of ``fem``:

* the BDF stencil of Sec. 3.1 (k = 1: gamma = 1, alpha_1 = -1; k = 2: gamma = 2/3,
  alpha_1 = -4/3, alpha_2 = 1/3);
* the explicit displacement u# = gamma tau w# - sum_i alpha_i u^{n-i} of the velocity
  splitting (Sec. 3.1.1), the same formula recovering u^n at the end of the step;
* the coefficients of the semi-implicit stress splitting: c_m = rho / (gamma tau), and
  eta = eta_f in the fluid, gamma tau mu_s in the solid;
* the right-hand sides g_vM (eq. form_g_j) and g_p (eq. form_g_p);
* the predictor and corrector convective velocities (the extrapolation of Sec. 3.1.1
  and v° = v# - w#) with the streamline parameter of Sec. 3.2;
* the stage loop: explicit step, new geometry, M-mode solve (direct), extension
  Ext(v) (Sec. 2, solved directly with the solid nodes fixed), w# := w;
* nonzero Dirichlet data (an inflow profile, Sec. 5 test problems) by lifting.

All fields are nodal arrays in the reference numbering of ``fem.Box``: the pull-back
u^{n,i} = u^{n-i} o A^{n-i} o (A^n)^{-1} of Sec. 3.1 has the same nodal values as
u^{n-i}, so the transported fields of the paper are the stored arrays, with their
gradients taken on the current (explicit) geometry.

Readings (where the paper is silent or misprinted):

* G1 (sign of the explicit solid stress).  Substituting the displacement
  u = gamma tau v - sum_i alpha_i u^{n,i} into the solid stress
  2 mu_s eps(u) - mu_s (grad u)^T grad u of the ALE weak form (Sec. 2.3) leaves the
  explicit part mu_s [-2 eps(sum_i alpha_i u^{n,i}) - (grad u#)^T grad u#]; the printed
  splitting has +2 eps(..).  The derivation is followed: with the printed sign the
  elastic term would push the solid away from its rest state (alpha_1 < 0).  Moved to
  the right-hand side it pairs with eps(v) (the stress is tested with eps(v)):
  g_vM gains (T, eps(v))_{Os#} with T = mu_s [2 eps(sum_i alpha_i u^{n,i})
  + (grad u#)^T grad u#].
* G2 (predictor convective velocity).  The k = 2 extrapolation is read as
  v° = 2 (v^{n,1} - w^{n,1}) - (v^{n,2} - w^{n,2}), the linear extrapolation of the
  relative velocity v - w (w# = w^{n-1} in the predictor stage); the printed second
  term carries w^{n,1}, which would convect the solid, where v = w.
* G3 (the predictor's convective term).  With v* and v° both explicit the whole term
  (rho (grad v*) v°, v) is known and moves to the right-hand side; the bilinear form is
  then the symmetric mass-plus-viscous form (as the paper notes).
* G4 (geometry).  The new geometry Id + u# is the multilinear map through the vertex
  values of the Q2 field u# (the map of ``fem.jacobians_q1``); gradients in eq.
  form_g_j are physical gradients on that geometry.  The volume correction uses the
  Q2 field itself: J# = det(I + grad-hat u#) at the Gauss points of the reference cell.
* G5 (body force and traction).  The body force is rho times a constant acceleration,
  rho = rho_s in the solid and rho_f in the fluid; the Neumann (outflow) traction is
  zero.
* G6 (density of the corrector convection).  The corrector's convection
  (rho (grad v) v°, w) takes rho_f: v° = v# - Ext(v#) vanishes on every node of a solid
  cell, so the solid density never multiplies a nonzero v°.
* G7 (extension).  Ext fixes every node of a solid cell (w = v there, Sec. 2: w = v_s
  in the solid) and the outer walls (w = 0), and solves (mu_A eps(w), eps(z)) = 0 on
  the fluid nodes, on the reference geometry.
* G8 (solid indicator).  The solid region is given per quadrature point (the
  coefficient sample of ``fem``); the density, viscosity, solid-stress and
  volume-correction integrands switch per point.

Pins: tests/test_oracle_gcsi.py (BDF exactness on polynomials in time, closed forms of
every right-hand-side term on affine geometry, the rigid translation and the uniformly
accelerated free solid reproduced exactly by a whole step, the hydrostatic state).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from . import fem, solvers

# BDF stencil of Sec. 3.1: order k -> (gamma, (alpha_1, .., alpha_k)), alpha_0 = 1
BDF = {1: (1.0, (-1.0,)), 2: (2.0 / 3.0, (-4.0 / 3.0, 1.0 / 3.0))}


@dataclass
class Params:
    k: int = 2
    tau: float = 0.005
    rho_f: float = 1e3
    rho_s: float = 1e4
    eta_f: float = 1.0
    mu_s: float = 5e5
    eta_V: float = 0.1            # 0 or inf: no volume correction
    body: tuple = (0.0, -2.0, 0.0)

    @property
    def gamma(self):
        return BDF[self.k][0]

    @property
    def alpha(self):
        return BDF[self.k][1]


@dataclass
class State:
    """History of Algorithm 1: u[i], v[i], w[i] hold u^{n-1-i}, .. (i < k); p the last
    pressure (the solver's initial guess only)."""
    u: List[np.ndarray]
    v: List[np.ndarray]
    w: List[np.ndarray]
    p: Optional[np.ndarray] = None


# ---------------------------------------------------------------- pointwise pieces
def explicit_displacement(prm: Params, w: np.ndarray, u_hist: Sequence[np.ndarray]) -> np.ndarray:
    """u = gamma tau w - sum_i alpha_i u^{n-i} (velocity splitting, Sec. 3.1.1; also the
    displacement recovery at the end of Algorithm 1)."""
    out = prm.gamma * prm.tau * w
    for a, ui in zip(prm.alpha, u_hist):
        out = out - a * ui
    return out


def vertex_values(box: fem.Box, f: np.ndarray) -> np.ndarray:
    """[dim][n_vert]: the Q2 nodal field at the mesh vertices (Q2 node (2i, 2j, 2k))."""
    vn = box.vel_nodes
    arr = f.reshape((box.dim,) + tuple(vn[::-1]))
    sl = (slice(None),) + tuple(slice(None, None, 2) for _ in range(box.dim))
    return np.ascontiguousarray(arr[sl].reshape(box.dim, -1))


def coefficients(prm: Params, solid_q: np.ndarray):
    """(c_m, eta) per quadrature point: rho / (gamma tau) and the viscosity of the stress
    splitting (eta_f in the fluid, gamma tau mu_s in the solid)."""
    gt = prm.gamma * prm.tau
    rho = np.where(solid_q, prm.rho_s, prm.rho_f)
    eta = np.where(solid_q, gt * prm.mu_s, prm.eta_f)
    return rho / gt, eta


def _cell_values(box: fem.Box, f: np.ndarray, cells: Optional[np.ndarray] = None):
    """[nc][dim][n_loc] local nodal values of a component-major Q2 field (of the given cells)."""
    vn = box.cell_vel_nodes(cells)
    F = f.reshape(box.dim, -1)
    return np.stack([F[a][vn] for a in range(box.dim)], axis=1)


def _phys_grad(fe: np.ndarray, G: np.ndarray):
    """[nc][Q][a][x] = d f_a / d x_x."""
    return np.einsum("cai,cqix->cqax", fe, G)


def rhs(box: fem.Box, ref: fem.Reference, prm: Params, mode: str, solid_q: np.ndarray,
        disp: np.ndarray, u_hash: np.ndarray, state: State, absolute: bool = False,
        cells: Optional[np.ndarray] = None):
    """(g_u, g_p) of the M-mode system (eq. form_g_j with readings G1-G5, eq. form_g_p).

      g_u(v) = (rho (body - (1/(gamma tau)) sum_i alpha_i v^{n,i}), v)_{O#}
               - [M = P] (rho (grad v*) v°, v)_{O#}                  (G3)
               + (T, eps(v))_{Os#}                                      (G1)
      g_p(q) = (-(1/eta_V) (J# - 1), q-hat)_{O-hat s}                   (G4)

    disp: vertex displacement of the explicit geometry O# = (Id + u#)(O-hat).  Rows of
    Dirichlet velocity dofs are zero.  absolute=True sums the magnitudes of every
    quadrature term instead (the rounding scale of any evaluation by this rule).  cells
    (lexicographic indices) restricts the sums to those cells: the rows of nodes whose cells
    are all among them are complete (sampled rows of large meshes)."""
    dim = box.dim
    if cells is not None:
        solid_q = solid_q[cells]
    J = fem.jacobians_q1(box, disp, ref, cells)
    Jinv, wdet = fem.geometry_factors(J, ref)
    G = np.einsum("cqbx,qib->cqix", Jinv, ref.dphi)               # physical basis gradients
    gt = prm.gamma * prm.tau
    rho = np.where(solid_q, prm.rho_s, prm.rho_f)                  # [nc][Q]
    al = prm.alpha
    V = [_cell_values(box, x, cells) for x in state.v]
    vsum = sum(a * x for a, x in zip(al, V))                        # sum_i alpha_i v^{n,i}
    body = np.asarray(prm.body, dtype=float)[None, None, :dim]
    U = [_cell_values(box, x, cells) for x in state.u]
    usum = sum(a * x for a, x in zip(al, U))
    uh = _cell_values(box, u_hash, cells)
    if mode == "P":
        W = [_cell_values(box, x, cells) for x in state.w]
        if prm.k == 1:
            vstar, vcirc = V[0], V[0] - W[0]
        else:
            vstar = 2.0 * V[0] - V[1]
            vcirc = 2.0 * (V[0] - W[0]) - (V[1] - W[1])             # G2
    if absolute:
        # every factor by its magnitude: the rounding scale of any evaluation by this rule
        phi, G, wdet, rho = np.abs(ref.phi), np.abs(G), np.abs(wdet), np.abs(rho)
        body = np.abs(body)
        vsum = sum(abs(a) * np.abs(x) for a, x in zip(al, V))
        usum = sum(abs(a) * np.abs(x) for a, x in zip(al, U))
        uh = np.abs(uh)
        if mode == "P":
            vstar = sum(np.abs(x) for x in V) * 2.0
            vcirc = 2.0 * sum(np.abs(x) for x in V + W)
    else:
        phi = ref.phi
    # value-paired integrand: F[c,q,a] multiplies phi_i e_a
    vval = np.einsum("qi,cai->cqa", phi, vsum)
    Fv = rho[..., None] * body + (rho / gt)[..., None] * (np.abs(vval) if absolute else -vval)
    if mode == "P":
        gv = _phys_grad(vstar, G)                                   # [c,q,a,x]
        vc = np.einsum("qi,cai->cqa", phi, vcirc)
        cv = np.einsum("cqax,cqx->cqa", gv, vc)
        Fv = Fv + rho[..., None] * (cv if absolute else -cv)
    # gradient-paired integrand (solid only): T[c,q,a,x] multiplies d_x phi_i e_a
    gs = _phys_grad(usum, G)
    gh = _phys_grad(uh, G)
    T2 = gs + np.swapaxes(gs, -1, -2)                               # 2 eps(sum alpha u)
    Tq = np.einsum("cqba,cqbx->cqax", gh, gh)                       # (grad u#)^T grad u#
    T = prm.mu_s * (T2 + Tq) * solid_q[..., None, None]
    ge = np.einsum("cq,cqa,qi->cai", wdet, Fv, phi) + np.einsum("cq,cqax,cqix->cai", wdet, T, G)
    g_u = np.zeros(box.n_vel)
    vnodes = box.cell_vel_nodes(cells)
    nn = box.n_vel_nodes
    for a in range(dim):
        np.add.at(g_u, vnodes + a * nn, ge[:, a, :])
    g_u[box.dirichlet_vel_dofs()] = 0.0
    g_p = volume_correction(box, ref, prm, solid_q, u_hash, absolute, cells)
    return g_u, g_p


def volume_correction(box: fem.Box, ref: fem.Reference, prm: Params, solid_q: np.ndarray,
                      u_hash: np.ndarray, absolute: bool = False, cells: Optional[np.ndarray] = None) -> np.ndarray:
    """g_p(q) = (-(1/eta_V) (J# - 1), q-hat) over the reference solid (eq. form_g_p):
    J# = det(I + grad-hat u#) of the Q2 field at the Gauss points, dx-hat = prod(h) w_q."""
    g_p = np.zeros(box.n_p)
    if not (prm.eta_V > 0 and math.isfinite(prm.eta_V)):
        return g_p
    h = box.h()
    gref = np.einsum("cai,qib->cqab", _cell_values(box, u_hash, cells), ref.dphi) / h[None, None, None, :]
    F = gref + np.eye(box.dim)[None, None]
    Jh = np.linalg.det(F)
    vol = np.prod(h) * ref.w                                          # [Q]
    s = -(1.0 / prm.eta_V) * (Jh - 1.0) * solid_q
    if absolute:
        s = (1.0 / prm.eta_V) * (np.abs(Jh) + 1.0) * solid_q
    ge = np.einsum("q,cq,qk->ck", vol, s, np.abs(ref.psi) if absolute else ref.psi)
    np.add.at(g_p, box.cell_p_nodes(cells), ge)
    return g_p


def _coth_minus_inv(pe: np.ndarray) -> np.ndarray:
    return 1.0 / np.tanh(pe) - 1.0 / pe


def convection_inputs(box: fem.Box, ref: fem.Reference, v_hash: np.ndarray, w_hash: np.ndarray,
                      eta: np.ndarray):
    """Corrector-mode terms of one level: v° = v# - w# at the Gauss points (physical
    components, interpolated with the Q2 basis) and the streamline parameter per cell of
    Sec. 3.2 (p1 = 2, h_K the cell diagonal, |v°|_K the largest point value, eta the
    cell mean): Pe_K = |v°|_K h_K / (2 eta p1), r = h_K / (2 |v°|_K p1)(coth Pe_K - 1/Pe_K)
    where Pe_K >= 1, else 0 (the same law as the corrector workloads)."""
    vc = _cell_values(box, v_hash - w_hash)
    vq = np.einsum("qi,cai->cqa", ref.phi, vc)
    hK = math.sqrt(float(np.sum(box.h() ** 2)))
    vmax = np.sqrt((vq ** 2).sum(axis=-1)).max(axis=1)
    mu = eta.mean(axis=1)
    p1 = 2.0
    pe = vmax * hK / (2.0 * mu * p1)
    r = np.zeros_like(pe)
    on = pe >= 1.0
    r[on] = hK / (2.0 * vmax[on] * p1) * _coth_minus_inv(pe[on])
    return vq, np.repeat(r[:, None], vq.shape[1], 1)


# ---------------------------------------------------------------- nonzero Dirichlet data
def lift_dirichlet(box: fem.Box, ref: fem.Reference, J: np.ndarray, c_mass: np.ndarray, eta: np.ndarray,
                   d: np.ndarray, g_u: np.ndarray, g_p: np.ndarray, conv=None):
    """Right-hand side of the constrained system for velocity data d on the Dirichlet dofs
    (an inflow profile): the unknown is split u = d_W + u_I, so the free rows lose the
    constrained columns applied to d, g_I - (A d_W)_I and g_p - B d_W, and the Dirichlet rows
    (identity) take d.  A and B are the unconstrained operators (with the corrector terms
    (vconv, rho, r) when conv is given).  Returns new arrays."""
    dm = box.dirichlet_vel_dofs()
    dw = np.where(dm, d, 0.0)
    op = fem.assemble_unconstrained(box, J, c_mass, eta, ref)
    A = op.A
    if conv is not None:
        b0 = fem.Box(box.dim, box.cells, box.extent, 0)
        A = A + fem.assemble_convection(b0, J, conv[0], conv[1], conv[2], ref)
    gu = np.where(dm, d, g_u - A @ dw)
    return gu, g_p - op.B @ dw


# ---------------------------------------------------------------- extension with fixed nodes
def fixed_nodes(box: fem.Box, solid_cells: np.ndarray) -> np.ndarray:
    """[n_vel_nodes] bool: nodes of solid cells (G7)."""
    m = np.zeros(box.n_vel_nodes, dtype=bool)
    m[box.cell_vel_nodes()[solid_cells].ravel()] = True
    return m


def extension(ext_box: fem.Box, ref: fem.Reference, mu: np.ndarray, v: np.ndarray,
              fixed: np.ndarray) -> np.ndarray:
    """w = Ext(v) of Sec. 2 (G7): w = v on the fixed nodes, 0 on the walls of ext_box,
    (mu eps(w), eps(z)) = 0 for z vanishing on both, on the reference geometry."""
    disp0 = np.zeros((ext_box.dim, ext_box.n_p))
    J = fem.jacobians_q1(ext_box, disp0, ref)
    g = np.where(np.tile(fixed, ext_box.dim), v, 0.0)
    return solvers.extension_solve(ext_box, J, mu, ref, g, fixed=np.tile(fixed, ext_box.dim))


# ---------------------------------------------------------------- the step
@dataclass
class Problem:
    box: fem.Box                  # Stokes box (walls and outflow of the channel)
    ext_box: fem.Box              # extension box (every face fixed)
    solid_q: np.ndarray           # [nc][Q] bool, finest level
    solid_cells: np.ndarray       # [nc] bool
    mu_A: np.ndarray              # [nc][Q] extension coefficient
    prm: Params = field(default_factory=Params)
    dirichlet: Optional[np.ndarray] = None   # velocity data on the Dirichlet dofs (inflow), else 0


def stage_system(pb: Problem, ref: fem.Reference, mode: str, u_hash: np.ndarray, state: State,
                 v_hash: Optional[np.ndarray] = None, w_hash: Optional[np.ndarray] = None):
    """Operator and right-hand side of the M-mode system of one stage."""
    box, prm = pb.box, pb.prm
    disp = vertex_values(box, u_hash)
    J = fem.jacobians_q1(box, disp, ref)
    cm, eta = coefficients(prm, pb.solid_q)
    op = fem.assemble(box, J, cm, eta, ref)
    conv = None
    if mode == "C":
        vq, r = convection_inputs(box, ref, v_hash, w_hash, eta)
        op.A = (op.A + fem.assemble_convection(box, J, vq, prm.rho_f, r, ref)).tocsr()
        conv = (vq, prm.rho_f, r)
    g_u, g_p = rhs(box, ref, prm, mode, pb.solid_q, disp, u_hash, state)
    if pb.dirichlet is not None:
        g_u, g_p = lift_dirichlet(box, ref, J, cm, eta, pb.dirichlet, g_u, g_p, conv)
    return op, g_u, g_p


def step(pb: Problem, state: State, modes: Sequence[str] = ("P", "C"),
         ref: Optional[fem.Reference] = None) -> dict:
    """One step of Algorithm 1: returns u^n, v^n, w^n, p^n and every stage's fields."""
    ref = ref or fem.Reference(pb.box.dim)
    prm = pb.prm
    fixed = fixed_nodes(pb.ext_box, pb.solid_cells)
    w_hash = state.w[0]
    v_hash = None
    stages = []
    for mode in modes:
        u_hash = explicit_displacement(prm, w_hash, state.u)
        op, g_u, g_p = stage_system(pb, ref, mode, u_hash, state, v_hash, w_hash)
        v, p = solvers.direct_solve(op, g_u, g_p)
        w = extension(pb.ext_box, ref, pb.mu_A, v, fixed)
        stages.append(dict(mode=mode, u_hash=u_hash, g_u=g_u, g_p=g_p, v=v, p=p, w=w))
        v_hash, w_hash = v, w
    u_new = explicit_displacement(prm, w_hash, state.u)
    return dict(u=u_new, v=v_hash, w=w_hash, p=stages[-1]["p"], stages=stages)


def run(pb: Problem, state: State, n_steps: int, modes: Sequence[str] = ("P", "C"),
        ref: Optional[fem.Reference] = None):
    """n_steps steps of Algorithm 1; after each the history moves back by one step
    (u^{n-2} := u^{n-1}, u^{n-1} := u^n, likewise v and w).  Returns the final state and the
    steps' outputs."""
    outs = []
    k = pb.prm.k
    for _ in range(n_steps):
        out = step(pb, state, modes, ref)
        state = State(u=[out["u"]] + state.u[:k - 1], v=[out["v"]] + state.v[:k - 1],
                      w=[out["w"]] + state.w[:k - 1], p=out["p"])
        outs.append(out)
    return state, outs
