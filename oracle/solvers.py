"""ORACLE -- test infrastructure only.  Never imported by the product path.

Plain FP64 CPU versions of the solver pieces of Sec. 4 on assembled CSR
level matrices:

* Chebyshev smoother Cheb(A, diag A, k) with zero initial guess (Sec. 4,
  definition of A-hat^{-1}; the recurrence is the classical Chebyshev
  iteration for D^{-1}A on [lo, hi]);
* ChebMINRES(n_S=1, k_S=1) for S = B A-hat^{-1} B^T (Sec. 4): one MINRES step
  from zero, preconditioned by one Chebyshev step on diag(B diag(A)^{-1} B^T),
  i.e. a scaled Jacobi step whose scale cancels;
* the block smoother K_j (Sec. 4, smoother definition) applied through its
  block-triangular factorisation;
* nested-space transfers (prolongation = evaluation of the coarse FE function
  at the fine nodes, restriction = transpose), built from the basis functions;
* n V-cycles with m pre- and m post-smoothing steps (Sec. 4), dense LU on the
  coarsest level;
* right-preconditioned flexible GMRES (Sec. 5, linear solver settings);
* Lanczos estimate of lambda_max(D^{-1}A) for the Chebyshev interval;
* the pseudo-elastic extension Ext of Sec. 2 (its defining boundary-value
  problem, solved directly).
Defaults follow Table 4 (predictor column): k_A=4, m=2, n=1, k_S=1, n_S=1.

Readings where the paper is silent (interval, eigenvalue estimate, start
vector, restart length) are stated at each function.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


# ---------------------------------------------------------------- direct solve
def direct_solve(op: fem.Operator, g_u: np.ndarray, g_p: np.ndarray):
    """Exact solution of [[A, B^T], [B, 0]] [u; p] = [g_u; g_p] (SuperLU)."""
    M = op.stokes().tocsc()
    lu = spla.splu(M)
    g = np.concatenate([g_u, g_p])
    x = lu.solve(g)
    for _ in range(3):                       # iterative refinement in FP64
        x = x + lu.solve(g - M @ x)
    return x[: op.box.n_vel], x[op.box.n_vel:]


# ---------------------------------------------------------------- eigenvalue estimate
def lanczos_start_vector(n: int) -> np.ndarray:
    """Deterministic start vector v_i = ((7919*i) mod 1021)/1021 - 1/2.

    The paper does not state how the Chebyshev interval is estimated; a fixed
    integer formula keeps the estimate reproducible without random draws.
    """
    i = np.arange(n, dtype=np.int64)
    return ((7919 * i) % 1021).astype(np.float64) / 1021.0 - 0.5


def lanczos_lambda_max(A: sp.spmatrix, diag: np.ndarray, free: np.ndarray, steps: int = 12):
    """Largest Ritz value of D^{-1/2} A D^{-1/2} after ``steps`` Lanczos steps.

    Start vector: ``lanczos_start_vector`` with constrained entries zeroed.
    Returns (lambda, alphas, betas).
    """
    s = 1.0 / np.sqrt(diag)
    v = lanczos_start_vector(A.shape[0]) * free
    v = v / np.linalg.norm(v)
    vprev = np.zeros_like(v)
    alphas, betas = [], []
    beta = 0.0
    for j in range(steps):
        w = s * (A @ (s * v))
        alpha = float(w @ v)
        w = w - alpha * v - beta * vprev
        alphas.append(alpha)
        beta = float(np.linalg.norm(w))
        if j == steps - 1 or beta <= 1e-300:
            break
        betas.append(beta)
        vprev, v = v, w / beta
    T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    lam = float(np.linalg.eigvalsh(T)[-1])
    return lam, np.array(alphas), np.array(betas)


# ---------------------------------------------------------------- Chebyshev
def chebyshev(apply_A: Callable, dinv: np.ndarray, r: np.ndarray, k: int, lo: float, hi: float):
    """k iterations of the Chebyshev smoother for D^{-1}A on [lo, hi], x0 = 0.

    theta = (hi+lo)/2, delta = (hi-lo)/2, sigma = theta/delta, rho_0 = 1/sigma;
    x_1 = d_0 = D^{-1} r / theta; for i = 1..k-1:
      r_i = r - A x_i, rho_i = 1/(2 sigma - rho_{i-1}),
      d_i = rho_i rho_{i-1} d_{i-1} + (2 rho_i / delta) D^{-1} r_i, x_{i+1} = x_i + d_i.
    k iterations use k-1 operator applications.
    """
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = dinv * r / theta
    x = d.copy()
    for _ in range(1, k):
        ri = r - apply_A(x)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * ri)
        x = x + d
        rho = rho_new
    return x


def chebyshev_coefficients(k: int, lo: float, hi: float):
    """(1/theta, [(rho_i rho_{i-1}, 2 rho_i/delta) for i=1..k-1])."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    out = []
    for _ in range(1, k):
        rn = 1.0 / (2.0 * sigma - rho)
        out.append((rn * rho, 2.0 * rn / delta))
        rho = rn
    return 1.0 / theta, out


# ---------------------------------------------------------------- Schur step
def minres1(apply_S: Callable, ds_inv: np.ndarray, r: np.ndarray):
    """One preconditioned MINRES step from zero with P = D_S^{-1}.

    x = beta z, z = P r, beta = <S z, z> / <S z, P S z> minimises ||r - S x||_P
    over span{P r}.  Returns (x, S z) so callers can reuse S z.
    """
    z = ds_inv * r
    y = apply_S(z)
    beta = float(y @ z) / float(y @ (ds_inv * y))
    return beta * z, y, beta


def bicgstab1(apply_S: Callable, ds_inv: np.ndarray, r: np.ndarray):
    """One right-preconditioned BiCGStab iteration from zero with P = D_S^{-1} (the
    corrector mode's ChebBiCGStab(1, 1) of Sec. 4: one Chebyshev step on the diagonal is
    a scaled Jacobi step, and BiCGStab is invariant to that scale).

    r_0 = r, shadow residual r_0; p = P r_0, v = S p, alpha = <r_0, r_0>/<r_0, v>;
    s = r_0 - alpha v, q = P s, t = S q, omega = <t, s>/<t, t> (0 if t = 0);
    x = alpha p + omega q.
    Returns (x, p, q, alpha, omega) so callers can reuse A^{-1} B^T p and A^{-1} B^T q.
    """
    p = ds_inv * r
    v = apply_S(p)
    alpha = float(r @ r) / float(r @ v)
    s_ = r - alpha * v
    q = ds_inv * s_
    t = apply_S(q)
    tt = float(t @ t)
    omega = float(t @ s_) / tt if tt > 0.0 else 0.0     # s = 0: the first half-step solved it
    return alpha * p + omega * q, p, q, alpha, omega


# ---------------------------------------------------------------- block smoother
def block_smoother(ainv: Callable, sinv: Callable, B, r_u: np.ndarray, r_p: np.ndarray):
    """K_j = [[Ah, B^T], [B, B Ah^{-1} B^T - Sh]]^{-1} applied to (r_u, r_p).

    The block matrix factors as [[I, 0], [B Ah^{-1}, I]] [[Ah, B^T], [0, -Sh]],
    hence w = Ah^{-1} r_u, y_p = Sh^{-1}(B w - r_p), y_u = w - Ah^{-1} B^T y_p:
    two solves with Ah and one with Sh (Sec. 4).
    """
    w = ainv(r_u)
    y_p = sinv(B @ w - r_p)
    y_u = w - ainv(B.T @ y_p)
    return y_u, y_p


# ---------------------------------------------------------------- levels
@dataclass
class Level:
    op: fem.Operator
    dA_inv: np.ndarray
    dS_inv: np.ndarray
    lo: float = 0.0
    hi: float = 0.0
    lam: float = 0.0
    P_u: Optional[sp.csr_matrix] = None    # prolongation from level-1 (velocity)
    P_p: Optional[sp.csr_matrix] = None
    lu: Optional[tuple] = None             # dense LU of the coarsest block matrix


def prolongation_1field(coarse: fem.Box, fine: fem.Box, nodes: np.ndarray, ncomp: int):
    """Embedding of the coarse FE space into the fine one.

    Entry (f, c) = value of coarse basis function c at fine node f, found by
    locating the coarse cell containing f and evaluating the Lagrange basis on
    ``nodes`` in that cell's reference coordinates (nested spaces, Sec. 4).
    """
    dim = coarse.dim
    k = len(nodes)
    order = k - 1
    fshape = tuple(order * c + 1 for c in fine.cells)
    cshape = tuple(order * c + 1 for c in coarse.cells)
    hc = [coarse.extent[d] / coarse.cells[d] for d in range(dim)]
    # 1D factors, then Kronecker product (x fastest => kron(z, y, x))
    mats = []
    for d in range(dim):
        nf = fshape[d]
        nc_ = cshape[d]
        P = np.zeros((nf, nc_))
        xf = np.linspace(0.0, coarse.extent[d], nf)
        for f in range(nf):
            cell = min(int(xf[f] / hc[d] + 1e-12), coarse.cells[d] - 1)
            xi = xf[f] / hc[d] - cell
            val, _ = fem.lagrange_1d(nodes, np.array([xi]))
            for a in range(k):
                if abs(val[0, a]) > 1e-15:
                    P[f, order * cell + a] = val[0, a]
        mats.append(sp.csr_matrix(P))
    P = mats[0]
    for d in range(1, dim):
        P = sp.kron(mats[d], P, format="csr")
    if ncomp > 1:
        P = sp.block_diag([P] * ncomp, format="csr")
    return P


@dataclass
class MGParams:
    k_A: int = 4
    m: int = 2
    n_cycles: int = 1
    cheb_upper: float = 1.2
    cheb_ratio: float = 20.0
    n_eig: int = 12
    schur: str = "minres"      # "bicgstab" in the corrector mode (Sec. 4)


class Hierarchy:
    """Assembled level matrices and the monolithic V-cycle of Sec. 4."""

    def __init__(self, levels_ops: List[fem.Operator], params: MGParams = MGParams()):
        self.params = params
        self.levels: List[Level] = []
        for j, op in enumerate(levels_ops):
            dA = op.A.diagonal()
            dS = np.asarray((op.B.multiply(op.B)) @ (1.0 / dA)).ravel()
            lv = Level(op=op, dA_inv=1.0 / dA, dS_inv=1.0 / dS)
            free = (~op.dir_mask).astype(float)
            lam, _, _ = lanczos_lambda_max(op.A, dA, free, params.n_eig)
            lv.lam = lam
            lv.hi = params.cheb_upper * lam
            lv.lo = lv.hi / params.cheb_ratio
            if j > 0:
                lv.P_u = prolongation_1field(levels_ops[j - 1].box, op.box, fem.Q2_NODES, op.box.dim)
                lv.P_p = prolongation_1field(levels_ops[j - 1].box, op.box, fem.Q1_NODES, 1)
            else:
                lv.lu = sla.lu_factor(op.stokes().toarray())
            self.levels.append(lv)

    # -- pieces ---------------------------------------------------------
    def cheb(self, j: int, r: np.ndarray):
        lv = self.levels[j]
        return chebyshev(lv.op.apply_A, lv.dA_inv, r, self.params.k_A, lv.lo, lv.hi)

    def smoother(self, j: int, r_u: np.ndarray, r_p: np.ndarray):
        """K_j of Sec. 4 with Ah^{-1} = Cheb(A, diag A, k_A), Sh^{-1} = ChebMINRES(1,1)."""
        lv = self.levels[j]
        B = lv.op.B
        ainv = lambda r: self.cheb(j, r)
        if self.params.schur == "bicgstab":
            sinv = lambda t: bicgstab1(lambda z: B @ ainv(B.T @ z), lv.dS_inv, t)[0]
        else:
            sinv = lambda t: minres1(lambda z: B @ ainv(B.T @ z), lv.dS_inv, t)[0]
        return block_smoother(ainv, sinv, B, r_u, r_p)

    def restrict(self, j: int, r_u: np.ndarray, r_p: np.ndarray):
        lv = self.levels[j]
        cu = lv.P_u.T @ r_u
        cu[self.levels[j - 1].op.dir_mask] = 0.0
        return cu, lv.P_p.T @ r_p

    def prolongate(self, j: int, e_u: np.ndarray, e_p: np.ndarray):
        lv = self.levels[j]
        fu = lv.P_u @ e_u
        fu[lv.op.dir_mask] = 0.0
        return fu, lv.P_p @ e_p

    def coarse_solve(self, f_u, f_p):
        x = sla.lu_solve(self.levels[0].lu, np.concatenate([f_u, f_p]))
        n = self.levels[0].op.box.n_vel
        return x[:n], x[n:]

    def vcycle(self, j: int, f_u: np.ndarray, f_p: np.ndarray):
        """One V-cycle on level j from a zero initial guess."""
        if j == 0:
            return self.coarse_solve(f_u, f_p)
        op = self.levels[j].op
        m = self.params.m
        x_u = np.zeros_like(f_u)
        x_p = np.zeros_like(f_p)
        for s in range(m):
            if s == 0:
                r_u, r_p = f_u, f_p
            else:
                a_u, a_p = op.apply_stokes(x_u, x_p)
                r_u, r_p = f_u - a_u, f_p - a_p
            y_u, y_p = self.smoother(j, r_u, r_p)
            x_u, x_p = x_u + y_u, x_p + y_p
        a_u, a_p = op.apply_stokes(x_u, x_p)
        c_u, c_p = self.restrict(j, f_u - a_u, f_p - a_p)
        e_u, e_p = self.vcycle(j - 1, c_u, c_p)
        p_u, p_p = self.prolongate(j, e_u, e_p)
        x_u, x_p = x_u + p_u, x_p + p_p
        for s in range(m):
            a_u, a_p = op.apply_stokes(x_u, x_p)
            y_u, y_p = self.smoother(j, f_u - a_u, f_p - a_p)
            x_u, x_p = x_u + y_u, x_p + y_p
        return x_u, x_p

    def precondition(self, r_u: np.ndarray, r_p: np.ndarray):
        """n V-cycles for M_J (n = 1 by default), zero initial guess."""
        J = len(self.levels) - 1
        op = self.levels[J].op
        x_u, x_p = self.vcycle(J, r_u, r_p)
        for _ in range(1, self.params.n_cycles):
            a_u, a_p = op.apply_stokes(x_u, x_p)
            e_u, e_p = self.vcycle(J, r_u - a_u, r_p - a_p)
            x_u, x_p = x_u + e_u, x_p + e_p
        return x_u, x_p


# ---------------------------------------------------------------- FGMRES
@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    rel_res: float
    history: list = field(default_factory=list)
    converged: bool = False


def fgmres(apply_M: Callable, precond: Callable, g: np.ndarray, x0: Optional[np.ndarray] = None,
           rtol: float = 1e-8, restart: int = 100, max_iter: int = 500) -> SolveResult:
    """Right-preconditioned flexible GMRES with restarts.

    Arnoldi by modified Gram-Schmidt, Givens rotations on the Hessenberg
    matrix; the stopping test uses the Arnoldi residual estimate and is
    confirmed on the true residual ||g - M x|| / ||g|| after each cycle.
    """
    n = g.size
    x = np.zeros(n) if x0 is None else x0.astype(float).copy()
    gnorm = float(np.linalg.norm(g))
    if gnorm == 0.0:
        return SolveResult(x=np.zeros(n), iters=0, rel_res=0.0, converged=True)
    r = g - apply_M(x)
    beta = float(np.linalg.norm(r))
    hist = [beta / gnorm]
    it = 0
    while beta / gnorm > rtol and it < max_iter:
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        s = np.zeros(restart + 1)
        s[0] = beta
        k_used = 0
        for k in range(restart):
            z = precond(V[k])
            Z.append(z)
            w = apply_M(z)
            for i in range(k + 1):
                H[i, k] = float(w @ V[i])
                w = w - H[i, k] * V[i]
            hnext = float(np.linalg.norm(w))
            H[k + 1, k] = hnext
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            s[k + 1] = -sn[k] * s[k]
            s[k] = cs[k] * s[k]
            it += 1
            k_used = k + 1
            hist.append(abs(s[k + 1]) / gnorm)
            if abs(s[k + 1]) / gnorm <= rtol or it >= max_iter:
                break
            if hnext == 0.0:
                break
            V.append(w / hnext)
        y = sla.solve_triangular(H[:k_used, :k_used], s[:k_used])
        for i in range(k_used):
            x = x + y[i] * Z[i]
        r = g - apply_M(x)
        beta = float(np.linalg.norm(r))
    return SolveResult(x=x, iters=it, rel_res=beta / gnorm, history=hist, converged=beta / gnorm <= rtol)


# ---------------------------------------------------------------- extension (Sec. 2)
def extension_solve(box: fem.Box, J: np.ndarray, mu: np.ndarray, ref: fem.Reference, g: np.ndarray,
                    fixed: Optional[np.ndarray] = None):
    """Ext of Sec. 2: the displacement u with u = g on the Dirichlet dofs of ``box`` and
    (mu eps(u), eps(v)) = 0 for every v that vanishes there.

    The bilinear form is the operator's a(u, v) = (c_m u, v) + (2 eta eps(u), eps(v)) with
    c_m = 0 and eta = mu / 2.  Interior dofs I, Dirichlet dofs W of the unconstrained
    matrix: A_II u_I = -A_IW g_W, solved by SuperLU.  Reading: the Dirichlet set is the box
    walls (the paper's fixed outer boundary, with data allowed to be nonzero) and, where
    ``fixed`` (a mask over the velocity vector) is given, those dofs too: the nodes of
    the solid, where the extension takes the solid's values.
    """
    zero = np.zeros_like(mu)
    A = fem.assemble_unconstrained(box, J, zero, 0.5 * mu, ref).A.tocsr()
    dm = box.dirichlet_vel_dofs()
    if fixed is not None:
        dm = dm | fixed
    I = np.nonzero(~dm)[0]
    W = np.nonzero(dm)[0]
    u = np.where(dm, g, 0.0)
    rhs = -(A[I][:, W] @ g[W])
    u[I] = spla.splu(A[I][:, I].tocsc()).solve(rhs)
    return u


def extension_energy(box: fem.Box, J: np.ndarray, mu: np.ndarray, ref: fem.Reference, u: np.ndarray) -> float:
    """(mu eps(u), eps(u)) / 2 of the whole box (the extension minimises it)."""
    A = fem.assemble_unconstrained(box, J, np.zeros_like(mu), 0.5 * mu, ref).A
    return 0.5 * float(u @ (A @ u))


# ---------------------------------------------------------------- glue
def build_levels(mesh, disp_fine: np.ndarray, c_mass: list, eta: list, ref: Optional[fem.Reference] = None):
    """Assemble every level (coarse displacement by vertex injection)."""
    from paper_2305_08986_amd.workloads import inject_displacement   # input layout only
    ref = ref or fem.Reference(mesh.dim)
    ops = []
    for j in range(mesh.n_levels):
        box = fem.level_box(mesh, j)
        dj = inject_displacement(mesh, disp_fine, j)
        J = fem.jacobians_q1(box, dj, ref)
        ops.append(fem.assemble(box, J, c_mass[j], eta[j], ref))
    return ops


def build_levels_corrector(mesh, disp_fine: np.ndarray, c_mass: list, eta: list, conv: list,
                           ref: Optional[fem.Reference] = None):
    """Levels of the corrector mode: A + N + S with the convection and streamline terms
    of ``fem.convection_matrices``; conv[j] = (vconv, rho, r) of level j."""
    from paper_2305_08986_amd.workloads import inject_displacement   # input layout only
    ref = ref or fem.Reference(mesh.dim)
    ops = []
    for j in range(mesh.n_levels):
        box = fem.level_box(mesh, j)
        Jq = fem.jacobians_q1(box, inject_displacement(mesh, disp_fine, j), ref)
        op = fem.assemble(box, Jq, c_mass[j], eta[j], ref)
        vconv, rho, r = conv[j]
        op.A = (op.A + fem.assemble_convection(box, Jq, vconv, rho, r, ref)).tocsr()
        ops.append(op)
    return ops


def solve_stokes(h: Hierarchy, g_u, g_p, x0=None, rtol=1e-8, restart=100, max_iter=500):
    op = h.levels[-1].op
    nv = op.box.n_vel

    def M(x):
        a, b = op.apply_stokes(x[:nv], x[nv:])
        return np.concatenate([a, b])

    def P(r):
        a, b = h.precondition(r[:nv], r[nv:])
        return np.concatenate([a, b])

    return fgmres(M, P, np.concatenate([g_u, g_p]), x0, rtol, restart, max_iter)
