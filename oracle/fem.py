"""ORACLE -- test infrastructure only (tests, the smoke check and the CPU
baseline leg of the benchmark).  Never imported by the product path.

Plain FP64 CPU definition of the discrete generalized-Stokes operator of the
paper: Taylor-Hood Q2-Q1 on quadrilaterals/hexahedra (Sec. 3.2 and the first
paragraph of Sec. 5: p1 = 2, p2 = 1) on the ALE-mapped mesh (Sec. 3.2, the
mapped spaces V_h, Q_h), with the symmetric predictor-mode bilinear forms of
Sec. 3.1.1,

    a(u, v) = (c_m u, v) + (2 eta eps(u), eps(v)),     b(v, q) = (div v, q),

assembled into the block matrix [[A, B^T], [B, 0]] of Sec. 4.

Every element matrix is evaluated by plain Gauss quadrature with full
tabulation of the basis at the quadrature points: no sum factorization.
Readings where the paper is silent are stated where they are used (the
factor 2 in the viscous form, the 3-point Gauss rule, the multilinear ALE
map, Dirichlet rows as identity).

Pins: tests/test_oracle_pins.py checks this module against closed forms
(1D element matrices, Gauss exactness), invariants (symmetry, rigid-motion
null space, volume, divergence of linear fields) and convergence rates.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------- 1D ingredients
def gauss_rule(npts: int = 3):
    """Gauss-Legendre rule on [0,1] (numpy's leggauss, mapped)."""
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_1d(nodes: np.ndarray, x: np.ndarray):
    """Values and derivatives of the Lagrange polynomials on ``nodes`` at ``x``.

    Returns (val[len(x)][len(nodes)], der[len(x)][len(nodes)]).
    """
    nodes = np.asarray(nodes, dtype=float)
    x = np.asarray(x, dtype=float)
    n = len(nodes)
    val = np.ones((len(x), n))
    der = np.zeros((len(x), n))
    for i in range(n):
        others = [m for m in range(n) if m != i]
        denom = np.prod([nodes[i] - nodes[m] for m in others])
        for m in others:
            val[:, i] *= (x - nodes[m])
        val[:, i] /= denom
        # product rule
        for m in others:
            term = np.ones(len(x))
            for l in others:
                if l != m:
                    term *= (x - nodes[l])
            der[:, i] += term
        der[:, i] /= denom
    return val, der


Q2_NODES = np.array([0.0, 0.5, 1.0])
Q1_NODES = np.array([0.0, 1.0])


def tensor_tabulation(dim: int, nodes: np.ndarray, pts: np.ndarray):
    """Tensor-product basis on ``nodes``^dim tabulated at ``pts``^dim.

    Local node index n = i0 + k*i1 (+ k^2*i2), point index q likewise (x fastest).
    Returns phi[q][n] and dphi[q][n][b] (derivative w.r.t. reference coordinate b).
    """
    v, d = lagrange_1d(nodes, pts)
    k = len(nodes)
    npt = len(pts)
    nloc = k ** dim
    nq = npt ** dim
    phi = np.zeros((nq, nloc))
    dphi = np.zeros((nq, nloc, dim))
    for q, qi in enumerate(itertools.product(range(npt), repeat=dim)):
        qi = qi[::-1]                  # itertools: last index fastest -> reverse => x fastest
        for n, ni in enumerate(itertools.product(range(k), repeat=dim)):
            ni = ni[::-1]
            phi[q, n] = np.prod([v[qi[a], ni[a]] for a in range(dim)])
            for b in range(dim):
                dphi[q, n, b] = np.prod([(d if a == b else v)[qi[a], ni[a]] for a in range(dim)])
    return phi, dphi


# ---------------------------------------------------------------- structured box mesh
@dataclass
class Box:
    """One level of the structured box mesh (reference configuration)."""
    dim: int
    cells: tuple           # cells per direction
    extent: tuple
    dirichlet_faces: int

    @property
    def n_cells(self):
        return int(np.prod(self.cells))

    @property
    def vel_nodes(self):
        return tuple(2 * c + 1 for c in self.cells)

    @property
    def p_nodes(self):
        return tuple(c + 1 for c in self.cells)

    @property
    def n_vel_nodes(self):
        return int(np.prod(self.vel_nodes))

    @property
    def n_vel(self):
        return self.dim * self.n_vel_nodes

    @property
    def n_p(self):
        return int(np.prod(self.p_nodes))

    def h(self):
        return np.array([self.extent[i] / self.cells[i] for i in range(self.dim)])

    def cell_index_grid(self):
        g = np.meshgrid(*[np.arange(c) for c in self.cells], indexing="ij")
        return [a.ravel(order="F") for a in g]           # cell c -> (ix, iy[, iz])

    def _lex(self, idx, dims):
        out = np.zeros_like(idx[0])
        stride = 1
        for d in range(self.dim):
            out = out + idx[d] * stride
            stride *= dims[d]
        return out

    def cell_vel_nodes(self, cells: Optional[np.ndarray] = None):
        """[nc][3^dim] global Q2 node index of local node (x fastest)."""
        ci = self.cell_index_grid()
        if cells is not None:
            ci = [a[cells] for a in ci]
        loc = list(itertools.product(range(3), repeat=self.dim))
        out = np.empty((len(ci[0]), 3 ** self.dim), dtype=np.int64)
        for n, li in enumerate(loc):
            li = li[::-1]
            out[:, n] = self._lex([2 * ci[d] + li[d] for d in range(self.dim)], self.vel_nodes)
        return out

    def cell_p_nodes(self, cells: Optional[np.ndarray] = None):
        ci = self.cell_index_grid()
        if cells is not None:
            ci = [a[cells] for a in ci]
        loc = list(itertools.product(range(2), repeat=self.dim))
        out = np.empty((len(ci[0]), 2 ** self.dim), dtype=np.int64)
        for n, li in enumerate(loc):
            li = li[::-1]
            out[:, n] = self._lex([ci[d] + li[d] for d in range(self.dim)], self.p_nodes)
        return out

    def vertex_coords(self):
        axes = [np.linspace(0.0, self.extent[i], self.p_nodes[i]) for i in range(self.dim)]
        g = np.meshgrid(*axes, indexing="ij")
        return np.stack([a.ravel(order="F") for a in g])

    def vel_node_ref_coords(self):
        axes = [np.linspace(0.0, self.extent[i], self.vel_nodes[i]) for i in range(self.dim)]
        g = np.meshgrid(*axes, indexing="ij")
        return np.stack([a.ravel(order="F") for a in g])

    def dirichlet_vel_dofs(self):
        """Boolean mask over the component-major velocity vector."""
        nn = self.vel_nodes
        g = np.meshgrid(*[np.arange(n) for n in nn], indexing="ij")
        g = [a.ravel(order="F") for a in g]
        m = np.zeros(self.n_vel_nodes, dtype=bool)
        for d in range(self.dim):
            if self.dirichlet_faces & (1 << (2 * d)):
                m |= g[d] == 0
            if self.dirichlet_faces & (1 << (2 * d + 1)):
                m |= g[d] == nn[d] - 1
        return np.tile(m, self.dim)

    def cells_of_vel_node(self, node: int):
        """Cells containing Q2 node ``node``."""
        nn = self.vel_nodes
        idx = []
        r = node
        for d in range(self.dim):
            idx.append(r % nn[d])
            r //= nn[d]
        ranges = []
        for d in range(self.dim):
            i = idx[d]
            if i % 2 == 1:
                ranges.append([i // 2])
            else:
                c = [i // 2 - 1, i // 2]
                ranges.append([x for x in c if 0 <= x < self.cells[d]])
        out = []
        for t in itertools.product(*ranges):
            c = 0
            stride = 1
            for d in range(self.dim):
                c += t[d] * stride
                stride *= self.cells[d]
            out.append(c)
        return out

    def cells_of_p_node(self, node: int):
        pn = self.p_nodes
        idx = []
        r = node
        for d in range(self.dim):
            idx.append(r % pn[d])
            r //= pn[d]
        ranges = []
        for d in range(self.dim):
            c = [idx[d] - 1, idx[d]]
            ranges.append([x for x in c if 0 <= x < self.cells[d]])
        out = []
        for t in itertools.product(*ranges):
            c = 0
            stride = 1
            for d in range(self.dim):
                c += t[d] * stride
                stride *= self.cells[d]
            out.append(c)
        return out


# ---------------------------------------------------------------- geometry
class Reference:
    """Tabulated reference-element data for one dimension."""

    def __init__(self, dim: int, npts: int = 3):
        self.dim = dim
        self.pts, self.w1 = gauss_rule(npts)
        self.phi, self.dphi = tensor_tabulation(dim, Q2_NODES, self.pts)      # velocity
        self.psi, self.dpsi = tensor_tabulation(dim, Q1_NODES, self.pts)      # pressure / map
        w = np.ones(1)
        for _ in range(dim):
            w = np.kron(self.w1, w)            # x fastest
        self.w = w


def jacobians_q1(box: Box, disp: np.ndarray, ref: Reference, cells: Optional[np.ndarray] = None):
    """J[c][q][a][b] = d x_a / d xi_b of the multilinear map x = X + d(X).

    The ALE map (Sec. 2.2 and the mapped spaces of Sec. 3.2) is the Q1
    interpolant of the vertex positions X_v + d_v of each cell; xi in [0,1]^dim.
    The box cell's own map X(xi) is affine with Jacobian diag(h), so
    J = diag(h) + sum_v d_v (grad psi_v)^T: the displacement part is formed from the
    displacements themselves, not from differences of positions (whose rounding grows
    with |X| / h).
    """
    vn = box.cell_p_nodes(cells)                          # [nc][2^d] vertices
    dv = disp[:, vn]                                      # [dim][nc][2^d]
    # J[c,q,a,b] = h_a delta_ab + sum_v dpsi[q,v,b] * dv[a,c,v]
    J = np.einsum("qvb,acv->cqab", ref.dpsi, dv)
    h = box.h()
    for a in range(box.dim):
        J[:, :, a, a] += h[a]
    return J


def geometry_factors(J: np.ndarray, ref: Reference):
    """(J^{-1}, det J * w_q) per cell and quadrature point."""
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    return Jinv, det * ref.w[None, :]


def element_matrices(J: np.ndarray, c_mass: np.ndarray, eta: np.ndarray, ref: Reference):
    """Element matrices on every cell of the batch.

    A_K[(a,i),(b,j)] = sum_q w_q det J_q [ c_m d_ab phi_i phi_j
                                          + eta ( d_ab grad phi_i . grad phi_j
                                                  + d_b phi_i d_a phi_j ) ]
    (this is (2 eta eps(phi_j e_b), eps(phi_i e_a)) + (c_m phi_j e_b, phi_i e_a)),
    B_K[k,(a,j)] = sum_q w_q det J_q psi_k d_a phi_j   (b(v,q) = (div v, q)).
    Local velocity dofs are component-major: (a, i) -> a*n_loc + i.
    """
    dim = ref.dim
    Jinv, wdet = geometry_factors(J, ref)
    if np.any(wdet <= 0):
        raise ValueError("inverted cell")
    # physical gradients: G[c,q,i,x] = sum_b Jinv[c,q,b,x] dphi[q,i,b]
    G = np.einsum("cqbx,qib->cqix", Jinv, ref.dphi)
    nl = ref.phi.shape[1]
    wm = wdet * c_mass
    we = wdet * eta
    mass = np.einsum("cq,qi,qj->cij", wm, ref.phi, ref.phi)
    lap = np.einsum("cq,cqix,cqjx->cij", we, G, G)
    cross = np.einsum("cq,cqib,cqja->caibj", we, G, G)     # [c][a][i][b][j]
    nc = J.shape[0]
    A = cross.copy()
    for a in range(dim):
        A[:, a, :, a, :] += mass + lap
    A = A.reshape(nc, dim * nl, dim * nl)
    B = np.einsum("cq,qk,cqja->ckaj", wdet, ref.psi, G).reshape(nc, ref.psi.shape[1], dim * nl)
    return A, B


def element_matrices_abs(J: np.ndarray, c_mass: np.ndarray, eta: np.ndarray, ref: Reference):
    """Magnitude scales of ``element_matrices``: the same quadrature with every factor of
    the integrand replaced by its absolute value, and the physical gradients by
    |G|_{j,x} = sum_b |J^{-1}_{b,x}| |d_b phi_j|,

      |A_K|_{(a,i),(b,j)} = sum_q |w_q det J_q| [ |c_m| d_ab |phi_i phi_j|
                                               + |eta| ( d_ab sum_x |G|_ix |G|_jx + |G|_ib |G|_ja ) ]
      |B_K|_{k,(a,j)}     = sum_q |w_q det J_q| |psi_k| |G|_ja.

    Applied to |x| they bound the sum of magnitudes of every term that an evaluation by
    this quadrature adds, which is the scale of its rounding error (an entry of A_K can
    vanish by cancellation of its quadrature terms, e.g. the 1D integral of N_1' N_1,
    while the terms themselves do not)."""
    dim = ref.dim
    Jinv, wdet = geometry_factors(J, ref)
    Ga = np.einsum("cqbx,qib->cqix", np.abs(Jinv), np.abs(ref.dphi))
    wd = np.abs(wdet)
    nl = ref.phi.shape[1]
    aphi = np.abs(ref.phi)
    mass = np.einsum("cq,qi,qj->cij", wd * np.abs(c_mass), aphi, aphi)
    lap = np.einsum("cq,cqix,cqjx->cij", wd * np.abs(eta), Ga, Ga)
    cross = np.einsum("cq,cqib,cqja->caibj", wd * np.abs(eta), Ga, Ga)
    nc = J.shape[0]
    A = cross.copy()
    for a in range(dim):
        A[:, a, :, a, :] += mass + lap
    A = A.reshape(nc, dim * nl, dim * nl)
    B = np.einsum("cq,qk,cqja->ckaj", wd, np.abs(ref.psi), Ga).reshape(nc, ref.psi.shape[1], dim * nl)
    return A, B


def convection_matrices_abs(J: np.ndarray, vconv: np.ndarray, rho: float, r: np.ndarray, ref: Reference):
    """Magnitude scales of ``convection_matrices`` (absolute integrand factors, |G| as in
    ``element_matrices_abs``)."""
    dim = ref.dim
    Jinv, wdet = geometry_factors(J, ref)
    Ga = np.einsum("cqbx,qib->cqix", np.abs(Jinv), np.abs(ref.dphi))
    vg = np.einsum("cqx,cqix->cqi", np.abs(vconv), Ga)
    wd = np.abs(wdet)
    conv = abs(rho) * np.einsum("cq,qi,cqj->cij", wd, np.abs(ref.phi), vg)
    stab = np.einsum("cq,cqi,cqj->cij", wd * np.abs(r), vg, vg)
    nc, nl = J.shape[0], ref.phi.shape[1]
    C = np.zeros((nc, dim, nl, dim, nl))
    for a in range(dim):
        C[:, a, :, a, :] = conv + stab
    return C.reshape(nc, dim * nl, dim * nl)


def convection_matrices(J: np.ndarray, vconv: np.ndarray, rho: float, r: np.ndarray, ref: Reference):
    """Element matrices of the corrector-mode terms on every cell of the batch.

    With the semi-implicit advection of the corrector mode (Sec. 3.1.1: v* is the
    unknown, v° the known convective velocity) the form a_j gains
    (rho (grad v) v°, w), and the streamline term of Sec. 3.2 adds
    sum_K int_K r (v° . grad v)(v° . grad w):

      N_K[(a,i),(b,j)] = d_ab sum_q w_q det J_q rho phi_i (v° . grad phi_j)
      S_K[(a,i),(b,j)] = d_ab sum_q w_q det J_q r_q (v° . grad phi_i)(v° . grad phi_j)

    vconv [nc][Q][dim]: v° at the points; r [nc][Q]: the stabilisation parameter.
    Returns N_K + S_K, component-major like ``element_matrices``.
    """
    dim = ref.dim
    Jinv, wdet = geometry_factors(J, ref)
    G = np.einsum("cqbx,qib->cqix", Jinv, ref.dphi)
    vg = np.einsum("cqx,cqix->cqi", vconv, G)                 # v° . grad phi_i
    conv = rho * np.einsum("cq,qi,cqj->cij", wdet, ref.phi, vg)
    stab = np.einsum("cq,cqi,cqj->cij", wdet * r, vg, vg)
    nc, nl = J.shape[0], ref.phi.shape[1]
    C = np.zeros((nc, dim, nl, dim, nl))
    for a in range(dim):
        C[:, a, :, a, :] = conv + stab
    return C.reshape(nc, dim * nl, dim * nl)


def assemble_convection(box: "Box", J: np.ndarray, vconv: np.ndarray, rho: float, r: np.ndarray,
                        ref: "Reference", chunk: int = 2048, absolute: bool = False) -> sp.csr_matrix:
    """Global velocity-block matrix of the corrector-mode terms; Dirichlet rows and
    columns are zero, so A + C keeps the identity rows of ``assemble``.  absolute=True
    assembles the magnitude scales of ``convection_matrices_abs`` (as ``assemble``)."""
    rows, cols, vals = [], [], []
    nc = box.n_cells
    for s0 in range(0, nc, chunk):
        cs = np.arange(s0, min(nc, s0 + chunk))
        CK = (convection_matrices_abs if absolute else convection_matrices)(J[cs], vconv[cs], rho, r[cs], ref)
        gd = _global_vel_dofs(box, box.cell_vel_nodes(cs))
        n = gd.shape[1]
        rows.append(np.repeat(gd, n, axis=1).ravel())
        cols.append(np.tile(gd, (1, n)).ravel())
        vals.append(CK.ravel())
    nv = box.n_vel
    Cm = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nv, nv)).tocsr()
    free = sp.diags((~box.dirichlet_vel_dofs()).astype(float))
    Cm = (free @ Cm @ free).tocsr()
    Cm.eliminate_zeros()
    return Cm


# ---------------------------------------------------------------- assembly
@dataclass
class Operator:
    box: Box
    A: sp.csr_matrix           # velocity block with Dirichlet rows/cols = identity
    B: sp.csr_matrix           # divergence block with Dirichlet columns zero
    dir_mask: np.ndarray       # Dirichlet velocity dofs

    def stokes(self):
        return sp.bmat([[self.A, self.B.T], [self.B, None]], format="csr")

    def apply_A(self, u):
        return self.A @ u

    def apply_B(self, u):
        return self.B @ u

    def apply_BT(self, p):
        return self.B.T @ p

    def apply_stokes(self, u, p):
        return self.A @ u + self.B.T @ p, self.B @ u


def _global_vel_dofs(box: Box, vn: np.ndarray):
    """[nc][dim*n_loc] component-major global velocity dof of each local dof."""
    nn = box.n_vel_nodes
    return np.concatenate([vn + a * nn for a in range(box.dim)], axis=1)


def assemble(box: Box, J: np.ndarray, c_mass: np.ndarray, eta: np.ndarray, ref: Reference,
             chunk: int = 2048, absolute: bool = False) -> Operator:
    """Global CSR matrices; Dirichlet rows/columns of A become identity, B columns zero.

    absolute=True assembles the magnitude scales of ``element_matrices_abs`` instead:
    applied to |x| they give, per row, the sum of magnitudes of every quadrature term
    of every cell, the scale of the rounding error of any evaluation of the operator by
    this quadrature (componentwise error bounds of the parity tests)."""
    rows, cols, vals = [], [], []
    brow, bcol, bval = [], [], []
    nc = box.n_cells
    for s in range(0, nc, chunk):
        cs = np.arange(s, min(nc, s + chunk))
        AK, BK = (element_matrices_abs if absolute else element_matrices)(J[cs], c_mass[cs], eta[cs], ref)
        gd = _global_vel_dofs(box, box.cell_vel_nodes(cs))
        gp = box.cell_p_nodes(cs)
        n = gd.shape[1]
        rows.append(np.repeat(gd, n, axis=1).ravel())
        cols.append(np.tile(gd, (1, n)).ravel())
        vals.append(AK.ravel())
        m = gp.shape[1]
        brow.append(np.repeat(gp, n, axis=1).ravel())
        bcol.append(np.tile(gd, (1, m)).ravel())
        bval.append(BK.ravel())
    nv, npr = box.n_vel, box.n_p
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nv, nv)).tocsr()
    B = sp.coo_matrix((np.concatenate(bval), (np.concatenate(brow), np.concatenate(bcol))),
                      shape=(npr, nv)).tocsr()
    dm = box.dirichlet_vel_dofs()
    free = sp.diags((~dm).astype(float))
    A = (free @ A @ free + sp.diags(dm.astype(float))).tocsr()
    B = (B @ free).tocsr()
    A.eliminate_zeros()
    B.eliminate_zeros()
    return Operator(box=box, A=A, B=B, dir_mask=dm)


def assemble_unconstrained(box: Box, J, c_mass, eta, ref: Reference) -> Operator:
    """Same as ``assemble`` but with no Dirichlet rows (for invariant pins)."""
    b2 = Box(box.dim, box.cells, box.extent, 0)
    return assemble(b2, J, c_mass, eta, ref)


# ---------------------------------------------------------------- sampled rows (large meshes)
def apply_rows(box: Box, disp: np.ndarray, c_mass: np.ndarray, eta: np.ndarray,
               ref: Reference, u: np.ndarray, p: Optional[np.ndarray],
               vel_dofs: Sequence[int], p_dofs: Sequence[int], conv=None, absolute: bool = False):
    """Selected entries of (A u + B^T p, B u) evaluated cell by cell.

    Only the cells touching the requested rows are integrated, so this works at
    any mesh size.  Dirichlet handling matches ``assemble``.  ``conv`` =
    (vconv, rho, r) adds the corrector-mode terms of ``convection_matrices`` to A.
    absolute=True evaluates the magnitude scales (|A| |u| + |B|^T |p|, |B| |u|) with the
    matrices of ``element_matrices_abs``, as ``assemble(absolute=True)``.
    """
    dm = box.dirichlet_vel_dofs()
    if absolute:
        u = np.abs(u)
        p = None if p is None else np.abs(p)
    uf = np.where(dm, 0.0, u)
    nn = box.n_vel_nodes
    needed = set()
    vel_cells = []
    for g in vel_dofs:
        cl = box.cells_of_vel_node(int(g) % nn)
        vel_cells.append(cl)
        needed.update(cl)
    p_cells = []
    for k in p_dofs:
        cl = box.cells_of_p_node(int(k))
        p_cells.append(cl)
        needed.update(cl)
    cells = np.array(sorted(needed), dtype=np.int64)
    pos = {c: i for i, c in enumerate(cells)}
    J = jacobians_q1(box, disp, ref, cells)
    AK, BK = (element_matrices_abs if absolute else element_matrices)(J, c_mass[cells], eta[cells], ref)
    if conv is not None:
        vconv, rho, r = conv
        AK = AK + (convection_matrices_abs if absolute else convection_matrices)(J, vconv[cells], rho, r[cells], ref)
    gd = _global_vel_dofs(box, box.cell_vel_nodes(cells))
    gp = box.cell_p_nodes(cells)
    ov = np.zeros(len(vel_dofs))
    for r, (g, cl) in enumerate(zip(vel_dofs, vel_cells)):
        g = int(g)
        if dm[g]:
            ov[r] = u[g]
            continue
        s = 0.0
        for c in cl:
            i = pos[c]
            loc = int(np.nonzero(gd[i] == g)[0][0])
            s += AK[i, loc, :] @ uf[gd[i]]
            if p is not None:
                s += BK[i, :, loc] @ p[gp[i]]
        ov[r] = s
    op = np.zeros(len(p_dofs))
    for r, (k, cl) in enumerate(zip(p_dofs, p_cells)):
        s = 0.0
        for c in cl:
            i = pos[c]
            loc = int(np.nonzero(gp[i] == int(k))[0][0])
            s += BK[i, loc, :] @ uf[gd[i]]
        op[r] = s
    return ov, op


def apply_ebe(box: Box, disp: np.ndarray, c_mass: np.ndarray, eta: np.ndarray, ref: Reference,
              u: np.ndarray, cells: np.ndarray):
    """Contributions of ``cells`` to A u, element by element (no global matrix).

    The operator on a mesh too large to assemble: for each cell the element matrix
    A_K of ``element_matrices`` times the cell's gathered velocity values (Dirichlet
    columns zero, as in ``assemble``), summed into the global dofs the cell touches.
    Returns (dofs, vals), the touched free velocity dofs in increasing order and their
    summed contributions; summed over all cells of the mesh this is A u on the free
    rows (the identity rows of the Dirichlet dofs are not cell contributions).
    """
    dm = box.dirichlet_vel_dofs()
    cells = np.asarray(cells, dtype=np.int64)
    J = jacobians_q1(box, disp, ref, cells)
    AK, _ = element_matrices(J, c_mass[cells], eta[cells], ref)
    gd = _global_vel_dofs(box, box.cell_vel_nodes(cells))
    uK = np.where(dm[gd], 0.0, u[gd])
    yK = np.einsum("cij,cj->ci", AK, uK)
    dofs, inv = np.unique(gd, return_inverse=True)
    vals = np.bincount(inv.ravel(), weights=yK.ravel(), minlength=len(dofs))
    keep = ~dm[dofs]
    return dofs[keep], vals[keep]


def level_box(mesh, level: int) -> Box:
    """Box of ``level`` from a mesh description (dim, n_coarse, extent, dirichlet_faces)."""
    cells = tuple(mesh.n_coarse[i] << level for i in range(mesh.dim))
    return Box(mesh.dim, cells, tuple(mesh.extent), mesh.dirichlet_faces)
