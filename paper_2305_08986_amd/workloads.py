"""Seeded synthetic inputs for the generalized-Stokes hot path.

This module only *draws and lays out input data*: the structured box meshes,
the fine-level vertex displacement of the ALE map, the per-quadrature-point
coefficient fields (mass coefficient and effective viscosity) and the
right-hand sides.  It holds none of the method's arithmetic (no basis
functions, no Jacobians, no operators) and is shared, unchanged, by the CPU
oracle tests and the HIP path.

The workloads stand in for the paper's channel/beam benchmarks (Sec. 5,
Tables 1 and 3), whose meshes are not available:

* ``C0`` 2D unit square 16x16, affine, viscosity 1 with an inclusion of
  viscosity 1e4 on [0.25,0.5]^2 (cell-aligned), mass coefficient 1e2.
* ``C1`` 2D channel [0,2.5]x[0,0.41], 256x64 cells, bilinear ALE map from a
  sum of four random sine modes (amplitude 0.02), viscosity 1e-3 with a strip
  [0.6,1.0]x[0.19,0.21] of viscosity 1e3 (contrast 1e6).
* ``C2`` 3D unit cube 64^3, trilinear warp (amplitude 0.05), log-uniform
  viscosity in [1e-3,1e3] per block of 8^3 fine cells.
* ``C3`` as C2 at 128^3 cells.
* ``C4`` 96^3 cells, a 20-step sequence: every step adds a displacement
  increment of amplitude 0.0025 and redraws the viscosity field.

The effective viscosity models the splitting of Sec. 3.1.1 (fluid viscosity
in the fluid, gamma*tau*mu_s in the solid); the mass coefficient is the
implicit BDF term rho/(gamma*tau) of Sec. 3.1.

Conventions (shared by every consumer):

* cells, Q2 velocity nodes, Q1 pressure nodes and mesh vertices are numbered
  lexicographically with x fastest;
* velocity vectors are component-major ``[dim][n_vel_nodes]``;
* per-cell quadrature points are the tensor 3-point Gauss points, numbered
  lexicographically (x fastest); coefficient arrays are ``[n_cells][3**dim]``;
* the vertex displacement is ``[dim][n_vertices]`` on the finest level and
  defines a multilinear (Q1) ALE map on every level by injection at that
  level's vertices;
* ``dirichlet_faces`` bit f marks face f in (x-, x+, y-, y+, z-, z+) as a
  homogeneous no-slip wall; the default leaves x+ as a do-nothing outflow.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

BASE_SEED = 230508986

# Reference positions of the 3 Gauss points per direction on [0,1]; used
# only to decide where a coefficient sample sits inside its cell.
_SAMPLE_PTS = np.array([0.5 - math.sqrt(15.0) / 10.0, 0.5, 0.5 + math.sqrt(15.0) / 10.0])


def default_dirichlet_faces(dim: int) -> int:
    """All faces except x+ (bit 1)."""
    return ((1 << (2 * dim)) - 1) & ~0b10


@dataclasses.dataclass
class MeshDesc:
    dim: int
    n_fine: tuple
    extent: tuple
    n_coarse: tuple
    dirichlet_faces: int

    @property
    def n_levels(self) -> int:
        r = [self.n_fine[i] // self.n_coarse[i] for i in range(self.dim)]
        lv = int(round(math.log2(r[0])))
        return lv + 1

    def cells(self, level: int) -> tuple:
        s = 1 << level
        return tuple(self.n_coarse[i] * s for i in range(self.dim))

    def n_cells(self, level: int) -> int:
        return int(np.prod(self.cells(level)))

    def vel_nodes(self, level: int) -> tuple:
        return tuple(2 * c + 1 for c in self.cells(level))

    def p_nodes(self, level: int) -> tuple:
        return tuple(c + 1 for c in self.cells(level))

    def n_vel(self, level: int) -> int:
        return self.dim * int(np.prod(self.vel_nodes(level)))

    def n_p(self, level: int) -> int:
        return int(np.prod(self.p_nodes(level)))


@dataclasses.dataclass
class Workload:
    name: str
    mesh: MeshDesc
    disp: np.ndarray                  # [dim][n_vert_fine] vertex displacement
    c_mass: List[np.ndarray]          # per level [n_cells][Q]
    eta: List[np.ndarray]             # per level [n_cells][Q]
    g_u: np.ndarray                   # [n_vel_fine], Dirichlet entries zero
    g_p: np.ndarray                   # [n_p_fine]
    info: dict


CONFIGS = {
    "C0": dict(dim=2, n=(16, 16), extent=(1.0, 1.0), n_coarse=(4, 4), amp=0.0,
               eta="inclusion", desc="2D unit square 16x16 affine, inclusion contrast 1e4"),
    "C1": dict(dim=2, n=(256, 64), extent=(2.5, 0.41), n_coarse=(8, 2), amp=0.02,
               eta="strip", desc="2D channel 256x64 warped, strip contrast 1e6"),
    "C2": dict(dim=3, n=(64, 64, 64), extent=(1.0, 1.0, 1.0), n_coarse=(4, 4, 4), amp=0.05,
               eta="loguniform", desc="3D box 64^3 warped, log-uniform eta per 8^3 block"),
    "C3": dict(dim=3, n=(128, 128, 128), extent=(1.0, 1.0, 1.0), n_coarse=(4, 4, 4), amp=0.05,
               eta="loguniform", desc="3D box 128^3 warped, log-uniform eta per 8^3 block"),
    "C4": dict(dim=3, n=(96, 96, 96), extent=(1.0, 1.0, 1.0), n_coarse=(3, 3, 3), amp=0.0025,
               eta="loguniform", steps=20, desc="3D box 96^3, 20 ALE steps"),
    # small cases used by the parity tests (same laws as C2 at reduced size)
    "T3_4": dict(dim=3, n=(4, 4, 4), extent=(1.0, 1.0, 1.0), n_coarse=(2, 2, 2), amp=0.05,
                 eta="loguniform", block=2, desc="3D 4^3 warped"),
    "T3_8": dict(dim=3, n=(8, 8, 8), extent=(1.0, 1.0, 1.0), n_coarse=(2, 2, 2), amp=0.05,
                 eta="loguniform", block=2, desc="3D 8^3 warped"),
    "T3_16": dict(dim=3, n=(16, 16, 16), extent=(1.0, 1.0, 1.0), n_coarse=(4, 4, 4), amp=0.05,
                  eta="loguniform", block=4, desc="3D 16^3 warped"),
    "T3_R": dict(dim=3, n=(12, 6, 10), extent=(1.2, 0.6, 1.0), n_coarse=(6, 3, 5), amp=0.04,
                 eta="loguniform", block=3, desc="3D 12x6x10 warped, odd coarse counts"),
    "T2_R": dict(dim=2, n=(22, 14), extent=(1.1, 0.7), n_coarse=(11, 7), amp=0.03,
                 eta="loguniform", block=3, desc="2D 22x14 warped, odd coarse counts"),
    "T4_S": dict(dim=3, n=(16, 16, 16), extent=(1.0, 1.0, 1.0), n_coarse=(4, 4, 4), amp=0.0025,
                 eta="loguniform", block=4, steps=3, desc="3D 16^3 step sequence (C4 law, small)"),
    # the C0 law refined (the inclusion stays aligned with the 4x4 coarse grid): robustness
    # of the iteration count with the number of levels
    "C0_32": dict(dim=2, n=(32, 32), extent=(1.0, 1.0), n_coarse=(4, 4), amp=0.0,
                  eta="inclusion", desc="2D unit square 32x32 affine, inclusion contrast 1e4"),
    "C0_64": dict(dim=2, n=(64, 64), extent=(1.0, 1.0), n_coarse=(4, 4), amp=0.0,
                  eta="inclusion", desc="2D unit square 64x64 affine, inclusion contrast 1e4"),
    "C0_128": dict(dim=2, n=(128, 128), extent=(1.0, 1.0), n_coarse=(4, 4), amp=0.0,
                   eta="inclusion", desc="2D unit square 128x128 affine, inclusion contrast 1e4"),
}

CONFIG_INDEX = {"C0": 0, "C1": 1, "C2": 2, "C3": 3, "C4": 4,
                "T3_4": 100, "T3_8": 101, "T3_16": 102, "T3_R": 103, "T2_R": 104, "T4_S": 105,
                "C0_32": 10, "C0_64": 11, "C0_128": 12}


# ---------------------------------------------------------------- geometry of the grids
def vertex_coords(mesh: MeshDesc, level: int) -> np.ndarray:
    """Reference coordinates of the vertices of ``level`` as [dim][n_vert]."""
    pn = mesh.p_nodes(level)
    axes = [np.linspace(0.0, mesh.extent[i], pn[i]) for i in range(mesh.dim)]
    grids = np.meshgrid(*axes, indexing="ij")           # axis 0 = x
    # lexicographic with x fastest: flatten in Fortran order over (x,y,z)
    return np.stack([g.ravel(order="F") for g in grids])


def velocity_node_coords(mesh: MeshDesc, level: int) -> np.ndarray:
    nn = mesh.vel_nodes(level)
    axes = [np.linspace(0.0, mesh.extent[i], nn[i]) for i in range(mesh.dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.ravel(order="F") for g in grids])


def dirichlet_node_mask(mesh: MeshDesc, level: int) -> np.ndarray:
    """Boolean [n_vel_nodes]: node lies on a wall face (all components fixed)."""
    nn = mesh.vel_nodes(level)
    idx = np.meshgrid(*[np.arange(n) for n in nn], indexing="ij")
    idx = [g.ravel(order="F") for g in idx]
    m = np.zeros(idx[0].shape, dtype=bool)
    for d in range(mesh.dim):
        if mesh.dirichlet_faces & (1 << (2 * d)):
            m |= idx[d] == 0
        if mesh.dirichlet_faces & (1 << (2 * d + 1)):
            m |= idx[d] == nn[d] - 1
    return m


def qpoint_ref_coords(mesh: MeshDesc, level: int) -> np.ndarray:
    """Reference coordinates of the coefficient samples, [n_cells][Q][dim]."""
    cells = mesh.cells(level)
    h = [mesh.extent[i] / cells[i] for i in range(mesh.dim)]
    cidx = np.meshgrid(*[np.arange(c) for c in cells], indexing="ij")
    cidx = [g.ravel(order="F") for g in cidx]            # per cell, x fastest
    q = np.meshgrid(*([np.arange(3)] * mesh.dim), indexing="ij")
    q = [g.ravel(order="F") for g in q]                  # per qpoint, x fastest
    out = np.empty((len(cidx[0]), 3 ** mesh.dim, mesh.dim))
    for d in range(mesh.dim):
        out[:, :, d] = (cidx[d][:, None] + _SAMPLE_PTS[q[d]][None, :]) * h[d]
    return out


# ---------------------------------------------------------------- random laws
def _sine_modes(rng: np.random.Generator, dim: int):
    k = rng.integers(1, 3, size=(4, dim))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=4)
    e = rng.normal(size=(4, dim))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    return k, phi, e


def _sine_displacement(X: np.ndarray, extent, amp: float, modes) -> np.ndarray:
    """d(X) = A*b(Xt)*(1/4)*sum_m e_m sin(2 pi k_m.Xt + phi_m); b vanishes on the boundary."""
    k, phi, e = modes
    dim = X.shape[0]
    Xt = X / np.asarray(extent, dtype=float)[:, None]
    b = np.ones(X.shape[1])
    for d in range(dim):
        b *= 4.0 * Xt[d] * (1.0 - Xt[d])
    out = np.zeros_like(X)
    for m in range(4):
        s = np.sin(2.0 * math.pi * (k[m] @ Xt) + phi[m])
        out += np.outer(e[m], s)
    return amp * b[None, :] * 0.25 * out


def _eta_law(cfg: dict, mesh: MeshDesc, rng: np.random.Generator, level_coords, contrast: Optional[float] = None):
    kind = cfg["eta"]
    if kind == "inclusion":
        c = 1e4 if contrast is None else contrast
        out = []
        for X in level_coords:
            inside = np.all((X >= 0.25) & (X <= 0.5), axis=-1)
            out.append(np.where(inside, c, 1.0))
        return out, None
    if kind == "strip":
        c = 1e6 if contrast is None else contrast
        out = []
        for X in level_coords:
            inside = (X[..., 0] >= 0.6) & (X[..., 0] <= 1.0) & (X[..., 1] >= 0.19) & (X[..., 1] <= 0.21)
            out.append(np.where(inside, 1e-3 * c, 1e-3))
        return out, None
    if kind == "loguniform":
        blk = cfg.get("block", 8)
        nb = [max(1, -(-mesh.n_fine[i] // blk)) for i in range(mesh.dim)]
        logeta = rng.uniform(-3.0, 3.0, size=tuple(nb[::-1]))   # indexed [z][y][x]
        hb = [mesh.extent[i] / mesh.n_fine[i] * blk for i in range(mesh.dim)]
        out = []
        for X in level_coords:
            bi = [np.minimum((X[..., d] / hb[d]).astype(np.int64), nb[d] - 1) for d in range(mesh.dim)]
            idx = tuple(bi[::-1])
            out.append(10.0 ** logeta[idx])
        return out, logeta
    raise ValueError(kind)


def make_mesh(name: str, dirichlet_faces: Optional[int] = None) -> MeshDesc:
    cfg = CONFIGS[name]
    dim = cfg["dim"]
    return MeshDesc(dim=dim, n_fine=tuple(cfg["n"]), extent=tuple(cfg["extent"]),
                    n_coarse=tuple(cfg["n_coarse"]),
                    dirichlet_faces=default_dirichlet_faces(dim) if dirichlet_faces is None
                    else dirichlet_faces)


def make_workload(name: str, step: Optional[int] = None, seed: int = BASE_SEED,
                  dirichlet_faces: Optional[int] = None,
                  prev_disp: Optional[np.ndarray] = None,
                  levels: Optional[Sequence[int]] = None,
                  contrast: Optional[float] = None) -> Workload:
    """Draw the inputs of workload ``name``.

    Draw order (numpy PCG64 seeded with ``[seed, config]`` or
    ``[seed, config, step]``): displacement modes, viscosity blocks, g_u
    (component-major, U[-1,1]), g_p (U[-1,1]); Dirichlet velocity entries are
    then zeroed.  For the time-step sequence the displacement of ``step`` is
    ``prev_disp`` plus a fresh increment.
    ``levels`` restricts which levels get coefficient arrays (all by default).
    ``contrast`` replaces the viscosity ratio of the inclusion (default 1e4) or the
    strip (default 1e6) laws.
    """
    cfg = CONFIGS[name]
    mesh = make_mesh(name, dirichlet_faces)
    key = [seed, CONFIG_INDEX[name]] + ([] if step is None else [step])
    rng = np.random.default_rng(key)
    dim = mesh.dim
    J = mesh.n_levels - 1
    Xv = vertex_coords(mesh, J)
    modes = _sine_modes(rng, dim)
    if cfg["amp"] > 0:
        disp = _sine_displacement(Xv, mesh.extent, cfg["amp"], modes)
    else:
        disp = np.zeros_like(Xv)
    if prev_disp is not None:
        disp = disp + prev_disp
    lvls = list(range(J + 1)) if levels is None else list(levels)
    coords = [qpoint_ref_coords(mesh, l) for l in lvls]
    eta_l, logeta = _eta_law(cfg, mesh, rng, coords, contrast)
    eta = [None] * (J + 1)
    cm = [None] * (J + 1)
    for l, e in zip(lvls, eta_l):
        eta[l] = np.ascontiguousarray(e, dtype=np.float64)
        cm[l] = np.full_like(eta[l], 1e2)
    del coords
    g_u = rng.uniform(-1.0, 1.0, size=mesh.n_vel(J))
    g_p = rng.uniform(-1.0, 1.0, size=mesh.n_p(J))
    mask = dirichlet_node_mask(mesh, J)
    g_u.reshape(dim, -1)[:, mask] = 0.0
    info = dict(config=name, desc=cfg["desc"], seed=seed, step=step,
                n_cells=mesh.n_cells(J), n_vel=mesh.n_vel(J), n_p=mesh.n_p(J),
                levels=mesh.n_levels)
    if logeta is not None:
        info["eta_contrast"] = float(10.0 ** (logeta.max() - logeta.min()))
    return Workload(name=name, mesh=mesh, disp=np.ascontiguousarray(disp), c_mass=cm, eta=eta,
                    g_u=g_u, g_p=g_p, info=info)


# ---------------------------------------------------------------- extension problem inputs
# The pseudo-elastic extension of Sec. 2 (the problem that defines Ext) with the
# mesh-quality coefficient law of Sec. 5: mu_A = 1 + 50 exp(-800 ((x - A_x)^2 +
# (y - A_y)^2)), evaluated at the reference quadrature-point coordinates, with A the
# control point (0.6, 0.2) of the channel benchmarks.  The boundary data is a smooth
# seeded field on the Dirichlet nodes (zero elsewhere).
EXT_STREAM = 7
EXT_POINT = (0.6, 0.2)


@dataclasses.dataclass
class ExtensionInputs:
    mu: list               # per level [n_cells][Q] mu_A
    g: np.ndarray          # fine-level [dim][n_vel_nodes] flattened; Dirichlet data, zero inside


def mu_law(X: np.ndarray) -> np.ndarray:
    """mu_A at reference points X[..., dim]."""
    r2 = (X[..., 0] - EXT_POINT[0]) ** 2 + (X[..., 1] - EXT_POINT[1]) ** 2
    return 1.0 + 50.0 * np.exp(-800.0 * r2)


def make_extension_inputs(name: str, mesh: MeshDesc, seed: int = BASE_SEED, amp: float = 0.01,
                          levels: Optional[Sequence[int]] = None, constant_mu: Optional[float] = None,
                          boundary_field=None) -> ExtensionInputs:
    """Coefficients and boundary data of the extension problem on ``mesh``.

    Draw order (PCG64 seeded with ``[seed, config, EXT_STREAM]``): the four sine modes of
    g(X) = amp * (1/4) sum_m e_m sin(2 pi k_m . X/extent + phi_m) on the Dirichlet nodes.
    ``constant_mu`` replaces the law by a constant; ``boundary_field(X)`` (X: [dim][n])
    replaces the drawn boundary data.
    """
    J = mesh.n_levels - 1
    rng = np.random.default_rng([seed, CONFIG_INDEX[name], EXT_STREAM])
    k, phi, e = _sine_modes(rng, mesh.dim)
    X = velocity_node_coords(mesh, J)
    if boundary_field is None:
        Xt = X / np.asarray(mesh.extent, dtype=float)[:, None]
        g = np.zeros_like(X)
        for m in range(4):
            g += np.outer(e[m], np.sin(2.0 * math.pi * (k[m] @ Xt) + phi[m]))
        g *= 0.25 * amp
    else:
        g = np.asarray(boundary_field(X), dtype=np.float64)
    g[:, ~dirichlet_node_mask(mesh, J)] = 0.0
    lvls = list(range(J + 1)) if levels is None else list(levels)
    mu = [None] * (J + 1)
    for l in lvls:
        Xq = qpoint_ref_coords(mesh, l)
        m = mu_law(Xq) if constant_mu is None else np.full(Xq.shape[:2], float(constant_mu))
        mu[l] = np.ascontiguousarray(m, dtype=np.float64)
    return ExtensionInputs(mu=mu, g=np.ascontiguousarray(g.ravel()))


# ---------------------------------------------------------------- corrector-mode inputs
# The corrector mode of Sec. 3.1.1 adds rho (grad v) v° (v° the known convective
# velocity) and the streamline term r (v° . grad v)(v° . grad w) of Sec. 3.2.  Inputs:
# v° per point, a smooth seeded field; rho consistent with the workloads' mass
# coefficient c_m = rho / (gamma tau) = 1e2 (second-order BDF, gamma = 2/3, and the time
# step tau = 0.005 of the 3D test); r per cell from the Peclet law of Sec. 3.2 with the
# cell's reference diameter h_K, max |v°| over its points, its mean eta and p1 = 2, and
# r = 0 where Pe_K < 1.
CONV_STREAM = 9
RHO_FLUID = 1.0e2 * (2.0 / 3.0) * 0.005


@dataclasses.dataclass
class ConvectionInputs:
    vconv: np.ndarray      # [n_cells][Q][dim]
    r: np.ndarray          # [n_cells][Q]
    rho: float


def make_convection_inputs(name: str, mesh: MeshDesc, level: int, eta: np.ndarray, seed: int = BASE_SEED,
                           speed: float = 1.0, rho: float = RHO_FLUID) -> ConvectionInputs:
    """v° = speed * (1/4) sum_m e_m sin(2 pi k_m . X/extent + phi_m) at the reference
    points (draw order: the four sine modes from PCG64 ``[seed, config, CONV_STREAM]``),
    and the streamline parameter per cell (Pe_K = |v°| h_K / (2 eta p1),
    r = h_K / (2 |v°| p1) (coth Pe_K - 1 / Pe_K), zero where Pe_K < 1)."""
    rng = np.random.default_rng([seed, CONFIG_INDEX[name], CONV_STREAM])
    k, phi, e = _sine_modes(rng, mesh.dim)
    X = qpoint_ref_coords(mesh, level)                       # [nc][Q][dim]
    Xt = X / np.asarray(mesh.extent, dtype=float)
    v = np.zeros_like(X)
    for m in range(4):
        v += np.sin(2.0 * math.pi * (Xt @ k[m]) + phi[m])[..., None] * e[m]
    v *= 0.25 * speed
    cells = mesh.cells(level)
    hK = math.sqrt(sum((mesh.extent[d] / cells[d]) ** 2 for d in range(mesh.dim)))
    vmax = np.sqrt((v ** 2).sum(axis=-1)).max(axis=1)        # per cell
    mu = eta.mean(axis=1)
    p1 = 2.0
    pe = vmax * hK / (2.0 * mu * p1)
    r = np.zeros_like(pe)
    on = pe >= 1.0
    r[on] = hK / (2.0 * vmax[on] * p1) * (1.0 / np.tanh(pe[on]) - 1.0 / pe[on])
    return ConvectionInputs(vconv=np.ascontiguousarray(v), r=np.ascontiguousarray(np.repeat(r[:, None], X.shape[1], 1)),
                            rho=float(rho))


def inject_displacement(mesh: MeshDesc, disp_fine: np.ndarray, level: int) -> np.ndarray:
    """Vertex displacement of ``level``: the fine values at the coarse vertices."""
    J = mesh.n_levels - 1
    s = 1 << (J - level)
    pf = mesh.p_nodes(J)
    arr = disp_fine.reshape((mesh.dim,) + tuple(pf[::-1]))
    if mesh.dim == 2:
        sub = arr[:, ::s, ::s]
    else:
        sub = arr[:, ::s, ::s, ::s]
    return np.ascontiguousarray(sub.reshape(mesh.dim, -1))


def random_vector(n: int, seed_key) -> np.ndarray:
    """A seeded U[-1,1] test vector (for parity tests)."""
    return np.random.default_rng(seed_key).uniform(-1.0, 1.0, size=n)


# ---------------------------------------------------------------- time-step (GCSI) inputs
# One step of the GCSI_2(P, C) scheme (Algorithm 1) on a channel with an elastic strip:
# the box [0, 2] x [0, 0.5] x [0, 0.5] (no-slip walls, x+ a do-nothing outflow) with a
# solid strip [0.5, 1.25] x [0.125, 0.25] spanning the channel depth (clamped by the
# z walls), cell-aligned on every level; the 2D cases are the x-y section of the same
# channel (the strip a rectangle attached to nothing, as the FSI2/FSI3-type flag is a
# rectangle in a 2D channel).  Material constants follow the FSI2-type
# setting of Sec. 5 (rho_f = 1e3, eta_f = 1, rho_s = 1e4, mu_s = 5e5, gravity 2 in -y,
# tau = 0.005, the volume-correction parameter 0.1); the extension coefficient is the law
# of Sec. 5 centred at the strip's tip.  The history (u, v, w at the two previous steps,
# the last pressure) is a set of smooth seeded fields vanishing on every face: four
# sine modes per field (as the displacement law), amplitude 0.005 for displacements and
# 0.5 for velocities; the mesh velocity w blends from v on the strip (the mesh moves with
# the solid) to its own sine field over the distance GCSI_BLEND from the strip, with the
# weight 1 - 3t^2 + 2t^3 of t = distance / GCSI_BLEND (continuous, so that the explicit
# geometry gamma tau w stays unfolded on fine meshes).
GCSI_STREAM = 11
GCSI_CONFIGS = {
    "G1": dict(n=(16, 4, 4), n_coarse=(8, 2, 2)),
    "G2": dict(n=(128, 32, 32), n_coarse=(8, 2, 2)),
    "G3": dict(n=(256, 64, 64), n_coarse=(8, 2, 2)),
    "G1_2D": dict(n=(32, 8), n_coarse=(8, 2)),
    "G2_2D": dict(n=(1024, 256), n_coarse=(8, 2)),
}
GCSI_EXTENT = (2.0, 0.5, 0.5)
GCSI_BLEND = 0.1
GCSI_STRIP = ((0.5, 1.25), (0.125, 0.25), (0.0, 0.5))
GCSI_CONFIG_INDEX = {"G1": 20, "G2": 21, "G3": 22, "G1_2D": 23, "G2_2D": 24}
GCSI_MATERIAL = dict(k=2, tau=0.005, rho_f=1e3, rho_s=1e4, eta_f=1.0, mu_s=5e5, eta_V=0.1,
                     body=(0.0, -2.0, 0.0))


@dataclasses.dataclass
class GcsiInputs:
    mesh: MeshDesc               # channel (walls, x+ outflow)
    ext_mesh: MeshDesc           # the same box with every face fixed (extension)
    solid_q: list                # per level [n_cells][Q] uint8: point inside the strip
    solid_cells: np.ndarray      # finest level [n_cells] uint8: cell inside the strip
    mu_A: list                   # per level [n_cells][Q]
    material: dict
    u: list                      # [u^{n-1}, u^{n-2}], each [n_vel] component-major
    v: list
    w: list
    p: np.ndarray                # [n_p]
    dirichlet: Optional[np.ndarray] = None   # [n_vel] velocity data on the Dirichlet nodes, or None


def _inside_strip(X: np.ndarray) -> np.ndarray:
    m = np.ones(X.shape[:-1], dtype=bool)
    for d in range(X.shape[-1]):
        lo, hi = GCSI_STRIP[d]
        m &= (X[..., d] >= lo) & (X[..., d] <= hi)
    return m


def _strip_weight(X: np.ndarray) -> np.ndarray:
    """1 on the strip, 0 beyond GCSI_BLEND from it, C^1 in between; X is [dim][n]."""
    d2 = np.zeros(X.shape[1])
    for d in range(X.shape[0]):
        lo, hi = GCSI_STRIP[d]
        d2 += np.maximum(np.maximum(lo - X[d], X[d] - hi), 0.0) ** 2
    t = np.minimum(np.sqrt(d2) / GCSI_BLEND, 1.0)
    return 1.0 - t * t * (3.0 - 2.0 * t)


def make_gcsi_inputs(name: str = "G1", seed: int = BASE_SEED, inflow: float = 0.0) -> GcsiInputs:
    """Draw the inputs of one GCSI step on the channel-with-strip ``name``.

    Draw order (PCG64 ``[seed, config, GCSI_STREAM]``): sine modes of u^{n-1}, u^{n-2},
    v^{n-1}, v^{n-2}, w^{n-1}, w^{n-2}, then p (U[-1, 1]) at the pressure nodes.
    ``inflow`` > 0 adds Dirichlet data on the inflow face x = 0: the x-velocity
    16 inflow y (H - y) z (W - z) / (H^2 W^2) in 3D, 4 inflow y (H - y) / H^2 in 2D (peak
    ``inflow`` at the centre, zero on the edges), zero on the other walls; the velocity
    history then carries the same profile, scaled by (1 - x / L), so that it matches the
    data on the inflow face."""
    cfg = GCSI_CONFIGS[name]
    dim = len(cfg["n"])
    mesh = MeshDesc(dim=dim, n_fine=tuple(cfg["n"]), extent=GCSI_EXTENT[:dim], n_coarse=tuple(cfg["n_coarse"]),
                    dirichlet_faces=default_dirichlet_faces(dim))
    ext_mesh = dataclasses.replace(mesh, dirichlet_faces=(1 << (2 * dim)) - 1)
    J = mesh.n_levels - 1
    rng = np.random.default_rng([seed, GCSI_CONFIG_INDEX[name], GCSI_STREAM])
    X = velocity_node_coords(mesh, J)

    def field(amp):
        return np.ascontiguousarray(_sine_displacement(X, mesh.extent, amp, _sine_modes(rng, dim)).ravel())

    u = [field(0.005), field(0.005)]
    v = [field(0.5), field(0.5)]
    w = [field(0.5), field(0.5)]
    p = rng.uniform(-1.0, 1.0, size=mesh.n_p(J))
    solid_q, mu_A = [], []
    tip = (GCSI_STRIP[0][1], 0.5 * (GCSI_STRIP[1][0] + GCSI_STRIP[1][1]))
    for l in range(J + 1):
        Xq = qpoint_ref_coords(mesh, l)
        solid_q.append(np.ascontiguousarray(_inside_strip(Xq).astype(np.uint8)))
        r2 = (Xq[..., 0] - tip[0]) ** 2 + (Xq[..., 1] - tip[1]) ** 2
        mu_A.append(np.ascontiguousarray(1.0 + 50.0 * np.exp(-800.0 * r2)))
    cells = mesh.cells(J)
    h = [mesh.extent[d] / cells[d] for d in range(dim)]
    ci = np.meshgrid(*[np.arange(c) for c in cells], indexing="ij")
    centres = np.stack([(g.ravel(order="F") + 0.5) * h[d] for d, g in enumerate(ci)], axis=-1)
    solid_cells = np.ascontiguousarray(_inside_strip(centres).astype(np.uint8))
    dirichlet = None
    if inflow > 0:
        L, H = mesh.extent[0], mesh.extent[1]
        if dim == 3:
            Wd = mesh.extent[2]
            prof = 16.0 * inflow * X[1] * (H - X[1]) * X[2] * (Wd - X[2]) / (H * H * Wd * Wd)
        else:
            prof = 4.0 * inflow * X[1] * (H - X[1]) / (H * H)
        dirichlet = np.zeros_like(X)
        dirichlet[0] = np.where(X[0] == 0.0, prof, 0.0)
        dirichlet = np.ascontiguousarray(dirichlet.ravel())
        for i in range(2):
            v[i].reshape(dim, -1)[0] += prof * (1.0 - X[0] / L)
    # the mesh velocity follows the velocity on (and near) the solid
    phi = _strip_weight(X)
    for i in range(2):
        wi, vi = w[i].reshape(dim, -1), v[i].reshape(dim, -1)
        wi[:] = phi * vi + (1.0 - phi) * wi
    return GcsiInputs(mesh=mesh, ext_mesh=ext_mesh, solid_q=solid_q, solid_cells=solid_cells, mu_A=mu_A,
                      material=dict(GCSI_MATERIAL), u=u, v=v, w=w, p=p, dirichlet=dirichlet)
