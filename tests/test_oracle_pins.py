"""Pins of the CPU oracle against closed forms, invariants and rates.

Nothing here compares the oracle with itself: every expected value comes from
a closed form (1D element integrals, Gauss exactness, Chebyshev polynomials,
exact polynomial integrals over the box), an invariant that holds for the
exact operator (symmetry, rigid-motion null space, volume, divergence of
linear fields), a special case that reduces to a textbook solve, or an
asymptotic rate.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import fem, solvers
from paper_2305_08986_amd import workloads as W

# 1D closed forms on a cell of length h (nodes 0, h/2, h for Q2; 0, h for Q1)
def M1(h):
    return h / 30.0 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]], float)


def K1(h):
    return 1.0 / (3.0 * h) * np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]], float)


C1 = np.array([[-3, -4, 1], [4, 0, -4], [-1, 4, 3]], float) / 6.0     # int N_i' N_j
E1 = np.array([[-5, 4, 1], [-1, -4, 5]], float) / 6.0                 # int L_k N_j'


def F1(h):
    return h / 6.0 * np.array([[1, 2, 0], [0, 2, 1]], float)          # int L_k N_j


def bubble_disp(box, amp, seed=0):
    """Smooth displacement vanishing on the boundary (mapped domain = the box)."""
    X = box.vertex_coords()
    rng = np.random.default_rng(seed)
    Xt = X / np.asarray(box.extent)[:, None]
    b = np.prod(4 * Xt * (1 - Xt), axis=0)
    out = np.zeros_like(X)
    for d in range(box.dim):
        k = rng.integers(1, 3, size=box.dim)
        out[d] = amp * b * np.sin(2 * np.pi * (k @ Xt) + rng.uniform(0, 6.28))
    return out


def test_gauss_rule_closed_form_and_exactness():
    x, w = fem.gauss_rule(3)
    s = math.sqrt(15) / 10
    assert np.allclose(x, [0.5 - s, 0.5, 0.5 + s], atol=1e-16, rtol=0)
    assert np.allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-16, rtol=0)
    for k in range(6):
        assert abs(w @ x ** k - 1.0 / (k + 1)) < 1e-15
    assert abs(w @ x ** 6 - 1.0 / 7) > 1e-5          # degree 6 is not exact


def test_lagrange_closed_forms():
    x = np.linspace(-0.3, 1.3, 17)
    v, d = fem.lagrange_1d(fem.Q2_NODES, x)
    assert np.allclose(v[:, 0], (1 - 2 * x) * (1 - x), atol=1e-14)
    assert np.allclose(v[:, 1], 4 * x * (1 - x), atol=1e-14)
    assert np.allclose(v[:, 2], x * (2 * x - 1), atol=1e-14)
    assert np.allclose(d[:, 0], 4 * x - 3, atol=1e-14)
    assert np.allclose(d[:, 1], 4 - 8 * x, atol=1e-14)
    assert np.allclose(d[:, 2], 4 * x - 1, atol=1e-14)
    v, d = fem.lagrange_1d(fem.Q1_NODES, x)
    assert np.allclose(v, np.stack([1 - x, x], 1), atol=1e-15)
    assert np.allclose(d, np.stack([-np.ones_like(x), np.ones_like(x)], 1), atol=1e-15)


def _single_cell(dim, h, cm, eta):
    ref = fem.Reference(dim)
    box = fem.Box(dim, (1,) * dim, tuple(h), 0)
    J = fem.jacobians_q1(box, np.zeros((dim, box.n_p)), ref)
    A, B = fem.element_matrices(J, np.full((1, 3 ** dim), cm), np.full((1, 3 ** dim), eta), ref)
    return A[0], B[0]


def test_element_matrices_2d_tensor_closed_form():
    hx, hy, cm, eta = 0.37, 0.21, 3.0, 1.7
    A, B = _single_cell(2, (hx, hy), cm, eta)
    Mx, My, Kx, Ky = M1(hx), M1(hy), K1(hx), K1(hy)
    mass = np.kron(My, Mx)
    lap = np.kron(My, Kx) + np.kron(Ky, Mx)
    A00 = cm * mass + eta * (lap + np.kron(My, Kx))
    A11 = cm * mass + eta * (lap + np.kron(Ky, Mx))
    A01 = eta * np.kron(C1, C1.T)          # int d_y phi_n d_x phi_m
    ref = np.block([[A00, A01], [A01.T, A11]])
    assert np.allclose(A, ref, rtol=0, atol=1e-14 * np.abs(ref).max())
    Bx = np.kron(F1(hy), E1)
    By = np.kron(E1, F1(hx))
    refB = np.concatenate([Bx, By], axis=1)
    assert np.allclose(B, refB, rtol=0, atol=1e-14 * np.abs(refB).max())


def test_element_matrices_3d_tensor_closed_form():
    h = (0.5, 0.3, 0.7)
    cm, eta = 2.0, 0.9
    A, B = _single_cell(3, h, cm, eta)
    M = [M1(t) for t in h]
    K = [K1(t) for t in h]
    F = [F1(t) for t in h]
    k3 = lambda a, b, c: np.kron(c, np.kron(b, a))       # x fastest
    mass = k3(M[0], M[1], M[2])
    d2 = [k3(K[0], M[1], M[2]), k3(M[0], K[1], M[2]), k3(M[0], M[1], K[2])]
    lap = sum(d2)
    n = 27
    for a in range(3):
        ref = cm * mass + eta * (lap + d2[a])
        blk = A[a * n:(a + 1) * n, a * n:(a + 1) * n]
        assert np.allclose(blk, ref, rtol=0, atol=1e-14 * np.abs(ref).max())
    # (0,1) block: int d_y phi_n d_x phi_m = [int N_i N'_i'] [int N'_j N_j'] [int N_k N_k']
    ref01 = eta * k3(C1.T, C1, M[2])
    assert np.allclose(A[0:n, n:2 * n], ref01, rtol=0, atol=1e-14 * np.abs(ref01).max())
    ref02 = eta * k3(C1.T, M[1], C1)
    assert np.allclose(A[0:n, 2 * n:], ref02, rtol=0, atol=1e-14 * np.abs(ref02).max())
    Bz = k3(F[0], F[1], E1)
    assert np.allclose(B[:, 2 * n:], Bz, rtol=0, atol=1e-14 * np.abs(Bz).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_symmetry_on_warped_mesh(dim):
    box = fem.Box(dim, (3,) * dim, (1.0,) * dim, 0)
    ref = fem.Reference(dim)
    J = fem.jacobians_q1(box, bubble_disp(box, 0.04), ref)
    rng = np.random.default_rng(1)
    eta = 10 ** rng.uniform(-3, 3, size=(box.n_cells, 3 ** dim))
    cm = rng.uniform(0, 5, size=(box.n_cells, 3 ** dim))
    op = fem.assemble(box, J, cm, eta, ref)
    x, y = rng.normal(size=(2, box.n_vel))
    lhs, rhs = x @ (op.A @ y), y @ (op.A @ x)
    assert abs(lhs - rhs) <= 1e-13 * abs(x) @ (abs(op.A) @ abs(y))


@pytest.mark.parametrize("dim", [2, 3])
def test_rigid_motions_in_null_space(dim):
    """eps(a + W x) = 0 for skew W, and linear fields lie in the mapped Q2 space."""
    box = fem.Box(dim, (3, 2, 2)[:dim], (1.0, 0.8, 0.9)[:dim], 0)
    ref = fem.Reference(dim)
    disp = bubble_disp(box, 0.05, seed=3)
    J = fem.jacobians_q1(box, disp, ref)
    rng = np.random.default_rng(2)
    eta = 10 ** rng.uniform(-3, 3, size=(box.n_cells, 3 ** dim))
    op = fem.assemble(box, J, np.zeros_like(eta), eta, ref)
    # physical coordinates of the Q2 nodes: Q1 map evaluated at the nodes
    Xn = box.vel_node_ref_coords()
    dn = _q1_interp_at_nodes(box, disp)
    x = Xn + dn
    modes = [np.eye(dim)[a][:, None] * np.ones_like(x[0]) for a in range(dim)]
    for (a, b) in [(0, 1), (0, 2), (1, 2)][: (1 if dim == 2 else 3)]:
        r = np.zeros_like(x)
        r[a] = -x[b]
        r[b] = x[a]
        modes.append(r)
    An = abs(op.A).max() * op.A.shape[0]
    for r in modes:
        v = r.ravel()
        assert np.linalg.norm(op.A @ v) <= 1e-12 * An * np.linalg.norm(v)
    # a strain field is NOT in the null space (sanity of the pin)
    s = np.zeros_like(x)
    s[0] = x[0]
    assert np.linalg.norm(op.A @ s.ravel()) > 1e-3 * np.linalg.norm(s)


def test_element_by_element_apply_invariants():
    """The element-by-element apply (used where no global matrix fits): the mass of a
    constant field is the mapped volume, rigid motions give zero viscous response on a
    warped mesh with random eta, the result does not depend on how the cells are
    split into blocks, and on a box with walls it is A u on the free rows."""
    box = fem.Box(3, (3, 2, 2), (1.0, 0.8, 0.9), 0)
    ref = fem.Reference(3)
    disp = bubble_disp(box, 0.05, seed=4)
    rng = np.random.default_rng(6)
    cells = np.arange(box.n_cells)
    one = np.ones((box.n_cells, 27))
    vol = float(np.prod(box.extent))
    for a in range(3):
        e = np.zeros(box.n_vel)
        e[a * box.n_vel_nodes:(a + 1) * box.n_vel_nodes] = 1.0
        d, v = fem.apply_ebe(box, disp, one, 0 * one, ref, e, cells)
        assert abs(v @ e[d] - vol) < 1e-13 * vol
    eta = 10 ** rng.uniform(-3, 3, size=(box.n_cells, 27))
    x = box.vel_node_ref_coords() + _q1_interp_at_nodes(box, disp)
    r = np.zeros_like(x)
    r[0], r[1] = -x[1], x[0]
    d, v = fem.apply_ebe(box, disp, 0 * one, eta, ref, r.ravel(), cells)
    trans = np.repeat([1.0, 0.0, 0.0], box.n_vel_nodes)
    d1, v1 = fem.apply_ebe(box, disp, 0 * one, eta, ref, trans, cells)
    assert np.abs(v).max() <= 1e-12 * eta.max() and np.abs(v1).max() <= 1e-12 * eta.max()
    s = np.zeros_like(x)
    s[0] = x[0]
    _, vs = fem.apply_ebe(box, disp, 0 * one, eta, ref, s.ravel(), cells)
    assert np.abs(vs).max() > 1e-3
    # walls, random data: blocks of cells summed = A u on the free rows
    wbox = fem.Box(3, (3, 2, 2), (1.0, 0.8, 0.9), W.default_dirichlet_faces(3))
    cm = rng.uniform(0, 5, size=(box.n_cells, 27))
    u = rng.normal(size=box.n_vel)
    op = fem.assemble(wbox, fem.jacobians_q1(wbox, disp, ref), cm, eta, ref)
    acc = np.zeros(box.n_vel)
    for blk in (cells[:5], cells[5:7], cells[7:]):
        d, v = fem.apply_ebe(wbox, disp, cm, eta, ref, u, blk)
        np.add.at(acc, d, v)
    free = ~wbox.dirichlet_vel_dofs()
    ref_v = op.A @ u
    assert np.allclose(acc[free], ref_v[free], rtol=0, atol=1e-13 * np.abs(ref_v).max())
    assert not acc[~free].any()


def _q1_interp_at_nodes(box, disp):
    """Displacement interpolated (multilinear) at every Q2 node."""
    nn = box.vel_nodes
    out = np.zeros((box.dim, box.n_vel_nodes))
    pn = box.p_nodes
    g = np.meshgrid(*[np.arange(n) for n in nn], indexing="ij")
    g = [a.ravel(order="F") for a in g]
    # node i along an axis sits at vertex i//2 (+1/2 if odd)
    lo = [np.minimum(a // 2, pn[d] - 2) for d, a in enumerate(g)]
    t = [(a - 2 * l) / 2.0 for a, l in zip(g, lo)]
    import itertools
    for corner in itertools.product([0, 1], repeat=box.dim):
        w = np.ones(box.n_vel_nodes)
        idx = np.zeros(box.n_vel_nodes, dtype=np.int64)
        stride = 1
        for d in range(box.dim):
            w *= t[d] if corner[d] else (1 - t[d])
            idx += (lo[d] + corner[d]) * stride
            stride *= pn[d]
        out += w * disp[:, idx]
    return out


def _box_integral_of_poly(f, dim, extent, npts=8):
    """Tensor Gauss integral over the box (exact for the low-degree integrands used)."""
    x, w = np.polynomial.legendre.leggauss(npts)
    pts = [(x + 1) / 2 * e for e in extent]
    ws = [w / 2 * e for e in extent]
    G = np.meshgrid(*pts, indexing="ij")
    Wt = np.ones_like(G[0])
    for d in range(dim):
        sh = [1] * dim
        sh[d] = npts
        Wt = Wt * ws[d].reshape(sh)
    return float(np.sum(f(*G) * Wt))


def test_quadratic_fields_energy_exact_on_warped_box():
    """u^T A v = int 2 eps(u):eps(v) for quadratic u, v on a Q1-warped mesh of the box.

    The mapped domain is the box itself; quadratics in x lie in the mapped Q2
    space, and the integrand has degree <= 4 per reference variable.
    """
    dim = 3
    box = fem.Box(dim, (2, 3, 2), (1.0, 1.2, 0.8), 0)
    ref = fem.Reference(dim)
    disp = bubble_disp(box, 0.04, seed=5)
    J = fem.jacobians_q1(box, disp, ref)
    one = np.ones((box.n_cells, 27))
    op = fem.assemble(box, J, 0 * one, one, ref)
    x = box.vel_node_ref_coords() + _q1_interp_at_nodes(box, disp)
    rng = np.random.default_rng(7)
    cu = rng.normal(size=(dim, 10))
    cv = rng.normal(size=(dim, 10))

    def quad_field(c, X):        # u_a = c0 + c.x + xy, xz, yz, x^2... terms
        mon = [np.ones_like(X[0]), X[0], X[1], X[2], X[0] * X[1], X[0] * X[2],
               X[1] * X[2], X[0] ** 2, X[1] ** 2, X[2] ** 2]
        return np.stack([sum(c[a, m] * mon[m] for m in range(10)) for a in range(dim)])

    def quad_grad(c, X):          # grad[a][b] = d u_a / d x_b
        g = np.zeros((dim, dim) + X[0].shape)
        for a in range(dim):
            g[a, 0] = c[a, 1] + c[a, 4] * X[1] + c[a, 5] * X[2] + 2 * c[a, 7] * X[0]
            g[a, 1] = c[a, 2] + c[a, 4] * X[0] + c[a, 6] * X[2] + 2 * c[a, 8] * X[1]
            g[a, 2] = c[a, 3] + c[a, 5] * X[0] + c[a, 6] * X[1] + 2 * c[a, 9] * X[2]
        return g

    u = quad_field(cu, x).ravel()
    v = quad_field(cv, x).ravel()

    def integrand(X, Y, Z):
        P = np.stack([X, Y, Z])
        gu, gv = quad_grad(cu, P), quad_grad(cv, P)
        eu = 0.5 * (gu + gu.transpose(1, 0, *range(2, gu.ndim)))
        ev = 0.5 * (gv + gv.transpose(1, 0, *range(2, gv.ndim)))
        return 2 * np.sum(eu * ev, axis=(0, 1))

    exact = _box_integral_of_poly(integrand, dim, box.extent)
    assert abs(u @ (op.A @ v) - exact) <= 1e-12 * abs(exact)


def test_mass_and_volume_on_warped_box():
    for dim in (2, 3):
        box = fem.Box(dim, (3, 2, 2)[:dim], (1.1, 0.9, 0.7)[:dim], 0)
        ref = fem.Reference(dim)
        J = fem.jacobians_q1(box, bubble_disp(box, 0.05, seed=11), ref)
        _, wdet = fem.geometry_factors(J, ref)
        vol = float(np.prod(box.extent))
        assert abs(wdet.sum() - vol) < 1e-14 * vol
        one = np.ones((box.n_cells, 3 ** dim))
        op = fem.assemble(box, J, one, 0 * one, ref)
        for a in range(dim):
            e = np.zeros(box.n_vel)
            e[a * box.n_vel_nodes:(a + 1) * box.n_vel_nodes] = 1.0
            assert abs(e @ (op.A @ e) - vol) < 1e-13 * vol


def test_cell_area_shoelace_2d():
    box = fem.Box(2, (4, 3), (1.0, 1.0), 0)
    ref = fem.Reference(2)
    rng = np.random.default_rng(4)
    disp = rng.uniform(-0.05, 0.05, size=(2, box.n_p))      # arbitrary bilinear quads
    J = fem.jacobians_q1(box, disp, ref)
    _, wdet = fem.geometry_factors(J, ref)
    X = box.vertex_coords() + disp
    vn = box.cell_p_nodes()
    for c in range(box.n_cells):
        ids = vn[c][[0, 1, 3, 2]]                # counter-clockwise
        xs, ys = X[0, ids], X[1, ids]
        area = 0.5 * abs(np.dot(xs, np.roll(ys, -1)) - np.dot(ys, np.roll(xs, -1)))
        assert abs(wdet[c].sum() - area) < 1e-15 * 10


def test_hex_volume_independent_rule():
    """Trilinear det J has degree <= 2 per variable: 3- and 5-point Gauss agree."""
    box = fem.Box(3, (2, 2, 2), (1.0, 1.0, 1.0), 0)
    rng = np.random.default_rng(8)
    disp = rng.uniform(-0.06, 0.06, size=(3, box.n_p))
    r3 = fem.Reference(3, 3)
    r5 = fem.Reference(3, 5)
    w3 = fem.geometry_factors(fem.jacobians_q1(box, disp, r3), r3)[1].sum(1)
    w5 = fem.geometry_factors(fem.jacobians_q1(box, disp, r5), r5)[1].sum(1)
    assert np.allclose(w3, w5, rtol=1e-14, atol=0)


def test_divergence_of_linear_field():
    for dim in (2, 3):
        box = fem.Box(dim, (3, 2, 3)[:dim], (1.0, 0.6, 0.9)[:dim], 0)
        ref = fem.Reference(dim)
        disp = bubble_disp(box, 0.05, seed=9)
        J = fem.jacobians_q1(box, disp, ref)
        one = np.ones((box.n_cells, 3 ** dim))
        op = fem.assemble(box, J, one, one, ref)
        x = box.vel_node_ref_coords() + _q1_interp_at_nodes(box, disp)
        G = np.random.default_rng(10).normal(size=(dim, dim))
        u = (G @ x).ravel()
        vol = float(np.prod(box.extent))
        assert abs(op.B @ u @ np.ones(box.n_p) - np.trace(G) * vol) < 1e-13 * vol * abs(G).sum()
    # per pressure node on an affine mesh: int psi_k = h^d * (#cells at vertex) / 2^d
    box = fem.Box(2, (3, 2), (0.9, 0.4), 0)
    ref = fem.Reference(2)
    J = fem.jacobians_q1(box, np.zeros((2, box.n_p)), ref)
    one = np.ones((box.n_cells, 9))
    op = fem.assemble(box, J, one, one, ref)
    xn = box.vel_node_ref_coords()
    u = np.concatenate([2.0 * xn[0], -0.5 * xn[1]])        # tr = 1.5
    hx, hy = 0.3, 0.2
    cnt = np.array([len(box.cells_of_p_node(k)) for k in range(box.n_p)])
    assert np.allclose(op.B @ u, 1.5 * hx * hy * cnt / 4, rtol=1e-13, atol=0)


def test_dirichlet_structure():
    wl = W.make_workload("C0")
    box = fem.level_box(wl.mesh, 2)
    ref = fem.Reference(2)
    J = fem.jacobians_q1(box, wl.disp, ref)
    op = fem.assemble(box, J, wl.c_mass[2], wl.eta[2], ref)
    assert op.A.shape == (2178, 2178) and op.B.shape == (289, 2178)
    dm = op.dir_mask
    Ad = op.A[dm][:, dm].toarray()
    assert np.array_equal(Ad, np.eye(dm.sum()))
    assert op.A[dm][:, ~dm].nnz == 0 and op.A[~dm][:, dm].nnz == 0
    assert op.B[:, dm].nnz == 0
    # no-slip on x-, y-, y+; x+ is free
    nn = box.vel_nodes
    ix = np.arange(box.n_vel_nodes) % nn[0]
    assert dm[: box.n_vel_nodes][ix == 0].all() and not dm[: box.n_vel_nodes][(ix == nn[0] - 1)].all()


def _manufactured_2d(n, warp):
    box = fem.Box(2, (n, n), (1.0, 1.0), 0b1111)
    ref = fem.Reference(2)
    disp = bubble_disp(box, 0.03, seed=1) if warp else np.zeros((2, box.n_p))
    J = fem.jacobians_q1(box, disp, ref)
    one = np.ones((box.n_cells, 9))
    op = fem.assemble(box, J, one, one, ref)
    pi = np.pi
    U = lambda x, y: np.stack([2 * pi * np.sin(pi * x) ** 2 * np.sin(pi * y) * np.cos(pi * y),
                               -2 * pi * np.sin(pi * x) * np.cos(pi * x) * np.sin(pi * y) ** 2])
    P = lambda x, y: np.cos(pi * x) * np.cos(pi * y)

    def lapU(x, y):
        s, c = np.sin, np.cos
        a = 2 * pi * (2 * pi ** 2 * c(2 * pi * x) * s(pi * y) * c(pi * y)
                      + s(pi * x) ** 2 * (-4 * pi ** 2) * s(pi * y) * c(pi * y))
        b = -2 * pi * (s(pi * x) * c(pi * x) * (-4 * pi ** 2) * s(pi * y) ** 2
                       + 2 * pi ** 2 * c(2 * pi * y) * s(pi * x) * c(pi * x))
        return np.stack([a, b])

    def gradP(x, y):
        return np.stack([-pi * np.sin(pi * x) * np.cos(pi * y), -pi * np.cos(pi * x) * np.sin(pi * y)])

    f = lambda x, y: U(x, y) - lapU(x, y) - gradP(x, y)
    # load vector and errors with a 5-point rule
    r5 = fem.Reference(2, 5)
    X = box.vertex_coords() + disp
    vn = box.cell_p_nodes()
    xq = np.einsum("qv,acv->acq", r5.psi, X[:, vn])             # physical qpoints [2][c][q]
    J5 = fem.jacobians_q1(box, disp, r5)
    wdet5 = fem.geometry_factors(J5, r5)[1]
    fq = f(xq[0], xq[1])                                          # [2][c][q]
    gd = np.concatenate([box.cell_vel_nodes() + a * box.n_vel_nodes for a in range(2)], axis=1)
    loc = np.einsum("acq,cq,qi->cai", fq, wdet5, r5.phi).reshape(box.n_cells, -1)
    g = np.zeros(box.n_vel)
    np.add.at(g, gd, loc)
    g[op.dir_mask] = 0.0
    # mean-zero pressure through a Lagrange multiplier
    mvec = np.zeros(box.n_p)
    np.add.at(mvec, box.cell_p_nodes(), np.einsum("cq,qk->ck", wdet5, r5.psi))
    Mfull = sp.bmat([[op.A, op.B.T, None], [op.B, None, sp.csr_matrix(mvec[:, None])],
                     [None, sp.csr_matrix(mvec[None, :]), None]], format="csc")
    sol = sp.linalg.spsolve(Mfull, np.concatenate([g, np.zeros(box.n_p + 1)]))
    u, p = sol[: box.n_vel], sol[box.n_vel: box.n_vel + box.n_p]
    uh = np.einsum("qi,cai->acq", r5.phi, u[gd].reshape(box.n_cells, 2, 9))
    ph = np.einsum("qk,ck->cq", r5.psi, p[box.cell_p_nodes()])
    eu = math.sqrt(np.sum(((uh - U(xq[0], xq[1])) ** 2).sum(0) * wdet5))
    ep = math.sqrt(np.sum((ph - P(xq[0], xq[1])) ** 2 * wdet5))
    return eu, ep


@pytest.mark.slow
@pytest.mark.parametrize("warp", [False, True])
def test_manufactured_convergence_rates(warp):
    errs = [_manufactured_2d(n, warp) for n in (8, 16, 32)]
    ru = [math.log2(errs[i][0] / errs[i + 1][0]) for i in range(2)]
    rp = [math.log2(errs[i][1] / errs[i + 1][1]) for i in range(2)]
    assert min(ru) >= 2.8, ru
    assert min(rp) >= 1.8, rp


def test_direct_solve_residual_c0():
    wl = W.make_workload("C0")
    ops = solvers.build_levels(wl.mesh, wl.disp, wl.c_mass, wl.eta)
    u, p = solvers.direct_solve(ops[-1], wl.g_u, wl.g_p)
    a, b = ops[-1].apply_stokes(u, p)
    g = np.concatenate([wl.g_u, wl.g_p])
    x = np.concatenate([u, p])
    r = np.linalg.norm(np.concatenate([a, b]) - g)
    # normwise backward error at FP64 rounding level; the pressure in the stiff
    # inclusion is ~1e7, so |M||x| is ~1e12 ||g|| and r/||g|| floors near 1e-11
    M = ops[-1].stokes()
    assert r <= 1e-15 * (np.linalg.norm(abs(M) @ abs(x)) + np.linalg.norm(g))
    assert r <= 1e-10 * np.linalg.norm(g)


def test_prolongation_stencils_and_reproduction():
    coarse = fem.Box(1 + 1, (2, 1), (1.0, 0.5), 0)
    fine = fem.Box(2, (4, 2), (1.0, 0.5), 0)
    P = fem_prol = solvers.prolongation_1field(coarse, fine, fem.Q2_NODES, 1).toarray()
    # x-line of fine nodes on y = 0 (rows 0..8) against coarse x-line (cols 0..4)
    line = P[:9, :5]
    exp = np.zeros((9, 5))
    rows = {0: [1, 0, 0], 1: [3 / 8, 3 / 4, -1 / 8], 2: [0, 1, 0], 3: [-1 / 8, 3 / 4, 3 / 8], 4: [0, 0, 1]}
    for cell in range(2):
        for f, r in rows.items():
            exp[4 * cell + f, 2 * cell:2 * cell + 3] = r
    assert np.array_equal(line, exp)
    Pp = solvers.prolongation_1field(coarse, fine, fem.Q1_NODES, 1).toarray()
    assert np.array_equal(Pp[:5, :3], np.array([[1, 0, 0], [.5, .5, 0], [0, 1, 0], [0, .5, .5], [0, 0, 1]]))
    # any coarse Q2 function (here a biquadratic) is reproduced exactly
    xc = coarse.vel_node_ref_coords()
    xf = fine.vel_node_ref_coords()
    q = lambda X: 1 + X[0] - 2 * X[1] + 3 * X[0] * X[1] + X[0] ** 2 * X[1] ** 2 - X[1] ** 2
    assert np.allclose(P @ q(xc), q(xf), rtol=0, atol=1e-14)


def _cheb_T(k, t):
    return np.cos(k * np.arccos(t)) if np.all(np.abs(t) <= 1) else np.cosh(k * np.arccosh(np.abs(t))) * np.sign(t) ** k


def test_chebyshev_matches_closed_form_polynomial():
    lam = np.linspace(0.05, 2.0, 40)
    b = np.random.default_rng(3).normal(size=40)
    lo, hi = 0.1, 2.2
    for k in (1, 2, 4, 6):
        x = solvers.chebyshev(lambda v: lam * v, np.ones(40), b, k, lo, hi)
        theta, delta = (hi + lo) / 2, (hi - lo) / 2
        t = (theta - lam) / delta
        Tk = np.array([np.cos(k * np.arccos(s)) if abs(s) <= 1 else np.cosh(k * np.arccosh(abs(s))) * np.sign(s) ** k
                       for s in t])
        exact = (1 - Tk / np.cosh(k * np.arccosh(theta / delta))) * b / lam
        assert np.allclose(x, exact, rtol=1e-13, atol=1e-14)


def test_block_smoother_exact_with_exact_blocks():
    wl = W.make_workload("T3_4")
    ops = solvers.build_levels(wl.mesh, wl.disp, wl.c_mass, wl.eta)
    op = ops[0]
    A = op.A.toarray()
    B = op.B.toarray()
    Ainv = np.linalg.inv(A)
    S = B @ Ainv @ B.T
    rng = np.random.default_rng(12)
    ru, rp = rng.normal(size=op.box.n_vel), rng.normal(size=op.box.n_p)
    yu, yp = solvers.block_smoother(lambda r: Ainv @ r, lambda t: np.linalg.solve(S, t), op.B, ru, rp)
    M = op.stokes().toarray()
    assert np.allclose(M @ np.concatenate([yu, yp]), np.concatenate([ru, rp]), rtol=0,
                       atol=1e-10 * np.linalg.norm(np.concatenate([ru, rp])))


def test_minres_one_step_is_the_p_norm_minimiser():
    rng = np.random.default_rng(13)
    Q = rng.normal(size=(30, 30))
    S = Q @ Q.T + 30 * np.eye(30)
    dinv = 1.0 / rng.uniform(0.5, 3.0, size=30)
    r = rng.normal(size=30)
    x, y, beta = solvers.minres1(lambda z: S @ z, dinv, r)
    z = dinv * r
    # brute force: ||r - b S z||_P^2 = a b^2 - 2 c b + const, minimised on a fine grid
    bs = np.linspace(beta - 1, beta + 1, 20001)
    f = [(r - t * (S @ z)) @ (dinv * (r - t * (S @ z))) for t in bs[::100]]
    tb = bs[::100][int(np.argmin(f))]
    assert abs(tb - beta) <= 0.011
    # stationarity of the P-norm residual at beta
    res = r - beta * (S @ z)
    assert abs((S @ z) @ (dinv * res)) <= 1e-12 * np.linalg.norm(S @ z) * np.linalg.norm(res) * dinv.max()


def test_lanczos_estimate_brackets_true_lambda_max():
    for name in ("C0", "T3_4"):
        wl = W.make_workload(name)
        ops = solvers.build_levels(wl.mesh, wl.disp, wl.c_mass, wl.eta)
        for op in ops:
            A = op.A.toarray()
            d = np.diag(A)
            free = ~op.dir_mask
            ev = sla.eigvalsh(A[np.ix_(free, free)] / np.sqrt(np.outer(d[free], d[free])))
            lam, _, _ = solvers.lanczos_lambda_max(op.A, d, free.astype(float), 12)
            assert lam <= ev[-1] * (1 + 1e-12)
            assert lam >= 0.9 * ev[-1]
            assert 1.2 * lam >= ev[-1]


def test_fgmres_textbook_cases():
    rng = np.random.default_rng(14)
    A = rng.normal(size=(40, 40)) + 10 * np.eye(40)
    b = rng.normal(size=40)
    res = solvers.fgmres(lambda v: A @ v, lambda v: v, b, rtol=1e-12, restart=15)
    assert res.converged and np.allclose(res.x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    # exact preconditioner -> one iteration
    Ai = np.linalg.inv(A)
    res = solvers.fgmres(lambda v: A @ v, lambda v: Ai @ v, b, rtol=1e-12)
    assert res.iters == 1


def test_vcycle_preconditioned_fgmres_reaches_direct_solution_c0():
    wl = W.make_workload("C0")
    ops = solvers.build_levels(wl.mesh, wl.disp, wl.c_mass, wl.eta)
    h = solvers.Hierarchy(ops)
    u, p = solvers.direct_solve(ops[-1], wl.g_u, wl.g_p)
    res = solvers.solve_stokes(h, wl.g_u, wl.g_p, rtol=1e-10)
    nv = ops[-1].box.n_vel
    assert res.converged and res.iters < 40
    assert np.linalg.norm(res.x[:nv] - u) <= 1e-8 * np.linalg.norm(u)
    # single-level hierarchy: the V-cycle is the exact coarse solve
    h0 = solvers.Hierarchy(ops[:1])
    fu, fp = solvers.direct_solve(ops[0], *[np.ones(ops[0].box.n_vel) * ~ops[0].dir_mask, np.ones(ops[0].box.n_p)])
    xu, xp = h0.precondition(np.ones(ops[0].box.n_vel) * ~ops[0].dir_mask, np.ones(ops[0].box.n_p))
    assert np.allclose(xu, fu, atol=1e-12) and np.allclose(xp, fp, atol=1e-10)


def _two_grid_by_error_propagation(h, f_u, f_p):
    """The two-grid cycle from a zero guess written as error propagation (Sec. 4: m
    smoothing steps x <- x + K_j(f - M x) before and after the coarse correction
    x <- x + P M_0^{-1} R (f - M x)).  With e = M^{-1} f - x every smoothing step maps
    e to e - K_j(M e) and the coarse correction maps e to e - P M_0^{-1} R M e, so the
    cycle returns M^{-1} f - S^m(C(S^m(M^{-1} f))).  M^{-1} f comes from a direct solve,
    M_0^{-1} from a dense solve; R zeroes the coarse wall entries, P the fine ones."""
    fine, coarse = h.levels[1], h.levels[0]
    M = fine.op.stokes().tocsc()
    nu = fine.op.box.n_vel
    ncu = coarse.op.box.n_vel
    M0 = coarse.op.stokes().toarray()
    xstar = sp.linalg.splu(M).solve(np.concatenate([f_u, f_p]))

    def smooth(e):
        r = M @ e
        y_u, y_p = h.smoother(1, r[:nu], r[nu:])
        return e - np.concatenate([y_u, y_p])

    def coarse_correction(e):
        r = M @ e
        cu = fine.P_u.T @ r[:nu]
        cu[coarse.op.dir_mask] = 0.0
        ec = np.linalg.solve(M0, np.concatenate([cu, fine.P_p.T @ r[nu:]]))
        pu = fine.P_u @ ec[:ncu]
        pu[fine.op.dir_mask] = 0.0
        return e - np.concatenate([pu, fine.P_p @ ec[ncu:]])

    e = xstar.copy()
    for _ in range(h.params.m):
        e = smooth(e)
    e = coarse_correction(e)
    for _ in range(h.params.m):
        e = smooth(e)
    x = xstar - e
    return x[:nu], x[nu:]


@pytest.mark.parametrize("name,levels,tol", [("C0", (1, 2), 1e-8), ("T3_4", (0, 1), 1e-10)])
def test_two_grid_vcycle_is_the_error_propagation_identity(name, levels, tol):
    """The oracle's V-cycle on two-level hierarchies equals the two-grid error
    propagation identity, which fixes the smoothing schedule (m pre- and m post-steps
    of the same K_j, the residual recomputed before each), the order of smoothing and
    coarse correction and the wall handling of the transfers.  The identity subtracts
    the propagated error from the direct solution, so it carries that solution's
    rounding times the conditioning of M (the 1e4 contrast of C0: about 4e-10); a
    schedule mistake changes the result by 0.1 or more."""
    wl = W.make_workload(name)
    ops = solvers.build_levels(wl.mesh, wl.disp, wl.c_mass, wl.eta)
    h = solvers.Hierarchy([ops[j] for j in levels])
    rng = np.random.default_rng(17)
    op = ops[levels[1]]
    f_u = rng.uniform(-1, 1, op.box.n_vel)
    f_p = rng.uniform(-1, 1, op.box.n_p)
    x_u, x_p = h.vcycle(1, f_u, f_p)
    r_u, r_p = _two_grid_by_error_propagation(h, f_u, f_p)
    eu = np.abs(x_u - r_u).max() / np.abs(r_u).max()
    ep = np.abs(x_p - r_p).max() / np.abs(r_p).max()
    assert eu <= tol and ep <= tol, (eu, ep)
    # the identity is not trivially satisfied: one V-cycle is far from the exact solve
    xs = sp.linalg.splu(op.stokes().tocsc()).solve(np.concatenate([f_u, f_p]))
    assert np.abs(x_u - xs[:op.box.n_vel]).max() > 1e3 * eu * np.abs(r_u).max()


def test_workload_generator_contract():
    a = W.make_workload("C0")
    b = W.make_workload("C0")
    assert np.array_equal(a.g_u, b.g_u) and np.array_equal(a.eta[2], b.eta[2])
    assert a.g_u.size == 2178 and a.g_p.size == 289
    dm = np.tile(W.dirichlet_node_mask(a.mesh, 2), 2)
    assert np.all(a.g_u[dm] == 0) and np.all(a.g_u[~dm] != 0)
    assert set(np.unique(a.eta[2])) == {1.0, 1e4}
    c1 = W.make_workload("C1", levels=[5])
    assert c1.g_u.size == 132354 and c1.g_p.size == 16705
    assert set(np.unique(c1.eta[5])) == {1e-3, 1e3}
    sizes = {n: (W.make_mesh(n).n_vel(W.make_mesh(n).n_levels - 1), W.make_mesh(n).n_p(W.make_mesh(n).n_levels - 1))
             for n in ("C2", "C3", "C4")}
    assert sizes == {"C2": (6440067, 274625), "C3": (50923779, 2146689), "C4": (21567171, 912673)}


# ---------------------------------------------------------------- extension solve (Sec. 2)
def _q2_node_displacement(mesh, disp):
    """Displacement of the multilinear ALE map at the Q2 nodes: vertex values at even
    node indices, averages of the two neighbours at odd ones (per direction)."""
    pn = mesh.p_nodes(mesh.n_levels - 1)
    a = disp.reshape((mesh.dim,) + tuple(pn[::-1]))
    for ax in range(1, mesh.dim + 1):
        n = a.shape[ax]
        shape = list(a.shape)
        shape[ax] = 2 * n - 1
        b = np.empty(shape)
        sl_even = [slice(None)] * a.ndim
        sl_even[ax] = slice(0, None, 2)
        b[tuple(sl_even)] = a
        lo = [slice(None)] * a.ndim
        hi = [slice(None)] * a.ndim
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        odd = [slice(None)] * a.ndim
        odd[ax] = slice(1, None, 2)
        b[tuple(odd)] = 0.5 * (a[tuple(lo)] + a[tuple(hi)])
        a = b
    return a.reshape(mesh.dim, -1)


def _extension_case(name, faces, constant_mu=None, boundary_field=None):
    from oracle import solvers
    wl = W.make_workload(name, dirichlet_faces=faces, levels=[])
    mesh = wl.mesh
    J = mesh.n_levels - 1
    ext = W.make_extension_inputs(name, mesh, levels=[J], constant_mu=constant_mu, boundary_field=boundary_field)
    box = fem.level_box(mesh, J)
    ref = fem.Reference(mesh.dim)
    Jq = fem.jacobians_q1(box, wl.disp, ref)
    u = solvers.extension_solve(box, Jq, ext.mu[J], ref, ext.g)
    return wl, box, ref, Jq, ext, u


@pytest.mark.parametrize("name,faces", [("T3_4", 63), ("T2_R", 15)])
def test_extension_reproduces_affine_fields_on_warped_mesh(name, faces):
    """Constant mu, every wall Dirichlet, boundary data of a physical affine field f(x) =
    Bx + c: f composed with the multilinear map lies in the mapped Q2 space and
    div(mu eps(f)) = 0, so the discrete extension is f itself at every node."""
    rng = np.random.default_rng(41)
    dim = 3 if name.startswith("T3") else 2
    Bm = rng.uniform(-0.02, 0.02, (dim, dim))
    c = rng.uniform(-0.01, 0.01, dim)
    holder = {}

    def field(X):
        mesh = holder["mesh"]
        x = X + _q2_node_displacement(mesh, holder["disp"])
        return Bm @ x + c[:, None]

    wl0 = W.make_workload(name, dirichlet_faces=faces, levels=[])
    holder["mesh"], holder["disp"] = wl0.mesh, wl0.disp
    wl, box, ref, Jq, ext, u = _extension_case(name, faces, constant_mu=3.7, boundary_field=field)
    want = field(W.velocity_node_coords(wl.mesh, wl.mesh.n_levels - 1)).ravel()
    assert np.abs(wl.disp).max() > 1e-3          # the mesh really is warped
    err = np.abs(u - want).max() / np.abs(want).max()
    assert err <= 1e-11, err


def test_extension_minimises_the_energy_with_variable_mu():
    """With the mu_A law and the default walls (do-nothing outflow face), the solution is
    the minimiser of (mu eps(u), eps(u))/2 over fields with the boundary data: the first
    variation along random interior perturbations vanishes and the energy grows."""
    from oracle import solvers
    wl, box, ref, Jq, ext, u = _extension_case("T3_R", None)
    J = wl.mesh.n_levels - 1
    mu = ext.mu[J]
    assert mu.max() > 10 and mu.min() < 1.01      # the law's peak lies inside the box
    E = lambda v: solvers.extension_energy(box, Jq, mu, ref, v)
    e0 = E(u)
    dm = box.dirichlet_vel_dofs()
    assert np.array_equal(u[dm], ext.g[dm])
    rng = np.random.default_rng(43)
    for _ in range(3):
        d = rng.uniform(-1, 1, u.size) * 1e-3
        d[dm] = 0.0
        ep, em = E(u + d), E(u - d)
        first = 0.5 * (ep - em)                   # a(u, d)
        second = 0.5 * (ep + em) - e0             # a(d, d) / 2
        assert second > 0
        assert abs(first) <= 1e-9 * np.sqrt(e0 * second), (first, e0, second)
    # the zero extension of the boundary data has more energy
    assert E(np.where(dm, ext.g, 0.0)) > e0


# ---------------------------------------------------------------- corrector-mode terms
def test_convection_matrices_closed_form():
    """One affine cell, constant v° in the x-y plane and constant r: the convection and
    streamline matrices are sums of Kronecker products of the 1D closed forms."""
    h = (0.5, 0.3, 0.7)
    rho, r = 1.7, 0.4
    ref = fem.Reference(3)
    box = fem.Box(3, (1, 1, 1), h, 0)
    J = fem.jacobians_q1(box, np.zeros((3, box.n_p)), ref)
    M = [M1(t) for t in h]
    K = [K1(t) for t in h]
    k3 = lambda a, b, c: np.kron(c, np.kron(b, a))       # x fastest
    n = 27
    for vx, vy in ((0.8, 0.0), (0.0, -0.6), (0.8, -0.5)):
        vconv = np.tile(np.array([vx, vy, 0.0]), (1, 27, 1))
        C = fem.convection_matrices(J, vconv, rho, np.full((1, 27), r), ref)[0]
        conv = rho * (vx * k3(C1.T, M[1], M[2]) + vy * k3(M[0], C1.T, M[2]))
        stab = r * (vx * vx * k3(K[0], M[1], M[2]) + vy * vy * k3(M[0], K[1], M[2])
                    + vx * vy * (k3(C1, C1.T, M[2]) + k3(C1.T, C1, M[2])))
        want = conv + stab
        for a in range(3):
            for b in range(3):
                blk = C[a * n:(a + 1) * n, b * n:(b + 1) * n]
                ref_blk = want if a == b else np.zeros_like(want)
                assert np.allclose(blk, ref_blk, rtol=0, atol=1e-14 * np.abs(want).max()), (vx, vy, a, b)


def test_convection_skew_and_streamline_psd_on_closed_box():
    """Constant (divergence-free) v° on an affinely mapped box with every wall Dirichlet:
    (v° . grad u, w) + (v° . grad w, u) is a boundary integral, so the interior block of
    the convection matrix is skew-symmetric; the streamline matrix is symmetric positive
    semi-definite."""
    box = fem.Box(3, (3, 2, 4), (1.2, 0.6, 1.0), 63)
    ref = fem.Reference(3)
    J = fem.jacobians_q1(box, np.zeros((3, box.n_p)), ref)
    v = np.array([0.3, -0.7, 0.5])
    vconv = np.tile(v, (box.n_cells, 27, 1))
    zero = np.zeros((box.n_cells, 27))
    I = np.nonzero(~box.dirichlet_vel_dofs())[0]
    N = fem.assemble_convection(box, J, vconv, 2.0, zero, ref)[I][:, I].toarray()
    assert np.abs(N).max() > 1e-3
    assert np.abs(N + N.T).max() <= 1e-13 * np.abs(N).max()
    S = fem.assemble_convection(box, J, vconv, 0.0, np.full_like(zero, 0.3), ref)[I][:, I].toarray()
    assert np.abs(S - S.T).max() <= 1e-13 * np.abs(S).max()
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() >= -1e-12 * np.abs(S).max()


# ---------------------------------------------------------------- BiCGStab Schur step
def test_bicgstab1_properties():
    """One BiCGStab step: the final residual is orthogonal to t = S P s (omega minimises
    ||s - omega t||), the half-step residual is orthogonal to the shadow residual r_0,
    the result does not depend on the scale of the Jacobi preconditioner, and an exact
    (scaled) preconditioner solves in the first half-step."""
    from oracle import solvers
    rng = np.random.default_rng(73)
    n = 12
    S = np.eye(n) * 4 + rng.uniform(-1, 1, (n, n))          # nonsymmetric, well conditioned
    d = rng.uniform(1, 3, n)
    r = rng.uniform(-1, 1, n)
    x, p, q, alpha, omega = solvers.bicgstab1(lambda z: S @ z, 1.0 / d, r)
    v = S @ p
    s_ = r - alpha * v
    assert abs(r @ s_) <= 1e-12 * np.linalg.norm(r) * np.linalg.norm(s_)
    t = S @ q
    res = r - S @ x
    assert np.allclose(res, s_ - omega * t, atol=1e-13)
    assert abs(t @ res) <= 1e-12 * np.linalg.norm(t) * np.linalg.norm(res)
    assert np.linalg.norm(res) < np.linalg.norm(r)
    x3 = solvers.bicgstab1(lambda z: S @ z, 3.0 / d, r)[0]
    assert np.allclose(x3, x, rtol=1e-12, atol=1e-14)
    c = 2.5
    xe = solvers.bicgstab1(lambda z: c * d * z, 1.0 / d, r)[0]
    assert np.allclose(xe, r / (c * d), rtol=1e-13)


def test_corrector_hierarchy_solves_the_nonsymmetric_system():
    """Corrector mode (A + N + S on every level, k_A = 6, BiCGStab Schur step) as the
    FGMRES preconditioner reaches the direct solution of the nonsymmetric system."""
    from oracle import solvers
    wl = W.make_workload("T3_4")
    conv = []
    for j in range(wl.mesh.n_levels):
        c = W.make_convection_inputs("T3_4", wl.mesh, j, wl.eta[j])
        conv.append((c.vconv, c.rho, c.r))
    ops = solvers.build_levels_corrector(wl.mesh, wl.disp, wl.c_mass, wl.eta, conv)
    A = ops[-1].A
    assert abs(A - A.T).max() > 1e-8 * abs(A).max()          # really nonsymmetric
    h = solvers.Hierarchy(ops, solvers.MGParams(k_A=6, schur="bicgstab"))
    res = solvers.solve_stokes(h, wl.g_u, wl.g_p, rtol=1e-10)
    u, p = solvers.direct_solve(ops[-1], wl.g_u, wl.g_p)
    nv = ops[-1].box.n_vel
    assert res.converged and res.iters < 40
    assert np.linalg.norm(res.x[:nv] - u) / np.linalg.norm(u) <= 1e-8


def test_absolute_scales_dominate_and_match_signed_diagonals():
    """The magnitude scales of the parity bounds (fem.element_matrices_abs) dominate the
    element matrices entry by entry (triangle inequality) and equal them where every
    integrand term is non-negative: the diagonal of A_K on an axis-aligned cell."""
    ref = fem.Reference(3)
    rng = np.random.default_rng(8)
    box = fem.Box(3, (2, 2, 2), (1.0, 0.9, 0.8), 0)
    J = fem.jacobians_q1(box, bubble_disp(box, 0.06, seed=9), ref)
    cm = rng.uniform(0, 3, (box.n_cells, 27))
    eta = 10 ** rng.uniform(-2, 2, (box.n_cells, 27))
    A, B = fem.element_matrices(J, cm, eta, ref)
    Aa, Ba = fem.element_matrices_abs(J, cm, eta, ref)
    assert (np.abs(A) <= Aa * (1 + 1e-14)).all() and (np.abs(B) <= Ba * (1 + 1e-14)).all()
    # strictly larger somewhere (cancelling quadrature terms), e.g. the divergence block
    assert (Ba > np.abs(B) * 1.5 + 1e-12).any()
    A1, _ = _single_cell(3, (0.5, 0.3, 0.7), 2.0, 0.9)
    box1 = fem.Box(3, (1, 1, 1), (0.5, 0.3, 0.7), 0)
    J1 = fem.jacobians_q1(box1, np.zeros((3, box1.n_p)), ref)
    Aa1, _ = fem.element_matrices_abs(J1, np.full((1, 27), 2.0), np.full((1, 27), 0.9), ref)
    assert np.allclose(np.diag(Aa1[0]), np.diag(A1), rtol=1e-14, atol=0)


@pytest.mark.slow
def test_oracle_iterations_bounded_with_levels_and_contrast():
    """The preconditioner of Sec. 4 with the interface aligned to the coarse grid: the
    oracle's FGMRES iteration count stays bounded as levels are added (C0 law, 16^2 to
    64^2) and as the inclusion contrast grows from 1 to 1e4."""
    its = []
    for name in ("C0", "C0_32", "C0_64"):
        wl = W.make_workload(name)
        h = solvers.Hierarchy(solvers.build_levels(wl.mesh, wl.disp, wl.c_mass, wl.eta))
        res = solvers.solve_stokes(h, wl.g_u, wl.g_p, rtol=1e-8, max_iter=100)
        assert res.converged
        its.append(res.iters)
    assert max(its) <= 1.5 * min(its), its
    byc = []
    for c in (1.0, 1e2, 1e4):
        wl = W.make_workload("C0_32", contrast=c)
        h = solvers.Hierarchy(solvers.build_levels(wl.mesh, wl.disp, wl.c_mass, wl.eta))
        res = solvers.solve_stokes(h, wl.g_u, wl.g_p, rtol=1e-8, max_iter=100)
        assert res.converged
        byc.append(res.iters)
    assert max(byc) <= 3 * byc[0], byc
