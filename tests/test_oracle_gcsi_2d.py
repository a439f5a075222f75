"""Pins of the time-step oracle (oracle/gcsi.py) in 2D, independent of its own code: the
terms of eq. form_g_j / eq. form_g_p on affine geometry (closed forms over the image of a
rectangle), and whole GCSI steps whose exact solutions the scheme reproduces (a free solid
uniformly accelerated by a body force; a fluid at rest under gravity with the hydrostatic
pressure).  The 2D determinant, adjugate and index orders are the parts a 3D pin cannot
reach.
"""
import math

import numpy as np
import pytest

from oracle import fem, gcsi

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")

REF = fem.Reference(2)
EXT = (1.0, 0.5)
CELLS = (4, 2)


def _box(faces=0):
    return fem.Box(2, CELLS, EXT, faces)


def _solid_cells(box, xr=(1, 3)):
    ci = box.cell_index_grid()
    return (ci[0] >= xr[0]) & (ci[0] < xr[1])


def _nodal(box, f):
    return np.ascontiguousarray(f(box.vel_node_ref_coords()).ravel())


def _prm(**kw):
    base = dict(k=2, tau=0.01, rho_f=2.0, rho_s=5.0, eta_f=0.3, mu_s=7.0, eta_V=0.1, body=(0.0, 0.0, 0.0))
    base.update(kw)
    return gcsi.Params(**base)


def _zero_state(box, k=2):
    z = np.zeros(box.n_vel)
    return gcsi.State(u=[z] * k, v=[z] * k, w=[z] * k)


def _area_moment(box, cells, D):
    """Area and first moment of the image (I + D) of the given cells."""
    h = box.h()
    ci = box.cell_index_grid()
    dj = np.linalg.det(np.eye(2) + D)
    area = np.prod(h) * np.count_nonzero(cells) * dj
    cen = np.stack([(ci[d][cells] + 0.5) * h[d] for d in range(2)])
    mom = (np.eye(2) + D) @ cen.sum(axis=1) * np.prod(h) * dj
    return area, mom


def test_rhs_body_and_mass_history_closed_form_2d():
    box = _box()
    D = np.array([[0.05, 0.02], [-0.03, 0.04]])
    prm = _prm(body=(0.3, -1.1, 99.0))           # the third component is not read in 2D
    sc = _solid_cells(box)
    sq = np.repeat(sc[:, None], 9, 1)
    c1, c2 = np.array([0.4, -0.2]), np.array([-0.6, 0.5])
    st = _zero_state(box)
    st.v = [_nodal(box, lambda X: np.tile(c1[:, None], X.shape[1])),
            _nodal(box, lambda X: np.tile(c2[:, None], X.shape[1]))]
    g_u, g_p = gcsi.rhs(box, REF, prm, "C", sq, D @ box.vertex_coords(), np.zeros(box.n_vel), st)
    F = np.asarray(prm.body[:2]) - (prm.alpha[0] * c1 + prm.alpha[1] * c2) / (prm.gamma * prm.tau)
    a_s, m_s = _area_moment(box, sc, D)
    a_f, m_f = _area_moment(box, ~sc, D)
    G = g_u.reshape(2, -1)
    assert np.allclose(G.sum(axis=1), (prm.rho_s * a_s + prm.rho_f * a_f) * F, rtol=1e-12)
    x = (np.eye(2) + D) @ box.vel_node_ref_coords()
    assert np.allclose(G @ x.T, np.outer(F, prm.rho_s * m_s + prm.rho_f * m_f), rtol=1e-12, atol=1e-14)
    assert not np.any(g_p)


def test_rhs_predictor_convection_closed_form_2d():
    box = _box()
    D = np.array([[0.04, -0.02], [0.01, 0.03]])
    prm = _prm()
    Gv = np.array([[0.3, -0.2], [0.1, 0.4]])
    b0 = np.array([0.2, -0.1])
    cc = np.array([0.7, -0.4])
    L = lambda X: Gv @ ((np.eye(2) + D) @ X) + b0[:, None]
    st = _zero_state(box)
    Ln = _nodal(box, L)
    cn = _nodal(box, lambda X: np.tile(cc[:, None], X.shape[1]))
    st.v = [Ln, Ln]
    st.w = [0.5 * (Ln - cn), np.zeros(box.n_vel)]          # v° = c, v* = L
    sq = np.zeros((box.n_cells, 9), dtype=bool)
    g_u, _ = gcsi.rhs(box, REF, prm, "P", sq, D @ box.vertex_coords(), np.zeros(box.n_vel), st)
    area, mom = _area_moment(box, np.ones(box.n_cells, dtype=bool), D)
    want = prm.rho_f / (prm.gamma * prm.tau) * (Gv @ mom + b0 * area) - prm.rho_f * (Gv @ cc) * area
    assert np.allclose(g_u.reshape(2, -1).sum(axis=1), want, rtol=1e-12)


def test_rhs_solid_stress_closed_form_2d():
    box = _box()
    D = np.array([[0.03, 0.05], [-0.01, 0.02]])
    prm = _prm()
    rng = np.random.default_rng(5)
    U1, U2, Uh = (0.05 * rng.normal(size=(2, 2)) for _ in range(3))
    st = _zero_state(box)
    st.u = [_nodal(box, lambda X: U1 @ X), _nodal(box, lambda X: U2 @ X)]
    uh = _nodal(box, lambda X: Uh @ X)
    sc = _solid_cells(box)
    sq = np.repeat(sc[:, None], 9, 1)
    g_u, _ = gcsi.rhs(box, REF, prm, "C", sq, D @ box.vertex_coords(), uh, st)
    Fi = np.linalg.inv(np.eye(2) + D)
    Gs = (prm.alpha[0] * U1 + prm.alpha[1] * U2) @ Fi
    Gh = Uh @ Fi
    T = prm.mu_s * (Gs + Gs.T + Gh.T @ Gh)
    a_s, _ = _area_moment(box, sc, D)
    G = g_u.reshape(2, -1)
    assert np.allclose(G.sum(axis=1), 0.0, atol=1e-12 * prm.mu_s)
    Bm = np.array([[0.3, -0.7], [0.5, 0.1]])
    phi = Bm @ ((np.eye(2) + D) @ box.vel_node_ref_coords())
    assert np.isclose(np.sum(G * phi), a_s * np.sum(T * Bm), rtol=1e-12)


def test_volume_correction_closed_forms_2d():
    box = _box()
    prm = _prm()
    sc = _solid_cells(box)
    sq = np.repeat(sc[:, None], 9, 1)
    h = box.h()
    x0, x1 = 1 * h[0], 3 * h[0]
    U = np.array([[0.1, 0.02], [-0.03, 0.05]])
    gp = gcsi.volume_correction(box, REF, prm, sq, _nodal(box, lambda X: U @ X))
    want = -((1 + U[0, 0]) * (1 + U[1, 1]) - U[0, 1] * U[1, 0] - 1.0) / prm.eta_V * (x1 - x0) * EXT[1]
    assert np.isclose(gp.sum(), want, rtol=1e-12)
    a = 0.2
    uq = _nodal(box, lambda X: np.stack([a * X[0] ** 2, 0 * X[0]]))
    gp = gcsi.volume_correction(box, REF, prm, sq, uq)
    Xp = box.vertex_coords()[0]
    assert np.isclose(gp.sum(), -(a / prm.eta_V) * (x1 ** 2 - x0 ** 2) * EXT[1], rtol=1e-12)
    assert np.isclose(gp @ Xp, -(2 * a / prm.eta_V) * (x1 ** 3 - x0 ** 3) / 3 * EXT[1], rtol=1e-12)
    us = _nodal(box, lambda X: np.stack([0.3 * X[1], 0 * X[0]]))
    assert np.abs(gcsi.volume_correction(box, REF, prm, sq, us)).max() < 1e-15
    assert not np.any(gcsi.volume_correction(box, REF, _prm(eta_V=math.inf), sq, uq))


@pytest.mark.parametrize("k", [1, 2])
def test_step_reproduces_a_uniformly_accelerated_free_solid_2d(k):
    b = np.array([0.4, -2.0]) if k == 2 else np.zeros(2)
    prm = _prm(k=k, body=(b[0], b[1], 0.0), tau=0.02)
    box = _box()
    pb = gcsi.Problem(box=box, ext_box=_box(faces=15), solid_q=np.ones((box.n_cells, 9), dtype=bool),
                      solid_cells=np.ones(box.n_cells, dtype=bool), mu_A=np.ones((box.n_cells, 9)), prm=prm)
    V0 = np.array([0.5, -0.75])
    tn = 0.3
    vel = lambda t: V0 + b * t
    disp = lambda t: V0 * t + 0.5 * b * t * t
    const = lambda c: _nodal(box, lambda X: np.tile(c[:, None], X.shape[1]))
    ts = [tn - (i + 1) * prm.tau for i in range(k)]
    st = gcsi.State(u=[const(disp(t)) for t in ts], v=[const(vel(t)) for t in ts], w=[const(vel(t)) for t in ts])
    out = gcsi.step(pb, st, ("P", "C"), REF)
    for key, want in (("v", vel(tn)), ("w", vel(tn)), ("u", disp(tn))):
        assert np.allclose(out[key], const(want), rtol=0, atol=1e-11), key
    assert np.abs(out["p"]).max() < 1e-9


def test_step_keeps_a_fluid_at_rest_with_the_hydrostatic_pressure_2d():
    """Walls but the outflow x = L, body force along x: v = 0 and p = rho b (L - x)."""
    box = fem.Box(2, CELLS, EXT, 0b1101)
    bx = 3.0
    prm = _prm(body=(bx, 0.0, 0.0))
    sq = np.zeros((box.n_cells, 9), dtype=bool)
    pb = gcsi.Problem(box=box, ext_box=_box(faces=15), solid_q=sq, solid_cells=np.zeros(box.n_cells, dtype=bool),
                      mu_A=np.ones((box.n_cells, 9)), prm=prm)
    out = gcsi.step(pb, _zero_state(box), ("P", "C"), REF)
    X = box.vertex_coords()[0]
    p_want = prm.rho_f * bx * (EXT[0] - X)
    assert np.abs(out["v"]).max() < 1e-10 * np.abs(p_want).max()
    assert np.allclose(out["p"], p_want, rtol=1e-10, atol=1e-10)
    assert not np.any(out["w"]) and not np.any(out["u"])
