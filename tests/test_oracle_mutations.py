"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each case monkeypatches one plausible slip into ``oracle.fem`` and re-runs the
pins that should catch it; the test passes only if at least one pin fails.
"""
import numpy as np
import pytest

from oracle import fem
import tests.test_oracle_pins as pins

_orig_elem = fem.element_matrices
_orig_geo = fem.geometry_factors


def _elem_cross_transposed(J, c_mass, eta, ref):
    A, B = _orig_elem(J, c_mass, eta, ref)
    dim = ref.dim
    nl = ref.phi.shape[1]
    nc = J.shape[0]
    Jinv, wdet = _orig_geo(J, ref)
    G = np.einsum("cqbx,qib->cqix", Jinv, ref.dphi)
    we = wdet * eta
    good = np.einsum("cq,cqib,cqja->caibj", we, G, G)
    bad = np.einsum("cq,cqia,cqjb->caibj", we, G, G)
    return (A.reshape(nc, dim, nl, dim, nl) - good + bad).reshape(A.shape), B


def _elem_dropped_mass(J, c_mass, eta, ref):
    return _orig_elem(J, 0 * c_mass, eta, ref)


def _geo_untransposed(J, ref):
    Jinv, wdet = _orig_geo(J, ref)
    return np.swapaxes(Jinv, -1, -2), wdet


def _elem_sign_flip_B(J, c_mass, eta, ref):
    A, B = _orig_elem(J, c_mass, eta, ref)
    return A, -B


CASES = {
    "cross term with swapped component indices": ("element_matrices", _elem_cross_transposed),
    "dropped mass term": ("element_matrices", _elem_dropped_mass),
    "J^{-1} used untransposed": ("geometry_factors", _geo_untransposed),
    "sign of the divergence": ("element_matrices", _elem_sign_flip_B),
}

PIN_SETS = [
    pins.test_element_matrices_2d_tensor_closed_form,
    pins.test_element_matrices_3d_tensor_closed_form,
    lambda: pins.test_rigid_motions_in_null_space(3),
    pins.test_quadratic_fields_energy_exact_on_warped_box,
    pins.test_mass_and_volume_on_warped_box,
    pins.test_divergence_of_linear_field,
]


@pytest.mark.parametrize("case", sorted(CASES))
def test_planted_mistake_is_caught(case, monkeypatch):
    attr, fn = CASES[case]
    monkeypatch.setattr(fem, attr, fn)
    caught = 0
    for pin in PIN_SETS:
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, case


# ---------------------------------------------------------------- extension solve
def _make_bad_extension(kind):
    import scipy.sparse.linalg as spla
    from oracle import solvers

    def bad(box, J, mu, ref, g):
        A = fem.assemble_unconstrained(box, J, np.zeros_like(mu), 0.5 * mu, ref).A.tocsr()
        dm = box.dirichlet_vel_dofs()
        I = np.nonzero(~dm)[0]
        W = np.nonzero(dm)[0]
        u = np.where(dm, g, 0.0)
        rhs = -(A[I][:, W] @ g[W])
        if kind == "sign":
            rhs = -rhs
        elif kind == "half":         # the boundary coupling counted once per pair of dofs, halved
            rhs = 0.5 * rhs
        u[I] = spla.splu(A[I][:, I].tocsc()).solve(rhs)
        return u
    return bad


@pytest.mark.parametrize("kind", ["sign", "half"])
def test_planted_extension_mistake_is_caught(kind, monkeypatch):
    from oracle import solvers
    monkeypatch.setattr(solvers, "extension_solve", _make_bad_extension(kind))
    caught = 0
    for pin in (lambda: pins.test_extension_reproduces_affine_fields_on_warped_mesh("T3_4", 63),
                pins.test_extension_minimises_the_energy_with_variable_mu):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, kind


# ---------------------------------------------------------------- corrector-mode terms
_orig_conv = fem.convection_matrices


def _conv_transposed(J, vconv, rho, r, ref):
    """the convection term with trial and test functions swapped"""
    C = _orig_conv(J, vconv, rho, 0.0 * r, ref)
    S = _orig_conv(J, vconv, 0.0, r, ref)
    return np.swapaxes(C, 1, 2) + S


def _conv_stab_dropped_cross(J, vconv, rho, r, ref):
    """the streamline term built from the squared components only"""
    C = _orig_conv(J, vconv, rho, 0.0 * r, ref)
    S = sum(_orig_conv(J, vconv * (np.arange(3) == d), 0.0, r, ref) for d in range(3))
    return C + S


@pytest.mark.parametrize("fn", [_conv_transposed, _conv_stab_dropped_cross])
def test_planted_convection_mistake_is_caught(fn, monkeypatch):
    monkeypatch.setattr(fem, "convection_matrices", fn)
    caught = 0
    for pin in (pins.test_convection_matrices_closed_form, pins.test_convection_skew_and_streamline_psd_on_closed_box):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, fn.__doc__


# ---------------------------------------------------------------- V-cycle composition
from oracle import solvers  # noqa: E402

_orig_vcycle = solvers.Hierarchy.vcycle


def _vcycle_no_post(self, j, f_u, f_p):
    """the post-smoothing steps left out"""
    if j == 0:
        return self.coarse_solve(f_u, f_p)
    op = self.levels[j].op
    x_u, x_p = np.zeros_like(f_u), np.zeros_like(f_p)
    for s in range(self.params.m):
        a_u, a_p = op.apply_stokes(x_u, x_p)
        y_u, y_p = self.smoother(j, f_u - a_u, f_p - a_p)
        x_u, x_p = x_u + y_u, x_p + y_p
    a_u, a_p = op.apply_stokes(x_u, x_p)
    c_u, c_p = self.restrict(j, f_u - a_u, f_p - a_p)
    e_u, e_p = _vcycle_no_post(self, j - 1, c_u, c_p)
    p_u, p_p = self.prolongate(j, e_u, e_p)
    return x_u + p_u, x_p + p_p


def _vcycle_one_step(self, j, f_u, f_p):
    """one pre- and one post-smoothing step where m = 2 are asked for"""
    m = self.params.m
    self.params.m = 1
    try:
        return _orig_vcycle(self, j, f_u, f_p)
    finally:
        self.params.m = m


def _vcycle_stale_residual(self, j, f_u, f_p):
    """the second pre-smoothing step applied to the first step's residual"""
    if j == 0:
        return self.coarse_solve(f_u, f_p)
    op = self.levels[j].op
    y_u, y_p = self.smoother(j, f_u, f_p)
    x_u, x_p = 2 * y_u, 2 * y_p
    a_u, a_p = op.apply_stokes(x_u, x_p)
    c_u, c_p = self.restrict(j, f_u - a_u, f_p - a_p)
    e_u, e_p = _vcycle_stale_residual(self, j - 1, c_u, c_p)
    p_u, p_p = self.prolongate(j, e_u, e_p)
    x_u, x_p = x_u + p_u, x_p + p_p
    for s in range(self.params.m):
        a_u, a_p = op.apply_stokes(x_u, x_p)
        y_u, y_p = self.smoother(j, f_u - a_u, f_p - a_p)
        x_u, x_p = x_u + y_u, x_p + y_p
    return x_u, x_p


_orig_smoother = solvers.Hierarchy.smoother


def _smoother_schur_sign(self, j, r_u, r_p):
    """the Schur right-hand side taken as r_p - B w instead of B w - r_p"""
    lv = self.levels[j]
    B = lv.op.B
    ainv = lambda r: self.cheb(j, r)
    sinv = lambda t: solvers.minres1(lambda z: B @ ainv(B.T @ z), lv.dS_inv, t)[0]
    w = ainv(r_u)
    y_p = sinv(r_p - B @ w)
    return w - ainv(B.T @ y_p), y_p


@pytest.mark.parametrize("attr,fn", [("vcycle", _vcycle_no_post), ("vcycle", _vcycle_one_step),
                                     ("vcycle", _vcycle_stale_residual), ("smoother", _smoother_schur_sign)])
def test_planted_vcycle_mistake_is_caught(attr, fn, monkeypatch):
    """The two-grid identity pin catches schedule mistakes in the V-cycle; the smoother's
    own mistake is caught by the V-cycle-preconditioned FGMRES pin (the identity takes the
    smoother as given)."""
    monkeypatch.setattr(solvers.Hierarchy, attr, fn)
    caught = 0
    for pin in (lambda: pins.test_two_grid_vcycle_is_the_error_propagation_identity("C0", (1, 2), 1e-8),
                lambda: pins.test_two_grid_vcycle_is_the_error_propagation_identity("T3_4", (0, 1), 1e-10),
                pins.test_vcycle_preconditioned_fgmres_reaches_direct_solution_c0):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, fn.__doc__


# ---------------------------------------------------------------- time step (Algorithm 1)
from oracle import gcsi  # noqa: E402
import tests.test_oracle_gcsi as gpins  # noqa: E402

_orig_rhs = gcsi.rhs
_orig_explicit = gcsi.explicit_displacement


def _with_state(fn):
    def rhs(box, ref, prm, mode, solid_q, disp, u_hash, state, absolute=False):
        return _orig_rhs(box, ref, prm, mode, solid_q, disp, u_hash, fn(state), absolute)
    return rhs


def _printed_stress_sign(st):
    """+2 eps(sum alpha u) in the explicit stress, as printed"""
    return gcsi.State(u=[-x for x in st.u], v=st.v, w=st.w, p=st.p)


def _printed_vcirc(st):
    """w^{n,1} in the second term of the predictor's extrapolation, as printed"""
    return gcsi.State(u=st.u, v=st.v, w=[st.w[0], st.w[0]], p=st.p)


def _mass_history_sign(st):
    """the BDF history of the velocity added instead of subtracted"""
    return gcsi.State(u=st.u, v=[-x for x in st.v], w=st.w, p=st.p)


def _explicit_last_only(prm, w, u_hist):
    """u^{n-k} in every term of the explicit step (the misprint of Algorithm 1)"""
    return _orig_explicit(prm, w, [u_hist[-1]] * len(u_hist))


GCSI_CASES = {
    "printed stress sign": ("rhs", _with_state(_printed_stress_sign)),
    "printed extrapolation": ("rhs", _with_state(_printed_vcirc)),
    "mass history sign": ("rhs", _with_state(_mass_history_sign)),
    "u^{n-k} in the explicit step": ("explicit_displacement", _explicit_last_only),
    "alpha_1 and alpha_2 swapped": ("BDF", {1: gcsi.BDF[1], 2: (2.0 / 3.0, (1.0 / 3.0, -4.0 / 3.0))}),
}

GCSI_PINS = [gpins.test_bdf_constants_exact_on_time_polynomials,
             gpins.test_rhs_body_and_mass_history_closed_form,
             gpins.test_rhs_predictor_convection_closed_form,
             gpins.test_rhs_solid_stress_closed_form,
             lambda: gpins.test_step_reproduces_a_uniformly_accelerated_free_solid(2)]


@pytest.mark.parametrize("case", sorted(GCSI_CASES))
def test_planted_time_step_mistake_is_caught(case, monkeypatch):
    attr, fn = GCSI_CASES[case]
    monkeypatch.setattr(gcsi, attr, fn)
    caught = 0
    for pin in GCSI_PINS:
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, case


_orig_lift = gcsi.lift_dirichlet


def _lift_no_pressure(box, ref, J, c_mass, eta, d, g_u, g_p, conv=None):
    """the constrained columns of B left out of the pressure right-hand side"""
    gu, _ = _orig_lift(box, ref, J, c_mass, eta, d, g_u, g_p, conv)
    return gu, g_p


def _lift_added(box, ref, J, c_mass, eta, d, g_u, g_p, conv=None):
    """the constrained columns added instead of subtracted"""
    gu, gp = _orig_lift(box, ref, J, c_mass, eta, -d, g_u, g_p, conv)
    dm = box.dirichlet_vel_dofs()
    gu[dm] = d[dm]
    return gu, gp


@pytest.mark.parametrize("fn", [_lift_no_pressure, _lift_added])
def test_planted_lifting_mistake_is_caught(fn, monkeypatch):
    monkeypatch.setattr(gcsi, "lift_dirichlet", fn)
    caught = 0
    for pin in (gpins.test_lifting_reproduces_uniform_flow_with_mass_and_convection,
                gpins.test_lifting_reproduces_a_linear_strain_field):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, fn.__doc__


def _run_no_shift(pb, state, n_steps, modes=("P", "C"), ref=None):
    """the oldest history entry kept instead of moved back"""
    outs = []
    for _ in range(n_steps):
        out = gcsi.step(pb, state, modes, ref)
        state = gcsi.State(u=[out["u"]] + state.u[1:], v=[out["v"]] + state.v[1:], w=[out["w"]] + state.w[1:],
                           p=out["p"])
        outs.append(out)
    return state, outs


def test_planted_history_shift_mistake_is_caught(monkeypatch):
    monkeypatch.setattr(gcsi, "run", _run_no_shift)
    with pytest.raises(AssertionError):
        gpins.test_run_shifts_the_history()
