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
