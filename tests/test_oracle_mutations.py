"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin fails.

Each mutation monkeypatches one oracle function with a wrong variant; the
listed pins must then raise.  This keeps the pins honest: a dropped term,
wrong sign, wrong index order or wrong scaling anywhere in the oracle is
caught by at least one of them.
"""
import numpy as np
import pytest

import tests.test_oracle_pins as pins
from oracle import basis, dense


def _wrong_sign_face_blocks(e0, g0, e1, g1, sigma):
    N = _ORIG_FACE(e0, g0, e1, g1, sigma)
    o = np.outer
    N["++"] = sigma * o(e0, e0) - 0.5 * (o(e0, g0) + o(g0, e0))
    return N


def _dropped_face_blocks(e0, g0, e1, g1, sigma):
    N = _ORIG_FACE(e0, g0, e1, g1, sigma)
    N["++"] = np.zeros_like(N["++"])
    return N


def _low_quadrature_mass_stiffness(p):
    nodes = basis.gll_nodes(p)
    xq, wq = basis.gauss_legendre(p)          # one point short of exact
    L = basis.lagrange_values(nodes, xq)
    D = basis.lagrange_derivatives(nodes, xq)
    return (L * wq[:, None]).T @ L, (D * wq[:, None]).T @ D


def _swapped_slot_operator(p, h, op=dense.NEUMANN, C=2.0):
    (Mx, Px), (My, Py), (Mz, Pz) = dense.direction_factors(p, h, op, C)
    # x-factor put in the last slot: transposed index order
    return (np.kron(np.kron(Mz, My), Px) + np.kron(np.kron(Mz, Py), Mx)
            + np.kron(np.kron(Pz, My), Mx))


def _dropped_term_operator(p, h, op=dense.NEUMANN, C=2.0):
    (Mx, Px), (My, Py), (Mz, Pz) = dense.direction_factors(p, h, op, C)
    return np.kron(np.kron(Px, My), Mz) + np.kron(np.kron(Mx, Py), Mz)


def _wrong_scaling_factors(p, h, op, C=2.0):
    M, Pm = dense.reference_pair(p, op, C)
    return [(float(hd) * M, Pm * float(hd)) for hd in h]


_ORIG_FACE = basis.face_blocks


def _run_all(fns):
    """True when at least one pin raises AssertionError."""
    for fn in fns:
        try:
            fn()
        except (AssertionError, np.linalg.LinAlgError):
            return True
    return False


PIN_SUITE = [
    lambda: pins.test_penalized_monomial_form(3, 2.0),
    lambda: pins.test_penalized_eigenvalues_p2_closed_form(),
    lambda: pins.test_face_blocks_reproduce_printed_hermite_stencil(),
    lambda: pins.test_p2_mass_stiffness_textbook(),
    lambda: pins.test_monomial_moments(3),
    lambda: pins.test_energy_of_interpolated_polynomial(3, (1, 2, 3)),
    lambda: pins.test_cell_block_energy_closed_form(3, (1, 2, 3), 2.0),
    lambda: pins.test_bruteforce_quadrature_assembly(2, dense.CELL),
    lambda: pins.test_neumann_block_properties(3),
    lambda: pins.test_isotropic_scaling(3),
]


@pytest.mark.parametrize("target,replacement", [
    ((basis, "face_blocks"), _wrong_sign_face_blocks),
    ((basis, "face_blocks"), _dropped_face_blocks),
    ((basis, "mass_stiffness"), _low_quadrature_mass_stiffness),
    ((dense, "dense_operator"), _swapped_slot_operator),
    ((dense, "dense_operator"), _dropped_term_operator),
    ((dense, "direction_factors"), _wrong_scaling_factors),
])
def test_planted_mistake_is_caught(monkeypatch, target, replacement):
    mod, name = target
    monkeypatch.setattr(mod, name, replacement)
    assert _run_all(PIN_SUITE), f"no pin caught the mutation of {mod.__name__}.{name}"


def test_unmutated_suite_passes():
    assert not _run_all(PIN_SUITE)


# ---------------------------------------------------------------- coupled SIPG operator
import tests.test_oracle_sipg as spins  # noqa: E402
from oracle import sipg  # noqa: E402

_ORIG_SIDE = sipg._side_data
_ORIG_FACE_MATRIX = sipg.face_matrix
_ORIG_CELL_INDEX = sipg.cell_index


def _half_boundary_average(p, hd, side, bname=sipg.LAGRANGE):
    t, d, j, a = _ORIG_SIDE(p, hd, side, bname)
    return t, d, j, 0.5                        # boundary average weighted like an interior one


def _flipped_coupling_penalty(p, hd, test_side, trial_side, C=2.0, bname=sipg.LAGRANGE):
    N = _ORIG_FACE_MATRIX(p, hd, test_side, trial_side, C, bname)
    if test_side != trial_side and "b" not in test_side:
        ti, _, ji, _ = _ORIG_SIDE(p, hd, test_side, bname)
        tj, _, jj, _ = _ORIG_SIDE(p, hd, trial_side, bname)
        sigma = basis.penalty_reference(p, C) / hd
        N = N - 2 * sigma * np.outer(ji * ti, jj * tj)
    return N


def _no_boundary_penalty(p, hd, test_side, trial_side, C=2.0, bname=sipg.LAGRANGE):
    if "b" in test_side:
        return _ORIG_FACE_MATRIX(p, hd, test_side, trial_side, 0.0, bname)
    return _ORIG_FACE_MATRIX(p, hd, test_side, trial_side, C, bname)


def _one_sided_symmetry_term(p, hd, test_side, trial_side, C=2.0, bname=sipg.LAGRANGE):
    ti, di, ji, ai = _ORIG_SIDE(p, hd, test_side, bname)
    tj, dj, jj, aj = _ORIG_SIDE(p, hd, trial_side, bname)
    sigma = basis.penalty_reference(p, C) / hd
    return -np.outer(ji * ti, aj * dj) + sigma * np.outer(ji * ti, jj * tj)   # [u]{d_n v} dropped


def _transposed_cell_index(m, cx, cy, cz):
    return (cx * m[2] + cz) * m[1] + cy         # y and z strides exchanged


def _tangential_mass_of_normal_length(p, h, d, N1, bname=sipg.LAGRANGE):
    M = sipg.ref_data(p, bname)[0]
    f = [h[d] * M for _ in range(3)]
    f[d] = N1
    return np.kron(np.kron(f[0], f[1]), f[2])


SIPG_PIN_SUITE = [
    lambda: spins.test_consistency_for_polynomials_vanishing_on_the_boundary(3, (3, 2, 4)),
    lambda: spins.test_consistency_with_boundary_data(3, (2, 3, 2)),
    lambda: spins.test_penalty_energy_of_piecewise_constants(3),
    lambda: spins.test_symmetric_positive_definite(2, (2, 3, 2)),
    lambda: spins.test_interior_diagonal_block_is_cell_block(2),
]


@pytest.mark.parametrize("target,replacement", [
    ((sipg, "_side_data"), _half_boundary_average),
    ((sipg, "face_matrix"), _flipped_coupling_penalty),
    ((sipg, "face_matrix"), _no_boundary_penalty),
    ((sipg, "face_matrix"), _one_sided_symmetry_term),
    ((sipg, "cell_index"), _transposed_cell_index),
    ((sipg, "_slot_kron"), _tangential_mass_of_normal_length),
])
def test_planted_sipg_mistake_is_caught(monkeypatch, target, replacement):
    mod, name = target
    monkeypatch.setattr(mod, name, replacement)
    assert _run_all(SIPG_PIN_SUITE), f"no pin caught the mutation of {mod.__name__}.{name}"


def test_unmutated_sipg_suite_passes():
    assert not _run_all(SIPG_PIN_SUITE)


# ---------------------------------------------------------------- multigrid
import tests.test_oracle_mg as mpins  # noqa: E402
from oracle import mg  # noqa: E402

_ORIG_P1D = mg.prolongation_1d
_ORIG_W = mg.chebyshev_weights


def _swapped_children(p, bname=sipg.LAGRANGE):
    P0, P1 = _ORIG_P1D(p, bname)
    return P1, P0


def _even_roots(a=mg.INTERVAL[0], b=mg.INTERVAL[1], degree=3):
    c, d = 0.5 * (a + b), 0.5 * (b - a)
    import math
    return [1.0 / (c - d * math.cos(2 * j * math.pi / (2 * degree))) for j in range(1, degree + 1)]


MG_PIN_SUITE = [
    lambda: mpins.test_chebyshev_weights_give_the_chebyshev_error_polynomial(),
    lambda: mpins.test_prolongation_embeds_polynomials(2),
    lambda: mpins.test_prolongation_preserves_the_mass(2),
]


@pytest.mark.parametrize("target,replacement", [
    ((mg, "prolongation_1d"), _swapped_children),
    ((mg, "chebyshev_weights"), _even_roots),
])
def test_planted_mg_mistake_is_caught(monkeypatch, target, replacement):
    mod, name = target
    monkeypatch.setattr(mod, name, replacement)
    assert _run_all(MG_PIN_SUITE), f"no pin caught the mutation of {mod.__name__}.{name}"


def test_unmutated_mg_suite_passes():
    assert not _run_all(MG_PIN_SUITE)


# ---------------------------------------------------------------- Hermite-type basis
import tests.test_oracle_hermite as hpins  # noqa: E402
from oracle import hermite  # noqa: E402

_ORIG_MONOMIALS = hermite.monomials
_ORIG_ENDPOINTS = hermite.endpoint_vectors


def _flipped_right_derivative(p):
    C = _ORIG_MONOMIALS(p).copy()
    C[:, p - 1] = -C[:, p - 1]                  # psi_{p-1}'(1) = -1 (outward instead of +x)
    return C


def _single_bubble(p):
    C = _ORIG_MONOMIALS(p).copy()
    if p >= 4:                                  # interior function x (1-x): nonzero end derivatives
        C[:, 2] = 0.0
        C[:3, 2] = [0.0, 1.0, -1.0]
    return C


def _uniform_nodes_transform(p):
    return hermite.values(p, np.linspace(0.0, 1.0, p + 1))


def _swapped_derivative_ends(p):
    e0, g0, e1, g1 = _ORIG_ENDPOINTS(p)
    return e0, g1, e1, g0


HERMITE_PIN_SUITE = [
    lambda: hpins.test_endpoint_conditions(4),
    lambda: hpins.test_mass_and_stiffness_two_routes(4),
    lambda: hpins.test_face_stencil_on_the_two_layers(3),
    lambda: hpins.test_assembled_operator_two_routes(3, (3, 2, 4), (0.3, 0.5, 0.25), sipg.FULL),
]


@pytest.mark.parametrize("target,replacement", [
    ((hermite, "monomials"), _flipped_right_derivative),
    ((hermite, "monomials"), _single_bubble),
    ((hermite, "transform"), _uniform_nodes_transform),
    ((hermite, "endpoint_vectors"), _swapped_derivative_ends),
])
def test_planted_hermite_mistake_is_caught(monkeypatch, target, replacement):
    mod, name = target
    monkeypatch.setattr(mod, name, replacement)
    assert _run_all(HERMITE_PIN_SUITE), f"no pin caught the mutation of {mod.__name__}.{name}"


def test_unmutated_hermite_suite_passes():
    assert not _run_all(HERMITE_PIN_SUITE)


# ---------------------------------------------------------------- vertex patches
import tests.test_oracle_patch as ppins  # noqa: E402
from oracle import patch  # noqa: E402

_ORIG_PATCH_FACTORS = patch.patch_factors


def _swapped_coupling_blocks(p, C=2.0):
    Mp, Kp, Ap = _ORIG_PATCH_FACTORS(p, C)
    n = p + 1
    Ap = Ap.copy()
    Ap[:n, n:], Ap[n:, :n] = Ap[n:, :n].copy(), Ap[:n, n:].copy()   # N^{+-} where N^{-+} belongs
    return Mp, Kp, Ap


def test_planted_patch_mistake_is_caught(monkeypatch):
    monkeypatch.setattr(patch, "patch_factors", _swapped_coupling_blocks)
    assert _run_all([lambda: ppins.test_patch_block_is_the_restricted_mesh_operator(2, dense.CELL, sipg.FULL)])


def test_unmutated_patch_suite_passes():
    assert not _run_all([lambda: ppins.test_patch_block_is_the_restricted_mesh_operator(2, dense.CELL, sipg.FULL)])
