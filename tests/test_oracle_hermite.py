"""Pins of the Hermite-type basis oracle (oracle/hermite.py) and of the SIPG
system assembled in it, against what the paper fixes and the mathematics
implies: the endpoint conditions, the cubic Hermite polynomials, the trace
property, the two-layer sparsity of the face coupling, the printed 4x4 face
stencil, and two independent routes to every matrix (quadrature of the new
basis vs the Lagrange matrices transformed by the change of basis)."""
import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

from oracle import basis, hermite, mg, sipg

PS = [3, 4, 5, 6, 7, 8]


@pytest.mark.parametrize("p", PS)
def test_endpoint_conditions(p):
    """eq. (hermite_conditions): psi_0 = value at 0, psi_1 = derivative at 0,
    psi_{p-1} = derivative at 1, psi_p = value at 1; all other endpoint data
    (interior functions included) vanish."""
    e0, g0, e1, g1 = hermite.endpoint_vectors(p)
    I = np.eye(p + 1)
    for got, want in ((e0, I[0]), (g0, I[1]), (g1, I[p - 1]), (e1, I[p])):
        assert np.allclose(got, want, atol=1e-11)


def test_cubic_hermite_closed_forms():
    """p = 3: the four functions are the textbook cubic Hermite polynomials."""
    x = np.random.default_rng(0).uniform(0, 1, 50)
    V = hermite.values(3, x)
    want = np.stack([2 * x**3 - 3 * x**2 + 1, x**3 - 2 * x**2 + x, x**3 - x**2, -2 * x**3 + 3 * x**2], axis=1)
    assert np.allclose(V, want, atol=1e-14)


@pytest.mark.parametrize("p", PS)
def test_traces_are_coefficients(p):
    """eq. (hermite_traces_1d) on random expansions, evaluated at the ends."""
    u = np.random.default_rng(p).standard_normal(p + 1)
    v0, v1 = hermite.values(p, [0.0, 1.0]) @ u
    d0, d1 = hermite.derivatives(p, [0.0, 1.0]) @ u
    assert np.allclose([v0, d0, d1, v1], [u[0], u[1], u[p - 1], u[p]], atol=1e-11 * np.abs(u).max())


@pytest.mark.parametrize("p", PS)
def test_basis_spans_P_p_and_interior_functions_are_bubbles(p):
    """The change of basis is invertible (the functions span P_p), and the
    interior functions are divisible by x^2 (1-x)^2 (double roots at both
    ends)."""
    T = hermite.transform(p)
    assert np.linalg.cond(T) < 1e4
    C = hermite.monomials(p)
    for j in range(2, p - 1):
        q, r = np.polynomial.polynomial.polydiv(C[:, j], [0.0, 0.0, 1.0, -2.0, 1.0])
        assert np.allclose(r, 0.0, atol=1e-12)


@pytest.mark.parametrize("p", PS)
def test_mass_and_stiffness_two_routes(p):
    """M and K by quadrature of the Hermite functions equal the Lagrange
    matrices transformed by the change of basis (T^T M_L T): the nodal values
    of psi_j are exactly its Lagrange coefficients."""
    T = hermite.transform(p)
    M, K = hermite.mass_stiffness(p)
    ML, KL = basis.mass_stiffness(p)
    assert np.allclose(M, T.T @ ML @ T, atol=1e-13 * np.abs(M).max())
    assert np.allclose(K, T.T @ KL @ T, atol=1e-12 * np.abs(K).max())


@pytest.mark.parametrize("p", [3, 4, 5])
def test_cell_block_eigenvalues_are_basis_independent(p):
    """The generalized eigenvalues of (A_hat, M_hat) do not depend on the
    basis (the same operator on the same space)."""
    M, _ = hermite.mass_stiffness(p)
    A = hermite.penalized_stiffness(p)
    ML, _ = basis.mass_stiffness(p)
    AL = basis.penalized_stiffness(p)
    lh = sl.eigh(A, M, eigvals_only=True)
    ll = sl.eigh(AL, ML, eigvals_only=True)
    assert np.allclose(lh, ll, rtol=1e-9)


@pytest.mark.parametrize("p", [3, 4, 5, 6])
def test_face_stencil_on_the_two_layers(p):
    """With the basis' own endpoint data, the four coupling blocks reduce to
    the printed stencil eq. (hermite_face_stencil) on (a-, b-, a+, b+) =
    (layer p and p-1 of K-, layer 0 and 1 of K+), beta = 1/(2h), and vanish
    elsewhere."""
    h, C = 0.3, 2.0
    e0, g0, e1, g1 = hermite.endpoint_vectors(p)
    sigma = basis.penalty_reference(p, C) / h
    N = basis.face_blocks(e0, g0 / h, e1, g1 / h, sigma)
    beta = 1.0 / (2 * h)
    stencil = np.array([[sigma, -beta, -sigma, -beta],
                        [-beta, 0, beta, 0],
                        [-sigma, beta, sigma, beta],
                        [-beta, 0, beta, 0]])
    minus, plus = [p, p - 1], [0, 1]
    got = np.zeros((4, 4))
    got[:2, :2] = N["--"][np.ix_(minus, minus)]
    got[:2, 2:] = N["-+"][np.ix_(minus, plus)]
    got[2:, :2] = N["+-"][np.ix_(plus, minus)]
    got[2:, 2:] = N["++"][np.ix_(plus, plus)]
    assert np.allclose(got, stencil, atol=1e-9 * sigma)
    for key, rows, cols in (("--", minus, minus), ("-+", minus, plus), ("+-", plus, minus), ("++", plus, plus)):
        rest = N[key].copy()
        rest[np.ix_(rows, cols)] = 0.0
        assert np.abs(rest).max() < 1e-9 * sigma


def _cell_transform(p, ncell):
    T = hermite.transform(p)
    return sp.block_diag([np.kron(np.kron(T, T), T)] * ncell, format="csr")


@pytest.mark.parametrize("p,m,h", [(3, (3, 2, 4), (0.3, 0.5, 0.25)), (4, (2, 3, 2), (0.5, 0.2, 0.4)),
                                   (5, (2, 2, 2), (0.5, 0.5, 0.5))])
@pytest.mark.parametrize("part", [sipg.FULL, sipg.FACE, sipg.VOLUME])
def test_assembled_operator_two_routes(p, m, h, part):
    """The operator assembled from the Hermite 1D data (masses, stiffness and
    endpoint vectors of the new basis in the face matrices) equals the
    Lagrange operator transformed cell by cell, Tb^T A_L Tb: the same
    bilinear form on the same space."""
    ncell = m[0] * m[1] * m[2]
    AH = sipg.assemble(p, m, h, part, bname=sipg.HERMITE)
    AL = sipg.assemble(p, m, h, part)
    Tb = _cell_transform(p, ncell)
    ref = (Tb.T @ AL @ Tb).toarray()
    assert np.abs(AH.toarray() - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("p", [3, 5])
def test_coupling_blocks_touch_two_layers(p):
    """eq. (hermite_traces_3d): the block of cell c's row for a neighbour
    across a face normal to axis d is nonzero only in c's two layers next to
    that face and the neighbour's two layers next to it."""
    m, h = (3, 3, 3), (0.4, 0.3, 0.5)
    n = p + 1
    c = sipg.cell_index(m, 1, 1, 1)
    cc = sipg.cell_coords(m, c)
    blocks = sipg.cell_row_blocks(p, m, h, c, bname=sipg.HERMITE)
    assert len(blocks) == 7
    idx = np.array(np.unravel_index(np.arange(n ** 3), (n, n, n)))   # (axis, q) -> layer along axis
    for nb, blk in blocks[1:]:
        d = [a for a in range(3) if sipg.cell_coords(m, nb)[a] != cc[a]][0]
        up = sipg.cell_coords(m, nb)[d] > cc[d]
        rows_ok = np.isin(idx[d], [p - 1, p] if up else [0, 1])
        cols_ok = np.isin(idx[d], [0, 1] if up else [p - 1, p])
        scale = np.abs(blk).max()
        assert np.abs(blk[~rows_ok, :]).max() <= 1e-12 * scale
        assert np.abs(blk[:, ~cols_ok]).max() <= 1e-12 * scale


@pytest.mark.parametrize("p", [3, 4])
def test_transforms_are_inverse_and_exact_on_polynomials(p):
    """to_lagrange(to_hermite(u)) = u; the Hermite coefficients of a
    polynomial of Q_p reproduce it at random points (through the basis'
    monomials, not the nodal route)."""
    rng = np.random.default_rng(3)
    n = p + 1
    u = rng.standard_normal(2 * n ** 3)
    assert np.allclose(hermite.to_lagrange(p, hermite.to_hermite(p, u, 2), 2), u, atol=1e-12)
    cx, cy, cz = rng.standard_normal((3, n))
    q = lambda X, Y, Z: np.polyval(cx, X) * np.polyval(cy, Y) * np.polyval(cz, Z)   # noqa: E731
    x = basis.gll_nodes(p)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    uh = hermite.to_hermite(p, q(X, Y, Z).reshape(-1), 1).reshape(n, n, n)
    pts = rng.uniform(0, 1, (3, 20))
    V = [hermite.values(p, pts[a]) for a in range(3)]
    got = np.einsum("qi,qj,qk,ijk->q", V[0], V[1], V[2], uh)
    assert np.allclose(got, q(*pts), atol=1e-11 * np.abs(uh).max())


@pytest.mark.parametrize("p", [3, 4])
def test_prolongation_embeds_and_preserves_mass(p):
    """The Hermite prolongation gives each child the coefficients of the
    parent's polynomial, and P^T M_fine P = M_coarse."""
    P0, P1 = hermite.prolongation_1d(p)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(p + 1)
    x = rng.uniform(0, 1, 15)
    for c, Pc in ((0, P0), (1, P1)):
        child = hermite.values(p, x) @ (Pc @ u)
        parent = hermite.values(p, (x + c) / 2) @ u
        assert np.allclose(child, parent, atol=1e-12 * np.abs(u).max() * 10)
    mc = 1
    Pm = mg.prolongation(p, mc, sipg.HERMITE)
    Mf = sipg.mass(p, (2,) * 3, (0.5,) * 3, sipg.HERMITE)
    Mc = sipg.mass(p, (1,) * 3, (1.0,) * 3, sipg.HERMITE)
    assert np.abs((Pm.T @ Mf @ Pm - Mc).toarray()).max() <= 1e-13 * np.abs(Mc.toarray()).max()


def test_mg_pcg_in_the_hermite_basis():
    """The same V-cycle in the new basis is the Lagrange one conjugated by
    the change of basis: MG-PCG converges in the same few iterations."""
    p, m = 3, 4
    A = sipg.assemble(p, (m,) * 3, (1.0 / m,) * 3, bname=sipg.HERMITE)
    b = np.random.default_rng(2).uniform(-1, 1, A.shape[0])
    x, it, rel = mg.mg_pcg(p, m, b, 1e-10, bname=sipg.HERMITE)
    _, it_l, _ = mg.mg_pcg(p, m, hermite.to_lagrange(p, b, m ** 3), 1e-10)
    assert rel <= 1e-10 and np.linalg.norm(b - A @ x) <= 2e-10 * np.linalg.norm(b)
    assert it <= 16 and abs(it - it_l) <= 3


def test_preconditioned_criterion_is_basis_invariant():
    """Sec. 6.1's stopping rule on <r, z>^{1/2}: CG with the V-cycle on the
    same problem written in the two bases (b_H = T3^T b_L) takes the same
    number of iterations, and the iterates are related by the change of
    basis (x_L = T3 x_H), because <r, z> is a pairing of a dual and a primal
    vector.  (The 2-norm of the residual is not invariant.)"""
    p, m = 3, 4
    ncell = m ** 3
    bL = np.random.default_rng(1).uniform(-1, 1, ncell * 64)
    T = hermite.transform(p)
    bH = (bL.reshape(ncell, -1) @ np.kron(np.kron(T, T), T)).reshape(-1)
    xL, itL, _ = mg.mg_pcg(p, m, bL, 1e-10, criterion="preconditioned")
    xH, itH, _ = mg.mg_pcg(p, m, bH, 1e-10, bname=sipg.HERMITE, criterion="preconditioned")
    assert itL == itH
    assert np.allclose(hermite.to_lagrange(p, xH, ncell), xL, atol=1e-9 * np.abs(xL).max())
