"""Pins of the FP64 oracle against facts the paper and mathematics fix.

None of these re-types the oracle's own formulas: each compares it with a
closed form, a textbook value, the stencil printed in the paper, or an
independent brute-force quadrature assembly built from numpy polynomials.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import basis, dense

P = np.polynomial.polynomial


# ---------------------------------------------------------------- nodes
def test_gll_nodes_closed_forms():
    assert np.allclose(basis.gll_nodes(1), [0, 1], atol=0)
    assert np.allclose(basis.gll_nodes(2), [0, 0.5, 1], atol=1e-16)
    r5 = 1 / math.sqrt(5)
    assert np.allclose(basis.gll_nodes(3), [0, (1 - r5) / 2, (1 + r5) / 2, 1], atol=2e-16)
    r37 = math.sqrt(3 / 7)
    assert np.allclose(basis.gll_nodes(4), [0, (1 - r37) / 2, 0.5, (1 + r37) / 2, 1], atol=2e-16)
    # p=5: interior roots of P5' are +-sqrt(1/3 -+ 2 sqrt(7)/21)
    a = math.sqrt(1 / 3 - 2 * math.sqrt(7) / 21)
    b = math.sqrt(1 / 3 + 2 * math.sqrt(7) / 21)
    ref = [0, (1 - b) / 2, (1 - a) / 2, (1 + a) / 2, (1 + b) / 2, 1]
    assert np.allclose(basis.gll_nodes(5), ref, atol=2e-16)


@pytest.mark.parametrize("p", range(1, 9))
def test_gll_nodes_are_lobatto_rule(p):
    """The (p+1)-point Lobatto rule with weights 2/(p(p+1) P_p(xi)^2) on [-1,1]
    integrates x^k exactly for k <= 2p-1."""
    x = basis.gll_nodes(p)
    xi = 2 * x - 1
    Pp = np.polynomial.legendre.Legendre.basis(p)(xi)
    w = 2.0 / (p * (p + 1) * Pp ** 2) / 2.0  # mapped to [0,1]
    for k in range(2 * p):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-14


# ---------------------------------------------------------------- M, K
def test_p2_mass_stiffness_textbook():
    M, K = basis.mass_stiffness(2)
    M_ref = np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30.0
    K_ref = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3.0
    assert np.allclose(M, M_ref, rtol=0, atol=1e-15)
    assert np.allclose(K, K_ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("p", range(1, 9))
def test_monomial_moments(p):
    """V^T M V and V^T K V with V_ia = x_i^a are the exact integrals of
    x^a x^b and (x^a)'(x^b)' on [0,1]."""
    x = basis.gll_nodes(p)
    M, K = basis.mass_stiffness(p)
    V = np.vander(x, p + 1, increasing=True)
    a = np.arange(p + 1)[:, None]
    b = np.arange(p + 1)[None, :]
    Mref = 1.0 / (a + b + 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        Kref = np.where((a == 0) | (b == 0), 0.0, a * b / np.maximum(a + b - 1, 1))
    tol = 1e-13 * 10 ** max(0, p - 4)
    assert np.max(np.abs(V.T @ M @ V - Mref)) < tol
    assert np.max(np.abs(V.T @ K @ V - Kref)) < tol * 10


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("C", [1.0, 2.0])
def test_penalized_monomial_form(p, C):
    """A_hat evaluated on monomials equals the 1D SIPG cell form written out:
    int u'v' + s(u(1)v(1) + u(0)v(0)) - 1/2(u'(1)v(1) + u(1)v'(1))
                                      + 1/2(u'(0)v(0) + u(0)v'(0)),  s = C p(p+1)."""
    x = basis.gll_nodes(p)
    A = basis.penalized_stiffness(p, C)
    V = np.vander(x, p + 1, increasing=True)
    s = C * p * (p + 1)
    n = p + 1
    ref = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            vol = a * b / (a + b - 1) if a > 0 and b > 0 else 0.0
            u1, du1, u0, du0 = 1.0, a, float(a == 0), float(a == 1)
            v1, dv1, v0, dv0 = 1.0, b, float(b == 0), float(b == 1)
            ref[a, b] = (vol + s * (u1 * v1 + u0 * v0)
                         - 0.5 * (du1 * v1 + u1 * dv1) + 0.5 * (du0 * v0 + u0 * dv0))
    tol = 1e-12 * 10 ** max(0, p - 4)
    assert np.max(np.abs(V.T @ A @ V - ref)) < tol * max(1, s)


def test_face_blocks_reproduce_printed_hermite_stencil():
    """In the cubic Hermite basis (p=3) the face blocks collapse to the 4x4
    stencil printed in eq. (hermite_face_stencil) on (a-, b-, a+, b+), with
    beta = 1/(2h).  Endpoint data of that basis: value at 0 is coefficient 0,
    derivative at 0 is coefficient 1, derivative at 1 coefficient 2, value at
    1 coefficient 3 (eq. (hermite_conditions))."""
    h, sigma = 0.37, 11.0
    e0 = np.array([1.0, 0, 0, 0])
    g0 = np.array([0, 1.0, 0, 0]) / h
    g1 = np.array([0, 0, 1.0, 0]) / h
    e1 = np.array([0, 0, 0, 1.0])
    N = basis.face_blocks(e0, g0, e1, g1, sigma)
    beta = 1.0 / (2 * h)
    stencil = np.array([[sigma, -beta, -sigma, -beta],
                        [-beta, 0, beta, 0],
                        [-sigma, beta, sigma, beta],
                        [-beta, 0, beta, 0]])
    # rows/cols: a- = layer p of K-, b- = layer p-1 of K-, a+ = layer 0, b+ = layer 1
    minus = [3, 2]
    plus = [0, 1]
    got = np.zeros((4, 4))
    got[:2, :2] = N["--"][np.ix_(minus, minus)]
    got[:2, 2:] = N["-+"][np.ix_(minus, plus)]
    got[2:, :2] = N["+-"][np.ix_(plus, minus)]
    got[2:, 2:] = N["++"][np.ix_(plus, plus)]
    assert np.allclose(got, stencil, atol=1e-14)
    # everything outside the two face layers vanishes
    assert np.count_nonzero(N["--"]) == np.count_nonzero(N["--"][np.ix_(minus, minus)])


# ---------------------------------------------------------------- eigenvalues
def test_neumann_eigenvalues_closed_forms():
    M, K = basis.mass_stiffness(2)
    assert np.allclose(sl.eigh(K, M, eigvals_only=True), [0, 12, 60], atol=1e-12)
    M, K = basis.mass_stiffness(3)
    r = math.sqrt(6420)
    assert np.allclose(sl.eigh(K, M, eigvals_only=True), [0, 90 - r, 60, 90 + r], atol=1e-11)


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7, 8])
def test_neumann_eigenvalues_rayleigh_ritz(p):
    """Galerkin eigenvalues of -u'' with Neumann ends on [0,1] bound the exact
    ones (k pi)^2 from above; the first converges spectrally."""
    M, K = basis.mass_stiffness(p)
    lam = sl.eigh(K, M, eigvals_only=True)
    assert abs(lam[0]) < 1e-10
    for k in range(1, p + 1):
        assert lam[k] >= (k * math.pi) ** 2 * (1 - 1e-13)
    if p == 7:
        assert abs(lam[1] / math.pi ** 2 - 1) < 1e-9


def test_penalized_eigenvalues_p2_closed_form():
    M = basis.mass_stiffness(2)[0]
    A = basis.penalized_stiffness(2, 2.0)
    r = 6 * math.sqrt(109)
    assert np.allclose(sl.eigh(A, M, eigvals_only=True), [72 - r, 72, 72 + r], atol=1e-11)


# ---------------------------------------------------------------- block operators
H_ANISO = (0.7, 1.9, 0.45)


@pytest.mark.parametrize("p", [1, 2, 3, 7])
def test_neumann_block_properties(p):
    A = dense.dense_operator(p, H_ANISO, dense.NEUMANN)
    n3 = (p + 1) ** 3
    assert np.max(np.abs(A @ np.ones(n3))) < 1e-12 * np.max(np.abs(A))
    assert np.allclose(A, A.T, atol=1e-14 * np.max(np.abs(A)))
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > -1e-12 * ev[-1]
    assert np.sum(ev < 1e-10 * ev[-1]) == 1   # only the constants


@pytest.mark.parametrize("p", [1, 2, 3, 7])
def test_cell_block_spd(p):
    D = dense.dense_operator(p, H_ANISO, dense.CELL)
    assert np.allclose(D, D.T, atol=1e-14 * np.max(np.abs(D)))
    assert np.linalg.eigvalsh(D)[0] > 0
    np.linalg.cholesky(D)


def _interp_monomial(p, h, a, b, c):
    x = basis.gll_nodes(p)
    X = x * h[0]
    Y = x * h[1]
    Z = x * h[2]
    return np.einsum("i,j,k->ijk", X ** a, Y ** b, Z ** c).reshape(-1)


def _sq(hd, e):
    return hd ** (2 * e + 1) / (2 * e + 1)


@pytest.mark.parametrize("p,abc", [(1, (1, 1, 1)), (2, (1, 2, 0)), (3, (1, 2, 3)),
                                   (3, (3, 0, 2)), (7, (7, 1, 4)), (7, (0, 5, 6))])
def test_energy_of_interpolated_polynomial(p, abc):
    """u^T A u = int |grad q|^2 exactly for q = x^a y^b z^c in Q_p on an
    anisotropic box; also 1^T M3 1 = hx hy hz.  Distinct exponents and edge
    lengths pin the Kronecker slot order and the per-axis scaling."""
    h = H_ANISO
    a, b, c = abc
    u = _interp_monomial(p, h, a, b, c)
    A = dense.dense_operator(p, h, dense.NEUMANN)
    e = np.array(abc)
    exact = 0.0
    for d in range(3):
        if e[d] == 0:
            continue
        term = e[d] ** 2 * h[d] ** (2 * e[d] - 1) / (2 * e[d] - 1)
        for o in range(3):
            if o != d:
                term *= _sq(h[o], e[o])
        exact += term
    got = u @ A @ u
    assert abs(got - exact) <= 1e-11 * max(1.0, abs(exact)) * 10 ** max(0, p - 4)
    M3 = dense.dense_mass(p, h)
    one = np.ones((p + 1) ** 3)
    assert abs(one @ M3 @ one - h[0] * h[1] * h[2]) < 1e-13


@pytest.mark.parametrize("p,abc", [(2, (1, 2, 0)), (3, (1, 2, 3)), (3, (0, 0, 0)),
                                   (7, (7, 1, 4))])
@pytest.mark.parametrize("C", [1.0, 2.0])
def test_cell_block_energy_closed_form(p, abc, C):
    """u^T D u for q = x^a y^b z^c equals the SIPG cell energy written out:
    int|grad q|^2 + sum over axes of the own-side face terms
      right face: int_F sigma q^2 - q d_n q,  left face: int_F sigma q^2 + q d_n q,
    with sigma = C p (p+1) / h_normal (Sec. 5.2, Sec. 6.2)."""
    h = H_ANISO
    e = np.array(abc)
    u = _interp_monomial(p, h, *abc)
    D = dense.dense_operator(p, h, dense.CELL, C)
    exact = 0.0
    for d in range(3):
        other = 1.0
        for o in range(3):
            if o != d:
                other *= _sq(h[o], e[o])
        if e[d] > 0:
            exact += e[d] ** 2 * h[d] ** (2 * e[d] - 1) / (2 * e[d] - 1) * other
        sigma = C * p * (p + 1) / h[d]
        q2_right = h[d] ** (2 * e[d]) * other
        qdq_right = (e[d] * h[d] ** (2 * e[d] - 1) if e[d] > 0 else 0.0) * other
        q2_left = (1.0 if e[d] == 0 else 0.0) * other
        exact += sigma * (q2_right + q2_left) - qdq_right
    got = u @ D @ u
    assert abs(got - exact) <= 1e-11 * max(1.0, abs(exact)) * 10 ** max(0, p - 4)


@pytest.mark.parametrize("p", [1, 2, 3, 7])
def test_isotropic_scaling(p):
    for op in (dense.NEUMANN, dense.CELL):
        A1 = dense.dense_operator(p, (1, 1, 1), op)
        Ah = dense.dense_operator(p, (0.3, 0.3, 0.3), op)
        assert np.allclose(Ah, 0.3 * A1, rtol=0, atol=1e-13 * np.max(np.abs(A1)))


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_kronecker_sum_eigenvalues(p):
    """Generalized eigenvalues of (D, M3) are all sums lx_i + ly_j + lz_k of
    the 1D generalized eigenvalues (the identity behind fast
    diagonalization, Sec. 5.2)."""
    h = H_ANISO
    D = dense.dense_operator(p, h, dense.CELL)
    M3 = dense.dense_mass(p, h)
    lam3 = np.sort(sl.eigh(D, M3, eigvals_only=True))
    M, A = dense.reference_pair(p, dense.CELL)
    lam1 = sl.eigh(A, M, eigvals_only=True)
    sums = np.sort((lam1[:, None, None] / h[0] ** 2 + lam1[None, :, None] / h[1] ** 2
                    + lam1[None, None, :] / h[2] ** 2).reshape(-1))
    assert np.allclose(lam3, sums, rtol=1e-10)


# ---------------------------------------------------------------- brute force
def _indep_basis(nodes):
    """Lagrange polynomials as power-series coefficients by exact interpolation."""
    n = len(nodes)
    polys = []
    for j in range(n):
        y = np.zeros(n)
        y[j] = 1.0
        polys.append(P.polyfit(nodes, y, n - 1))
    return polys


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("op", [dense.NEUMANN, dense.CELL])
def test_bruteforce_quadrature_assembly(p, op):
    """Assemble the block by 3D Gauss quadrature of grad phi_q . grad phi_r
    (plus, for the cell block, 2D face quadrature of the own-side SIPG terms
    on all six faces) with a basis built independently from closed-form
    nodes, then compare with the dense Kronecker oracle."""
    nodes = {1: [0.0, 1.0], 2: [0.0, 0.5, 1.0],
             3: [0.0, (1 - 1 / math.sqrt(5)) / 2, (1 + 1 / math.sqrt(5)) / 2, 1.0]}[p]
    nodes = np.array(nodes)
    polys = _indep_basis(nodes)
    dpolys = [P.polyder(c) for c in polys]
    n = p + 1
    h = H_ANISO
    C = 2.0
    xg, wg = np.polynomial.legendre.leggauss(p + 2)
    xg = 0.5 * (xg + 1)
    wg = 0.5 * wg

    def ev(cs, t):
        return np.array([P.polyval(t, c) for c in cs])  # (n, len(t))

    # 1D tables in reference coordinates
    Lq, Dq = ev(polys, xg), ev(dpolys, xg)
    n3 = n ** 3
    A = np.zeros((n3, n3))
    idx = [(i, j, k) for i in range(n) for j in range(n) for k in range(n)]
    for qa, ia in enumerate(xg):
        for qb, ib in enumerate(xg):
            for qc, ic in enumerate(xg):
                w = wg[qa] * wg[qb] * wg[qc] * h[0] * h[1] * h[2]
                grad = np.array([[Dq[i, qa] / h[0] * Lq[j, qb] * Lq[k, qc],
                                  Lq[i, qa] * Dq[j, qb] / h[1] * Lq[k, qc],
                                  Lq[i, qa] * Lq[j, qb] * Dq[k, qc] / h[2]] for (i, j, k) in idx])
                A += w * grad @ grad.T
    if op == dense.CELL:
        for d in range(3):
            sigma = C * p * (p + 1) / h[d]
            t1, t2 = [o for o in range(3) if o != d]
            for side, t in ((+1, 1.0), (-1, 0.0)):
                Lt = ev(polys, np.array([t]))[:, 0]
                Dt = ev(dpolys, np.array([t]))[:, 0] / h[d]
                for qa in range(len(xg)):
                    for qb in range(len(xg)):
                        w = wg[qa] * wg[qb] * h[t1] * h[t2]
                        val = np.empty(n3)
                        dn = np.empty(n3)
                        for q, ijk in enumerate(idx):
                            tang = Lq[ijk[t1], qa] * Lq[ijk[t2], qb]
                            val[q] = Lt[ijk[d]] * tang
                            dn[q] = Dt[ijk[d]] * tang
                        # right face (cell is K-): sigma u v - 1/2(du v + u dv)
                        # left face  (cell is K+): sigma u v + 1/2(du v + u dv)
                        A += w * (sigma * np.outer(val, val)
                                  - side * 0.5 * (np.outer(val, dn) + np.outer(dn, val)))
    ref = dense.dense_operator(p, h, op, C)
    assert np.max(np.abs(A - ref)) < 1e-12 * np.max(np.abs(ref))


# ---------------------------------------------------------------- solve
@pytest.mark.parametrize("p,h", [(2, (0.125,) * 3), (3, (0.5, 4.0, 4.0)), (7, (0.5, 4.0, 1.3))])
def test_solve_long_double_residual(p, h):
    """The dense-solve oracle leaves a residual, formed in long double, at the
    level of a few ulps of |D||x| (the exact solution up to rounding)."""
    rng = np.random.default_rng(11)
    n3 = (p + 1) ** 3
    r = rng.uniform(-1, 1, size=(2, n3))
    x = dense.solve(p, np.array([h, h]), r)
    D = dense.dense_operator(p, h, dense.CELL)
    for b in range(2):
        res = r[b].astype(np.longdouble) - D.astype(np.longdouble) @ x[b].astype(np.longdouble)
        scale = np.abs(D) @ np.abs(x[b])
        assert np.max(np.abs(res.astype(np.float64)) / scale) < 4 * np.finfo(float).eps


def test_solve_recovers_unit_vectors():
    """D applied to the oracle's D^{-1} e_j gives e_j (A A^{-1} = I)."""
    p, h = 3, (0.6, 1.7, 0.9)
    n3 = (p + 1) ** 3
    E = np.eye(n3)
    X = dense.solve(p, np.tile(h, (n3, 1)), E)
    D = dense.dense_operator(p, h, dense.CELL)
    assert np.max(np.abs(X @ D.T - E)) < 1e-13


# ---------------------------------------------------------------- explicit per-block factors
def _brute_kronecker_sum(pairs):
    """Entry by entry: A[(i,j,k),(a,b,c)] = Px[i,a] My[j,b] Mz[k,c] + Mx[i,a] Py[j,b] Mz[k,c]
    + Mx[i,a] My[j,b] Pz[k,c], with the DoF index q = (i n + j) n + k."""
    (Mx, Px), (My, Py), (Mz, Pz) = pairs
    n = Mx.shape[0]
    A = np.zeros((n ** 3, n ** 3))
    for i in range(n):
        for j in range(n):
            for k in range(n):
                for a in range(n):
                    for b in range(n):
                        for c in range(n):
                            A[(i * n + j) * n + k, (a * n + b) * n + c] = (
                                Px[i, a] * My[j, b] * Mz[k, c] + Mx[i, a] * Py[j, b] * Mz[k, c]
                                + Mx[i, a] * My[j, b] * Pz[k, c])
    return A


@pytest.mark.parametrize("n", [2, 3])
def test_kronecker_sum_entrywise(n):
    rng = np.random.default_rng(90 + n)
    pairs = [(rng.standard_normal((n, n)), rng.standard_normal((n, n))) for _ in range(3)]
    assert np.allclose(dense.kronecker_sum(pairs), _brute_kronecker_sum(pairs), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("p", [2, 3])
def test_explicit_factors_reduce_to_scaled_operator(p):
    rng = np.random.default_rng(7 + p)
    h = rng.uniform(0.5, 2.0, size=(4, 3))
    u = rng.uniform(-1, 1, size=(4, (p + 1) ** 3))
    for op in (dense.NEUMANN, dense.CELL):
        M_all = np.array([[f[0] for f in dense.direction_factors(p, hb, op)] for hb in h])
        P_all = np.array([[f[1] for f in dense.direction_factors(p, hb, op)] for hb in h])
        assert np.array_equal(dense.apply_factors(M_all, P_all, u), dense.apply(p, h, u, op))
    x = dense.solve_factors(M_all, P_all, u)
    assert np.allclose(x, dense.solve(p, h, u), rtol=1e-13, atol=0)


def test_solve_factors_residual():
    rng = np.random.default_rng(5)
    n = 3
    M_all = np.empty((2, 3, n, n))
    P_all = np.empty((2, 3, n, n))
    for b in range(2):
        for d in range(3):
            G = rng.standard_normal((n, n))
            M_all[b, d] = G @ G.T + n * np.eye(n)
            H = rng.standard_normal((n, n))
            P_all[b, d] = H @ H.T + np.eye(n)
    r = rng.standard_normal((2, n ** 3))
    x = dense.solve_factors(M_all, P_all, r)
    for b in range(2):
        A = _brute_kronecker_sum([(M_all[b, d], P_all[b, d]) for d in range(3)]).astype(np.longdouble)
        res = r[b].astype(np.longdouble) - A @ x[b].astype(np.longdouble)
        assert float(np.abs(res).max()) < 1e-14 * float(np.abs(r[b]).max()) * 10
