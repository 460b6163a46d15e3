"""Pins of the coupled SIPG oracle (oracle/sipg.py) against what the
mathematics fixes: Galerkin consistency of eq. (sipg) for polynomials of
Q_p, the penalty energy of piecewise constants, symmetry and definiteness,
and the paper's statement that the cell block of eq. (cell_block) is the
cell-diagonal part of the operator."""
import math

import numpy as np
import numpy.polynomial.polynomial as P
import pytest
import scipy.sparse as sp

from oracle import basis, dense, sipg

H = (0.7, 1.3, 0.45)


def node_coords(p, m, h):
    """Global (x, y, z) of every DoF in canonical order."""
    x = basis.gll_nodes(p)
    n = p + 1
    out = np.empty((m[0] * m[1] * m[2], n, n, n, 3))
    for c in range(m[0] * m[1] * m[2]):
        cc = sipg.cell_coords(m, c)
        X = (cc[0] + x) * h[0]
        Y = (cc[1] + x) * h[1]
        Z = (cc[2] + x) * h[2]
        out[c, ..., 0] = X[:, None, None]
        out[c, ..., 1] = Y[None, :, None]
        out[c, ..., 2] = Z[None, None, :]
    return out.reshape(-1, 3)


def poly_factors(p, m, h, vanish, seed):
    """Per-axis polynomial factors q_d of a product q = q_x(x) q_y(y) q_z(z)
    in Q_p (power-series coefficients): x (L - x) (x + c)^k with k <= p - 2
    when vanish, else a random polynomial of degree p."""
    rng = np.random.default_rng(seed)
    fac = []
    for d in range(3):
        L = m[d] * h[d]
        if vanish:
            k = min(p - 2, 1 + d % 2)
            c = np.array([0.0, L, -1.0])                            # x (L - x)
            for _ in range(k):
                c = P.polymul(c, [rng.uniform(0.2, 0.9), 1.0])
            fac.append(c)
        else:
            fac.append(rng.uniform(-1, 1, p + 1))
    return fac


def eval_q(fac, X, deriv=(0, 0, 0)):
    v = np.ones(len(X))
    for d in range(3):
        c = fac[d]
        for _ in range(deriv[d]):
            c = P.polyder(c)
        v *= P.polyval(X[:, d], c)
    return v


def neg_laplacian(fac, X):
    return -(eval_q(fac, X, (2, 0, 0)) + eval_q(fac, X, (0, 2, 0)) + eval_q(fac, X, (0, 0, 2)))


@pytest.mark.parametrize("p", [2, 3, 7])
def test_interior_face_matrices_match_face_blocks(p):
    """The 1D face matrices written from the bilinear form equal the four
    interior blocks pinned against the printed Hermite stencil."""
    e0, g0, e1, g1 = basis.endpoint_vectors(p)
    ref = basis.face_blocks(e0, g0, e1, g1, basis.penalty_reference(p, 2.0))
    for hd in (1.0, 0.37):
        for key in ref:
            got = sipg.face_matrix(p, hd, key[0], key[1]) * hd
            assert np.allclose(got, ref[key], rtol=0, atol=1e-12 * np.max(np.abs(ref[key])))


@pytest.mark.parametrize("p", [2, 3])
def test_interior_diagonal_block_is_cell_block(p):
    """Sec. 5.2: the cell block is the cell-diagonal part of the operator; for
    a cell with no boundary face it is exactly eq. (cell_block)."""
    m = (3, 3, 3)
    c = sipg.cell_index(m, 1, 1, 1)
    blocks = dict(sipg.cell_row_blocks(p, m, H, c))
    D = dense.dense_operator(p, H, dense.CELL)
    assert np.max(np.abs(blocks[c] - D)) < 1e-12 * np.max(np.abs(D))
    # a corner cell's block differs (Nitsche faces), by a symmetric correction
    c0 = sipg.cell_index(m, 0, 0, 0)
    b0 = dict(sipg.cell_row_blocks(p, m, H, c0))[c0]
    assert np.max(np.abs(b0 - D)) > 1e-3 * np.max(np.abs(D))
    assert np.allclose(b0, b0.T, atol=1e-12 * np.max(np.abs(D)))


@pytest.mark.parametrize("p,m", [(2, (2, 3, 2)), (3, (3, 2, 4)), (7, (2, 1, 2))])
def test_consistency_for_polynomials_vanishing_on_the_boundary(p, m):
    """Eq. (sipg) is consistent: for q in Q_p with q = 0 on the boundary of
    the box, A u_q = M f with f = -Lap q (f in Q_p, exact mass)."""
    fac = poly_factors(p, m, H, vanish=True, seed=p)
    X = node_coords(p, m, H)
    u = eval_q(fac, X)
    f = neg_laplacian(fac, X)
    A = sipg.assemble(p, m, H)
    lhs = A @ u
    rhs = sipg.mass(p, m, H) @ f
    scale = np.max(np.abs(abs(A) @ np.abs(u)))
    assert np.max(np.abs(lhs - rhs)) < 1e-11 * scale * 10 ** max(0, p - 4)


def _indep_basis(nodes):
    polys = []
    for j in range(len(nodes)):
        y = np.zeros(len(nodes))
        y[j] = 1.0
        polys.append(P.polyfit(nodes, y, len(nodes) - 1))
    return polys


def boundary_functional(p, m, h, fac, C=2.0):
    """b_i = sum over boundary faces of int_F (sigma q phi_i - q d_n phi_i),
    by 2D Gauss quadrature with a Lagrange basis built independently of the
    oracle (power-series interpolation on the nodes)."""
    n = p + 1
    nodes = basis.gll_nodes(p)
    L = _indep_basis(nodes)
    dL = [P.polyder(c) for c in L]
    xg, wg = np.polynomial.legendre.leggauss(p + 2)
    xg = 0.5 * (xg + 1)
    wg = 0.5 * wg
    Lq = np.array([P.polyval(xg, c) for c in L])           # (n, nq)
    ncell = m[0] * m[1] * m[2]
    b = np.zeros((ncell, n, n, n))
    for c in range(ncell):
        cc = sipg.cell_coords(m, c)
        for d in range(3):
            t1, t2 = [o for o in range(3) if o != d]
            for end in (0, 1):
                if (end == 0 and cc[d] != 0) or (end == 1 and cc[d] != m[d] - 1):
                    continue
                sigma = C * p * (p + 1) / h[d]
                outward = 1.0 if end == 1 else -1.0
                tr = np.array([P.polyval(float(end), c_) for c_ in L])
                dn = outward * np.array([P.polyval(float(end), c_) for c_ in dL]) / h[d]
                # quadrature points on the face
                pts = np.zeros((len(xg), len(xg), 3))
                pts[..., d] = (cc[d] + end) * h[d]
                pts[..., t1] = ((cc[t1] + xg) * h[t1])[:, None]
                pts[..., t2] = ((cc[t2] + xg) * h[t2])[None, :]
                qv = eval_q(fac, pts.reshape(-1, 3)).reshape(len(xg), len(xg))
                w = np.outer(wg, wg) * h[t1] * h[t2]
                # tangential integrals of q against L_a(t1) L_b(t2)
                T = np.einsum("ab,ia,jb->ij", w * qv, Lq, Lq)
                term = np.einsum("k,ij->kij", sigma * tr - dn, T)   # (normal, t1, t2)
                b[c] += np.moveaxis(term, [0, 1, 2], [d, t1, t2])
    return b.reshape(-1)


@pytest.mark.parametrize("p,m", [(2, (2, 2, 3)), (3, (2, 3, 2)), (7, (1, 2, 1))])
def test_consistency_with_boundary_data(p, m):
    """For any q in Q_p, integrating the cell terms by parts gives
    A u_q = M (-Lap q) + b with b the boundary functional of the Nitsche
    terms, int_F (sigma q phi - q d_n phi), computed here by quadrature."""
    fac = poly_factors(p, m, H, vanish=False, seed=10 + p)
    X = node_coords(p, m, H)
    u = eval_q(fac, X)
    A = sipg.assemble(p, m, H)
    rhs = sipg.mass(p, m, H) @ neg_laplacian(fac, X) + boundary_functional(p, m, H, fac)
    scale = np.max(np.abs(abs(A) @ np.abs(u)))
    assert np.max(np.abs(A @ u - rhs)) < 1e-11 * scale * 10 ** max(0, p - 4)


@pytest.mark.parametrize("p", [2, 3, 7])
def test_penalty_energy_of_piecewise_constants(p):
    """For cell-wise constants the gradient terms vanish and
    u^T A u = sum_F sigma_F |F| [u]^2 over interior and boundary faces."""
    m = (3, 2, 2)
    h = H
    n3 = (p + 1) ** 3
    A = sipg.assemble(p, m, h)
    sig = [basis.penalty_reference(p, 2.0) / h[d] for d in range(3)]
    area = [h[1] * h[2], h[0] * h[2], h[0] * h[1]]
    rng = np.random.default_rng(p)
    vals = rng.uniform(-1, 1, m)
    u = np.repeat(np.array([vals[sipg.cell_coords(m, c)] for c in range(12)]), n3)
    exact = 0.0
    for cx in range(m[0]):
        for cy in range(m[1]):
            for cz in range(m[2]):
                cc = (cx, cy, cz)
                for d in range(3):
                    lo = list(cc)
                    lo[d] -= 1
                    jump_lo = vals[cc] - (vals[tuple(lo)] if cc[d] > 0 else 0.0)
                    exact += sig[d] * area[d] * jump_lo ** 2
                    if cc[d] == m[d] - 1:
                        exact += sig[d] * area[d] * vals[cc] ** 2
    got = u @ (A @ u)
    assert abs(got - exact) < 1e-11 * abs(exact) * 10 ** max(0, p - 4)


@pytest.mark.parametrize("p,m", [(2, (2, 3, 2)), (3, (2, 2, 2))])
def test_symmetric_positive_definite(p, m):
    A = sipg.assemble(p, m, H)
    assert abs(A - A.T).max() < 1e-12 * abs(A).max()
    lam = np.linalg.eigvalsh(A.toarray())
    assert lam[0] > 0
    # and the volume part alone annihilates constants (Neumann cells)
    one = np.ones(A.shape[0])
    V = sipg.assemble(p, m, H, sipg.VOLUME)
    assert np.max(np.abs(V @ one)) < 1e-12 * abs(V).max()
    F = sipg.assemble(p, m, H, sipg.FACE)
    assert abs(A - V - F).max() < 1e-13 * abs(A).max()


def test_cell_apply_equals_assembled_rows():
    p, m = 3, (3, 4, 2)
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, 24 * 64)
    cells = [0, 5, 13, 23]
    for part in (sipg.FULL, sipg.FACE):
        full = sipg.apply(p, m, H, u, part).reshape(-1, 64)
        got = sipg.cell_apply(p, m, H, u, cells, part)
        assert np.allclose(got, full[cells], rtol=0, atol=1e-13 * np.max(np.abs(full)))


@pytest.mark.parametrize("p,m", [(2, (3, 3, 4)), (3, (2, 3, 3))])
def test_pcg_reaches_the_direct_solution(p, m):
    """The oracle's PCG with the block-Jacobi preconditioner converges to the
    sparse direct solution within its residual bound, and its iterates satisfy
    the stopping rule on the true residual."""
    import scipy.sparse.linalg as spl
    A = sipg.assemble(p, m, H)
    b = np.random.default_rng(3).uniform(-1, 1, A.shape[0])
    xs = spl.spsolve(A.tocsc(), b)
    x, it, rel = sipg.pcg(A, b, lambda r: sipg.block_jacobi(p, m, H, r), 1e-10, 500)
    assert rel <= 1e-10 and 0 < it < 500
    assert np.linalg.norm(b - A @ x) <= 1.01e-10 * np.linalg.norm(b)
    cond = np.linalg.cond(A.toarray())
    assert np.linalg.norm(x - xs) <= 2 * cond * 1e-10 * np.linalg.norm(xs)
    # the preconditioner is the inverse of the cell-diagonal blocks
    r = np.random.default_rng(4).uniform(-1, 1, A.shape[0])
    z = sipg.block_jacobi(p, m, H, r)
    n3 = (p + 1) ** 3
    c = sipg.cell_index(m, 1, 1, 1)
    D = dense.dense_operator(p, H, dense.CELL)
    assert np.allclose(D @ z[c * n3:(c + 1) * n3], r[c * n3:(c + 1) * n3], atol=1e-12)


def test_pcg_without_preconditioner_is_cg_with_exact_termination():
    """Unpreconditioned CG on a small SPD system reaches the solution in at
    most N iterations (exact-arithmetic termination, up to rounding)."""
    A = sipg.assemble(1, (2, 1, 2), H)
    b = np.random.default_rng(5).uniform(-1, 1, A.shape[0])
    x, it, rel = sipg.pcg(A, b, lambda r: r.copy(), 1e-12, 10 * A.shape[0])
    assert rel <= 1e-12
    import scipy.sparse.linalg as spl
    xs = spl.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
