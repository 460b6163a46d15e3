"""Pins of the multigrid oracle (oracle/mg.py): the Chebyshev error
polynomial of eq. (chebyshev_error_polynomial), the polynomial embedding of
the level transfers, the smoother's error propagator, the V-cycle's symmetry
and the CG iteration counts the paper reports for this solver class."""
import numpy as np
import numpy.polynomial.chebyshev as Ch
import numpy.polynomial.polynomial as P
import pytest

from oracle import basis, dense, mg, sipg


def test_chebyshev_weights_give_the_chebyshev_error_polynomial():
    """prod_j (1 - omega_j lam) = T_3((c - lam)/d) / T_3(c/d) on [0, 3]."""
    a, b = mg.INTERVAL
    c, d = (a + b) / 2, (b - a) / 2
    w = mg.chebyshev_weights(a, b)
    lam = np.linspace(0.0, 3.0, 301)
    lhs = np.prod([1.0 - wj * lam for wj in w], axis=0)
    T3 = Ch.Chebyshev.basis(3)
    rhs = T3((c - lam) / d) / T3(c / d)
    assert np.max(np.abs(lhs - rhs)) < 1e-13
    # worst case on [a, b] is 1 / |T_3(c/d)|, below the constant-weight (d/c)^3
    inside = (lam >= a) & (lam <= b)
    assert abs(np.max(np.abs(lhs[inside])) - 1 / abs(T3(c / d))) < 1e-3
    assert 1 / abs(T3(c / d)) < (d / c) ** 3


@pytest.mark.parametrize("p", [1, 2, 3])
def test_prolongation_embeds_polynomials(p):
    """The coarse interpolant of q in Q_p, prolonged, is the fine interpolant."""
    mc = 2
    rng = np.random.default_rng(p)
    fac = [rng.uniform(-1, 1, p + 1) for _ in range(3)]

    def interp(m):
        x = basis.gll_nodes(p)
        out = []
        for c in range(m ** 3):
            cc = sipg.cell_coords((m,) * 3, c)
            X, Y, Z = [(cc[d] + x) / m for d in range(3)]
            out.append(np.einsum("i,j,k->ijk", P.polyval(X, fac[0]), P.polyval(Y, fac[1]),
                                 P.polyval(Z, fac[2])).reshape(-1))
        return np.concatenate(out)

    Pm = mg.prolongation(p, mc)
    assert np.max(np.abs(Pm @ interp(mc) - interp(2 * mc))) < 1e-12


@pytest.mark.parametrize("p", [2, 3])
def test_prolongation_preserves_the_mass(p):
    """Nested spaces with exact integration: P^T M_fine P = M_coarse."""
    mc = 2
    Pm = mg.prolongation(p, mc)
    Mf = sipg.mass(p, (2 * mc,) * 3, (1.0 / (2 * mc),) * 3)
    Mc = sipg.mass(p, (mc,) * 3, (1.0 / mc,) * 3)
    assert abs(Pm.T @ Mf @ Pm - Mc).max() < 1e-14 * abs(Mc).max()


def test_smoother_error_propagator():
    """Three Richardson updates act on the error as p_3(D^{-1} A), evaluated
    through the eigen-decomposition of the symmetric D^{-1/2} A D^{-1/2}."""
    p, m = 2, 2
    H = mg.Hierarchy(p, m)
    A = H.A[0].toarray()
    n3 = (p + 1) ** 3
    D = dense.dense_operator(p, (0.5,) * 3, dense.CELL)
    Dfull = np.kron(np.eye(m ** 3), D)
    L = np.linalg.cholesky(Dfull)
    Li = np.linalg.inv(L)
    S = Li @ A @ Li.T
    lam, Q = np.linalg.eigh((S + S.T) / 2)
    pol = np.prod([1.0 - w * lam for w in H.omega], axis=0)
    rng = np.random.default_rng(0)
    xs = rng.uniform(-1, 1, A.shape[0])
    b = A @ xs
    e0 = -xs                                   # start from u = 0
    e3 = H.smooth(0, np.zeros_like(b), b) - xs
    # e3 = D^{-1/2}... in L-coordinates: L^T e3 = Q diag(pol) Q^T L^T e0
    pred = np.linalg.solve(L.T, Q @ (pol * (Q.T @ (L.T @ e0))))
    assert np.max(np.abs(e3 - pred)) < 1e-10 * np.max(np.abs(e0))


def test_vcycle_is_a_symmetric_positive_definite_preconditioner():
    p, m = 2, 4
    H = mg.Hierarchy(p, m)
    N = H.A[0].shape[0]
    rng = np.random.default_rng(1)
    u, w = rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)
    Bu, Bw = H.vcycle(u), H.vcycle(w)
    assert abs(w @ Bu - u @ Bw) < 1e-10 * abs(w @ Bu)
    assert u @ Bu > 0


@pytest.mark.parametrize("p,m", [(3, 4), (2, 8), (3, 6)])
def test_mg_pcg_iteration_counts_are_small_and_mesh_independent(p, m):
    """The paper's CG with this V-cycle converges in about ten iterations on
    uniform meshes (Sec. 6.2); here: at most 16 to 1e-10 in the residual
    norm, far below block-Jacobi's hundred-plus."""
    H = mg.Hierarchy(p, m)
    b = np.random.default_rng(2).uniform(-1, 1, H.A[0].shape[0])
    x, it, rel = sipg.pcg(H.A[0], b, H.vcycle, 1e-10, 200)
    x_bj, it_bj, _ = sipg.pcg(H.A[0], b, lambda r: sipg.block_jacobi(p, (m,) * 3, (1.0 / m,) * 3, r), 1e-10, 2000)
    print(f"p={p} m={m} mg_iters={it} bj_iters={it_bj}")
    assert rel <= 1e-10 and it <= 16 and it < it_bj / 3
    assert np.linalg.norm(x - x_bj) <= 1e-7 * np.linalg.norm(x_bj)


def test_box_hierarchy_reduces_to_the_cube_and_is_symmetric():
    """The hierarchy of a box: on a cube it is the cube's hierarchy bit for
    bit; on a box with unequal counts and lengths its V-cycle is symmetric
    and positive, and its transfers preserve the mass."""
    b = np.random.default_rng(3).uniform(-1, 1, 64 * 27)
    Hc = mg.Hierarchy(2, 4)
    Hb = mg.Hierarchy(2, (4, 4, 4), h=(0.25,) * 3)
    assert np.array_equal(Hc.vcycle(b), Hb.vcycle(b))
    H = mg.Hierarchy(2, (4, 8, 2), h=(0.25, 0.125, 0.4))
    assert H.cells == [(4, 8, 2), (2, 4, 1)]
    rng = np.random.default_rng(4)
    a, c = rng.standard_normal((2, H.A[0].shape[0]))
    Va, Vc = H.vcycle(a), H.vcycle(c)
    assert abs(Va @ c - a @ Vc) <= 1e-11 * np.linalg.norm(Va) * np.linalg.norm(c)
    assert Va @ a > 0
    Mf = sipg.mass(2, H.cells[0], H.hs[0])
    Mc = sipg.mass(2, H.cells[1], H.hs[1])
    P = H.P[0]
    assert np.abs((P.T @ Mf @ P - Mc).toarray()).max() <= 1e-13 * np.abs(Mc.toarray()).max()


# ------------------------------------------------ degree-coarsened coarsest level
@pytest.mark.parametrize("p", [2, 3, 5, 7])
def test_degree_embedding_reproduces_trilinear_functions(p):
    """E maps the degree-1 nodal values of q in Q_1 to its degree-p nodal
    values (the degree-1 nodes are the cell's end points 0 and 1)."""
    rng = np.random.default_rng(20 + p)
    fac = [rng.uniform(-1, 1, 2) for _ in range(3)]
    q = lambda x: [P.polyval(x, f) for f in fac]
    xc, xf = np.array([0.0, 1.0]), basis.gll_nodes(p)
    coarse = np.einsum("i,j,k->ijk", *q(xc)).reshape(-1)
    fine = np.einsum("i,j,k->ijk", *q(xf)).reshape(-1)
    E = mg.degree_embedding(p, 1, (1, 1, 1))
    assert np.max(np.abs(E @ coarse - fine)) < 1e-14
    # a partition of unity per direction, and the end nodes are kept
    E1 = mg.degree_embedding_1d(p, 1)
    assert np.max(np.abs(E1.sum(axis=1) - 1.0)) < 1e-15
    assert np.allclose(E1[0], [1.0, 0.0]) and np.allclose(E1[-1], [0.0, 1.0])


@pytest.mark.parametrize("p", [2, 3])
def test_degree_embedding_preserves_the_mass(p):
    """Nested spaces with exact quadrature: E^T M_p E = M_1 on the same cells."""
    cells, h = (2, 3, 1), (0.5, 1.0 / 3, 0.7)
    E = mg.degree_embedding(p, 1, cells)
    Mf, Mc = sipg.mass(p, cells, h), sipg.mass(1, cells, h)
    assert np.abs((E.T @ Mf @ E - Mc).toarray()).max() <= 1e-14 * np.abs(Mc.toarray()).max()


@pytest.mark.parametrize("p", [2, 3, 4])
def test_galerkin_degree_level_is_the_degree_one_form_with_the_fine_penalty(p):
    """E^T A_p E is the degree-1 SIPG operator assembled with the penalty of
    degree p: sigma = C p (p+1) / h = C' 1 (1+1) / h for C' = C p (p+1) / 2
    (all integrals exact for the embedded functions)."""
    cells, h, C = (3, 2, 1), (1.0 / 3, 0.5, 0.8), 2.0
    H = mg.Hierarchy(p, cells, C=C, h=h, coarse_degree=1)
    assert H.degrees == [p, 1] and H.cells == [cells, cells]
    A1 = sipg.assemble(1, cells, h, sipg.FULL, C * p * (p + 1) / 2.0)
    assert np.abs((H.A[1] - A1).toarray()).max() <= 1e-12 * np.abs(A1.toarray()).max()
    # rediscretizing at degree 1 with its own penalty is a different operator
    A1own = sipg.assemble(1, cells, h, sipg.FULL, C)
    assert np.abs((H.A[1] - A1own).toarray()).max() > 1e-3 * np.abs(A1.toarray()).max()


def test_degree_coarsened_vcycle_is_symmetric_and_converges():
    """The V-cycle with the degree-1 coarsest level: symmetric and positive,
    and CG with it converges in a number of iterations of the same order as
    with the exact coarse solve of the degree-p coarsest level."""
    p, m = 2, 6
    H = mg.Hierarchy(p, m, coarse_degree=1)
    assert H.cells == [(6,) * 3, (3,) * 3, (3,) * 3] and H.degrees == [2, 2, 1]
    rng = np.random.default_rng(5)
    a, c = rng.standard_normal((2, H.A[0].shape[0]))
    Va, Vc = H.vcycle(a), H.vcycle(c)
    assert abs(Va @ c - a @ Vc) <= 1e-11 * np.linalg.norm(Va) * np.linalg.norm(c)
    assert Va @ a > 0
    b = rng.uniform(-1, 1, H.A[0].shape[0])
    _, it_deg, rel = sipg.pcg(H.A[0], b, H.vcycle, 1e-10, 200)
    _, it_exact, _ = sipg.pcg(H.A[0], b, mg.Hierarchy(p, m).vcycle, 1e-10, 200)
    print(f"p={p} m={m} iterations: degree-coarsened {it_deg}, exact coarse {it_exact}")
    assert rel <= 1e-10 and it_deg <= it_exact + 6


def test_degree_coarsening_planted_transpose_is_caught():
    """A plausible slip (the embedding's transpose layout, i.e. kron order
    reversed per direction with swapped factors) must break the Galerkin pin."""
    p, cells, h = 2, (2, 1, 1), (0.5, 1.0, 1.0)
    E1 = mg.degree_embedding_1d(p, 1)
    bad = sp_block([np.kron(np.kron(E1[::-1], E1), E1)] * 2)
    A = sipg.assemble(p, cells, h)
    A1 = sipg.assemble(1, cells, h, sipg.FULL, 2.0 * p * (p + 1) / 2.0)
    assert np.abs((bad.T @ A @ bad - A1).toarray()).max() > 1e-3 * np.abs(A1.toarray()).max()


def sp_block(blocks):
    import scipy.sparse as sp
    return sp.block_diag([sp.csr_matrix(b) for b in blocks], format="csr")
