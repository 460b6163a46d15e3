"""1D reference data of the method, written out plainly in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed:

* Sec. 3.1, eq. (eval_pipeline): the volume operator needs only the 1D mass
  matrix M and stiffness matrix K of the basis, computed exactly once
  ("no quadrature loop" on Cartesian cells).  Here they are the exact
  integrals of products of Lagrange polynomials on the Gauss-Lobatto nodes of
  [0, 1], evaluated by a Gauss-Legendre rule with p+2 points, which is exact
  for the polynomial degree 2p of the integrands.
* Sec. 3, eq. (sipg) and eq. (face_coupling): the SIPG face-coupling blocks
  N^{ss'} built from endpoint values e and scaled endpoint derivatives g, with
  the penalty sigma_F = C p (p+1) / h_F of Sec. 6.2.
* Sec. 5.2, eq. (cell_block): the 1D factor A_hat of the cell block is the
  stiffness matrix plus the own-side 2x2 blocks of both face stencils, i.e.
  K + N^{--}(right face) + N^{++}(left face).

Pins: Gauss-Lobatto nodes against their closed forms; M and K at p=2 against
the textbook matrices; M, K and A_hat against the bilinear forms evaluated on
monomials (closed forms); the own-side and mixed face blocks in a cubic
Hermite basis against the printed stencil eq. (hermite_face_stencil);
generalized eigenvalues against closed forms.
"""
from __future__ import annotations

import numpy as np


def gll_nodes(p: int) -> np.ndarray:
    """Gauss-Lobatto nodes on [0, 1] for degree p (p+1 nodes).

    Endpoints 0 and 1 plus the affine images (1+xi)/2 of the roots xi of the
    derivative of the Legendre polynomial P_p.  The roots come from numpy's
    Legendre class (a library root finder) and are then polished by Newton's
    method on P_p'(xi) using the three-term Legendre recurrence.
    """
    if p < 1:
        raise ValueError("degree must be >= 1")
    if p == 1:
        return np.array([0.0, 1.0])
    dP = np.polynomial.legendre.Legendre.basis(p).deriv()
    xi = np.sort(np.real(dP.roots()))
    for _ in range(20):
        # P_p'(x) and P_p''(x) from the recurrence and the Legendre ODE
        # (1 - x^2) P'' = 2 x P' - p (p+1) P.
        P, dPv = _legendre_and_derivative(p, xi)
        d2P = (2.0 * xi * dPv - p * (p + 1) * P) / (1.0 - xi * xi)
        step = dPv / d2P
        xi = xi - step
        if np.max(np.abs(step)) < 1e-17:
            break
    return np.concatenate(([0.0], 0.5 * (1.0 + xi), [1.0]))


def _legendre_and_derivative(p: int, x: np.ndarray):
    """P_p(x) and P_p'(x) by the Bonnet recurrence (k+1)P_{k+1} = (2k+1)xP_k - kP_{k-1}."""
    x = np.asarray(x, dtype=np.float64)
    P0 = np.ones_like(x)
    P1 = x.copy()
    if p == 0:
        return P0, np.zeros_like(x)
    for k in range(1, p):
        P0, P1 = P1, ((2 * k + 1) * x * P1 - k * P0) / (k + 1)
    # derivative identity (x^2 - 1) P_p' = p (x P_p - P_{p-1})
    dP = p * (x * P1 - P0) / (x * x - 1.0)
    return P1, dP


def gauss_legendre(nq: int):
    """Gauss-Legendre points and weights mapped from [-1, 1] to [0, 1]."""
    xi, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (1.0 + xi), 0.5 * w


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """L[q, j] = l_j(x_q), the Lagrange polynomials of ``nodes``, product form."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    L = np.ones((len(x), n))
    for j in range(n):
        for k in range(n):
            if k != j:
                L[:, j] *= (x - nodes[k]) / (nodes[j] - nodes[k])
    return L


def lagrange_derivatives(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[q, j] = l_j'(x_q) by the product rule applied to the product form:

    l_j'(x) = sum_{m != j} 1/(x_j - x_m) * prod_{k != j, m} (x - x_k)/(x_j - x_k).
    Valid at every x, nodes included.
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for j in range(n):
        for m in range(n):
            if m == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[m]))
            for k in range(n):
                if k != j and k != m:
                    term *= (x - nodes[k]) / (nodes[j] - nodes[k])
            D[:, j] += term
    return D


def mass_stiffness(p: int):
    """Exact reference mass and stiffness matrices of the GLL Lagrange basis.

    M_hat[i, j] = int_0^1 l_i l_j dx,  K_hat[i, j] = int_0^1 l_i' l_j' dx
    (Sec. 3.1, the 1D factors of eq. (eval_pipeline)).  A Gauss-Legendre rule
    with p+2 points integrates polynomials of degree 2p+3 exactly.
    """
    nodes = gll_nodes(p)
    xq, wq = gauss_legendre(p + 2)
    L = lagrange_values(nodes, xq)
    D = lagrange_derivatives(nodes, xq)
    M = (L * wq[:, None]).T @ L
    K = (D * wq[:, None]).T @ D
    return M, K


def endpoint_vectors(p: int):
    """Endpoint data of the GLL basis: e0 = l(0), g0 = l'(0), e1 = l(1), g1 = l'(1).

    These are the vectors e and g of eq. (face_coupling) on the reference
    interval (before the 1/h scaling of g).
    """
    nodes = gll_nodes(p)
    e0 = lagrange_values(nodes, [0.0])[0]
    e1 = lagrange_values(nodes, [1.0])[0]
    g0 = lagrange_derivatives(nodes, [0.0])[0]
    g1 = lagrange_derivatives(nodes, [1.0])[0]
    return e0, g0, e1, g1


def penalty_reference(p: int, C: float = 2.0) -> float:
    """sigma_hat = C p (p+1): the penalty sigma_F = C p(p+1)/h_F of Sec. 6.2 times h_F."""
    return C * p * (p + 1)


def face_blocks(e0, g0, e1, g1, sigma):
    """The four SIPG face-coupling blocks of one face on the reference scale.

    Eq. (sipg) with jump [u] = u^- - u^+, average {d_n u} = (u^-' + u^+')/2,
    both cells mapped with the same orientation so derivatives are along the
    positive axis (Sec. 3.1.1).  The face sits at the right end of cell K^-
    (endpoint data e1, g1) and the left end of cell K^+ (e0, g0).  Row index:
    test function, column index: trial function.  Returns a dict keyed by
    '--', '-+', '+-', '++'.  eq. (face_coupling) prints N^{--}; the other three
    follow from the same bilinear form:

      N^{--} =  sigma e1 e1^T - 1/2 (e1 g1^T + g1 e1^T)
      N^{-+} = -sigma e1 e0^T - 1/2 e1 g0^T + 1/2 g1 e0^T
      N^{+-} = -sigma e0 e1^T + 1/2 e0 g1^T - 1/2 g0 e1^T
      N^{++} =  sigma e0 e0^T + 1/2 (e0 g0^T + g0 e0^T)
    """
    e0, g0, e1, g1 = (np.asarray(v, dtype=np.float64) for v in (e0, g0, e1, g1))
    o = np.outer
    return {
        "--": sigma * o(e1, e1) - 0.5 * (o(e1, g1) + o(g1, e1)),
        "-+": -sigma * o(e1, e0) - 0.5 * o(e1, g0) + 0.5 * o(g1, e0),
        "+-": -sigma * o(e0, e1) + 0.5 * o(e0, g1) - 0.5 * o(g0, e1),
        "++": sigma * o(e0, e0) + 0.5 * (o(e0, g0) + o(g0, e0)),
    }


def penalized_stiffness(p: int, C: float = 2.0) -> np.ndarray:
    """A_hat of eq. (cell_block) on the reference interval:

    A_hat = K_hat + N^{--} (own side of the right face) + N^{++} (own side of
    the left face), with sigma_hat = C p (p+1).  For a cell of length h the
    physical factor is A_hat / h (g carries 1/h, sigma_F carries 1/h).
    """
    _, K = mass_stiffness(p)
    e0, g0, e1, g1 = endpoint_vectors(p)
    N = face_blocks(e0, g0, e1, g1, penalty_reference(p, C))
    return K + N["--"] + N["++"]
