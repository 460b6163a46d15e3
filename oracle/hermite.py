"""The Hermite-type 1D basis and its reference data, written out plainly in
FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed:

* Sec. 3.1 (the Hermite-type basis), eq. (hermite_conditions): for p >= 3 the
  basis {psi_0, ..., psi_p} of P_p([0, 1]) is fixed by its endpoint data:
  psi_0 carries the value at 0, psi_1 the derivative at 0, psi_{p-1} the
  derivative at 1 and psi_p the value at 1; every other endpoint value and
  derivative of these four vanishes, and the p-3 interior functions have
  vanishing values and derivatives at both ends.  The four endpoint
  functions are the cubic Hermite polynomials; the interior functions are
  Lagrange polynomials on interior Gauss-Lobatto nodes times the quartic
  bubble x^2 (1-x)^2.
* eq. (hermite_traces_1d): value and derivative at each end are
  coefficients of the expansion.
* The change of basis to the Lagrange basis is a fixed (p+1) x (p+1) matrix
  per direction; M and K are tabulated for the new basis.

Readings (the paper leaves them open): the endpoint functions are the cubic
Hermite polynomials themselves (no added bubbles: they already meet every
endpoint condition); the interior Lagrange factors (degree p-4) use the p-3
interior nodes of the Gauss-Lobatto rule with p-1 points.

Polynomials are held as monomial coefficient columns and evaluated and
differentiated exactly with numpy.polynomial.polynomial.

Pins (tests/test_oracle_hermite.py): the endpoint conditions, the cubic
Hermite polynomials in closed form at p = 3, the trace property on random
expansions, M and K against the Lagrange ones transformed by the change of
basis, the generalized eigenvalues of the cell block equal to the Lagrange
ones, the two-layer sparsity of the assembled coupling blocks, and the
assembled operator against the Lagrange operator transformed cell by cell.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import polynomial as P

from . import basis


def monomials(p: int) -> np.ndarray:
    """C[:, j]: monomial coefficients (ascending powers) of psi_j."""
    if p < 3:
        raise ValueError("the Hermite-type basis needs p >= 3")
    C = np.zeros((p + 1, p + 1))
    cubic = {
        0: [1.0, 0.0, -3.0, 2.0],      # value at 0:       1 - 3x^2 + 2x^3
        1: [0.0, 1.0, -2.0, 1.0],      # derivative at 0:  x - 2x^2 + x^3
        p - 1: [0.0, 0.0, -1.0, 1.0],  # derivative at 1:  -x^2 + x^3
        p: [0.0, 0.0, 3.0, -2.0],      # value at 1:       3x^2 - 2x^3
    }
    for j, c in cubic.items():
        C[: len(c), j] = c
    bubble = [0.0, 0.0, 1.0, -2.0, 1.0]                 # x^2 (1-x)^2
    z = basis.gll_nodes(p - 2)[1:-1]                    # p-3 interior nodes
    for k in range(p - 3):
        lk = np.array([1.0])
        for l, zl in enumerate(z):
            if l != k:
                lk = P.polymul(lk, np.array([-zl, 1.0]) / (z[k] - zl))
        c = P.polymul(lk, bubble)
        C[: len(c), 2 + k] = c
    return C


def values(p: int, x) -> np.ndarray:
    """V[q, j] = psi_j(x_q)."""
    C = monomials(p)
    x = np.asarray(x, dtype=np.float64)
    return np.stack([P.polyval(x, C[:, j]) for j in range(p + 1)], axis=-1)


def derivatives(p: int, x) -> np.ndarray:
    """D[q, j] = psi_j'(x_q)."""
    C = monomials(p)
    x = np.asarray(x, dtype=np.float64)
    return np.stack([P.polyval(x, P.polyder(C[:, j])) for j in range(p + 1)], axis=-1)


def transform(p: int) -> np.ndarray:
    """T[i, j] = psi_j(x_i) at the Gauss-Lobatto nodes: Lagrange coefficients
    (nodal values) = T @ Hermite coefficients."""
    return values(p, basis.gll_nodes(p))


def mass_stiffness(p: int):
    """M[i, j] = int psi_i psi_j, K[i, j] = int psi_i' psi_j' by a
    Gauss-Legendre rule with p+2 points (exact for degree 2p+3)."""
    xq, wq = basis.gauss_legendre(p + 2)
    V = values(p, xq)
    D = derivatives(p, xq)
    return (V * wq[:, None]).T @ V, (D * wq[:, None]).T @ D


def endpoint_vectors(p: int):
    """e0 = psi(0), g0 = psi'(0), e1 = psi(1), g1 = psi'(1) (reference scale)."""
    return values(p, [0.0])[0], derivatives(p, [0.0])[0], values(p, [1.0])[0], derivatives(p, [1.0])[0]


def penalized_stiffness(p: int, C: float = 2.0) -> np.ndarray:
    """A_hat of eq. (cell_block) in this basis: K plus the own-side blocks of
    both face stencils."""
    _, K = mass_stiffness(p)
    e0, g0, e1, g1 = endpoint_vectors(p)
    N = basis.face_blocks(e0, g0, e1, g1, basis.penalty_reference(p, C))
    return K + N["--"] + N["++"]


def to_hermite(p: int, u_lagrange, ncell: int) -> np.ndarray:
    """Hermite coefficients of canonical Lagrange (nodal) cell vectors: the
    inverse transform in each of the three directions."""
    n = p + 1
    Ti = np.linalg.inv(transform(p))
    u = np.asarray(u_lagrange, dtype=np.float64).reshape(ncell, n, n, n)
    return np.einsum("ai,bj,ck,eijk->eabc", Ti, Ti, Ti, u).reshape(-1)


def to_lagrange(p: int, u_hermite, ncell: int) -> np.ndarray:
    """Nodal values of canonical Hermite cell vectors."""
    n = p + 1
    T = transform(p)
    u = np.asarray(u_hermite, dtype=np.float64).reshape(ncell, n, n, n)
    return np.einsum("ai,bj,ck,eijk->eabc", T, T, T, u).reshape(-1)


def prolongation_1d(p: int):
    """(P_0, P_1) in this basis: P_c[i, j] = Hermite coefficient i, on child
    c, of psi_j((x + c) / 2): the coarse function evaluated at the child's
    Gauss-Lobatto nodes, then converted to coefficients."""
    x = basis.gll_nodes(p)
    Ti = np.linalg.inv(transform(p))
    return tuple(Ti @ values(p, (x + c) / 2.0) for c in (0, 1))
