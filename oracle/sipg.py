"""The coupled SIPG operator on a uniform Cartesian box mesh, assembled as a
sparse matrix from its definition.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed:

* Sec. 3, eq. (sipg): the bilinear form sums the cell integrals of
  grad u . grad v and, over every face F, the terms -{d_n u}[v] - [u]{d_n v}
  + sigma_F [u][v].  The problem has homogeneous Dirichlet data, imposed
  weakly: on a boundary face the jump is the inner trace and the average is
  the inner normal derivative (the usual Nitsche modification the paper
  refers to).
* Eq. (operator_split): A = A^vol + A^face, the cell integrals and the face
  integrals kept apart.
* Sec. 3 (face integrals), eq. (face_factorized): on an axis-aligned face the
  coupling of the two adjacent cells is a Kronecker product with a 1D face
  matrix N^{ss'} in the normal slot and the 1D mass matrix in the two
  tangential slots; eq. (face_coupling) gives N^{--}.
* Sec. 6.2: sigma_F = C p (p+1) / h_F with h_F the cell length normal to F.

Basis: every function takes ``bname``, the 1D basis of each cell's
coefficients: the Lagrange basis on the Gauss-Lobatto nodes (default) or the
Hermite-type basis of Sec. 3.1 (``hermite``); the operator is assembled from
that basis' own mass and stiffness matrices and endpoint vectors.

Mesh: mx x my x mz cells, all with edge lengths (hx, hy, hz).  Cell
(cx, cy, cz) has index c = (cx my + cy) mz + cz and its DoFs are the global
unknowns c n^3 + q with the block-local q = (ix n + iy) n + iz.

The 1D face matrices are written directly from the bilinear form (function
``face_matrix``): no sum factorization, no fast diagonalization, no
rank-two shortcut.  Every cell row is assembled from dense n^3 x n^3 blocks.

Pins (tests/test_oracle_sipg.py): Galerkin consistency for polynomials of
Q_p that vanish on the boundary (A u_q = M f with f = -Lap q), the same for
polynomials that do not vanish there against a boundary functional computed
by independent face quadrature, the penalty energy of piecewise constants,
symmetry and definiteness, the interior cell-diagonal block equal to the cell
block of eq. (cell_block), and the interior face matrices equal to the
printed-stencil-pinned ``basis.face_blocks``.  ``pcg`` (textbook
preconditioned CG) with ``block_jacobi`` (dense solves with the cell blocks,
the preconditioner of Sec. 5.2) is pinned by the sparse direct solution.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis, dense, hermite

LAGRANGE = "lagrange"   # Lagrange basis on the Gauss-Lobatto nodes
HERMITE = "hermite"     # the Hermite-type basis of Sec. 3.1 (p >= 3)

FULL = "full"       # A = A^vol + A^face
VOLUME = "volume"   # A^vol: the cell integrals only (the Neumann volume operator per cell)
FACE = "face"       # A^face: every face integral, interior and boundary


def cell_index(m, cx, cy, cz) -> int:
    return (cx * m[1] + cy) * m[2] + cz


def cell_coords(m, c):
    cz = c % m[2]
    cy = (c // m[2]) % m[1]
    cx = c // (m[1] * m[2])
    return cx, cy, cz


def ref_data(p: int, bname: str = LAGRANGE):
    """(M_hat, K_hat, (e0, g0, e1, g1)) of the 1D basis."""
    if bname == LAGRANGE:
        M, K = basis.mass_stiffness(p)
        return M, K, basis.endpoint_vectors(p)
    if bname == HERMITE:
        M, K = hermite.mass_stiffness(p)
        return M, K, hermite.endpoint_vectors(p)
    raise ValueError(f"unknown basis {bname!r}")


def _side_data(p: int, hd: float, side: str, bname: str = LAGRANGE):
    """(trace row, normal-derivative row, jump sign, average weight) of one
    side of a face normal to an axis, with the normal pointing along +axis.

    '-' : the cell below the face (the face is its right end), jump sign +1
    '+' : the cell above the face (the face is its left end), jump sign -1
    'b-': a boundary face at a cell's right end (outside is empty)
    'b+': a boundary face at a cell's left end
    Interior averages weigh each side by 1/2; on a boundary face the inner
    side carries the whole average.
    """
    e0, g0, e1, g1 = ref_data(p, bname)[2]
    if side in ("-", "b-"):
        t, d, j = e1, g1 / hd, 1.0
    else:
        t, d, j = e0, g0 / hd, -1.0
    return t, d, j, (0.5 if side in ("-", "+") else 1.0)


def face_matrix(p: int, hd: float, test_side: str, trial_side: str, C: float = 2.0,
                bname: str = LAGRANGE) -> np.ndarray:
    """1D face matrix N[i, j] of eq. (sipg) restricted to the normal direction:
    test function i on test_side, trial function j on trial_side,

      N = -(avg d_n trial) (jump test) - (jump trial) (avg d_n test)
          + sigma (jump trial) (jump test),  sigma = C p (p+1) / hd.
    """
    sigma = basis.penalty_reference(p, C) / hd
    ti, di, ji, ai = _side_data(p, hd, test_side, bname)
    tj, dj, jj, aj = _side_data(p, hd, trial_side, bname)
    return (-np.outer(ji * ti, aj * dj) - np.outer(ai * di, jj * tj)
            + sigma * np.outer(ji * ti, jj * tj))


def _slot_kron(p, h, d, N1, bname=LAGRANGE):
    """Kronecker product with N1 in slot d and the physical mass h_o M_hat in
    the other two slots (eq. (face_factorized))."""
    M = ref_data(p, bname)[0]
    f = [h[o] * M for o in range(3)]
    f[d] = N1
    return np.kron(np.kron(f[0], f[1]), f[2])


def cell_row_blocks(p: int, m, h, c: int, part: str = FULL, C: float = 2.0, bname: str = LAGRANGE):
    """The blocks of cell c's row of A: a list of (neighbour cell, n^3 x n^3
    block), the cell itself first."""
    h = [float(x) for x in h]
    n3 = (p + 1) ** 3
    diag = np.zeros((n3, n3))
    off = []
    M, K, _ = ref_data(p, bname)
    if part in (FULL, VOLUME):
        diag += dense.kronecker_sum([(hd * M, K / hd) for hd in h])
    if part in (FULL, FACE):
        cc = list(cell_coords(m, c))
        for d in range(3):
            # right end of the cell along d
            if cc[d] + 1 < m[d]:
                nb = cc.copy()
                nb[d] += 1
                diag += _slot_kron(p, h, d, face_matrix(p, h[d], "-", "-", C, bname), bname)
                off.append((cell_index(m, *nb), _slot_kron(p, h, d, face_matrix(p, h[d], "-", "+", C, bname), bname)))
            else:
                diag += _slot_kron(p, h, d, face_matrix(p, h[d], "b-", "b-", C, bname), bname)
            # left end
            if cc[d] > 0:
                nb = cc.copy()
                nb[d] -= 1
                diag += _slot_kron(p, h, d, face_matrix(p, h[d], "+", "+", C, bname), bname)
                off.append((cell_index(m, *nb), _slot_kron(p, h, d, face_matrix(p, h[d], "+", "-", C, bname), bname)))
            else:
                diag += _slot_kron(p, h, d, face_matrix(p, h[d], "b+", "b+", C, bname), bname)
    return [(c, diag)] + off


def assemble(p: int, m, h, part: str = FULL, C: float = 2.0, bname: str = LAGRANGE) -> sp.csr_matrix:
    """The global operator (or its volume or face part) as a sparse matrix."""
    n3 = (p + 1) ** 3
    ncell = int(m[0] * m[1] * m[2])
    rows, cols, vals = [], [], []
    li = np.repeat(np.arange(n3), n3)
    lj = np.tile(np.arange(n3), n3)
    for c in range(ncell):
        for nb, blk in cell_row_blocks(p, m, h, c, part, C, bname):
            rows.append(c * n3 + li)
            cols.append(nb * n3 + lj)
            vals.append(blk.reshape(-1))
    N = ncell * n3
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return A.tocsr()


def apply(p: int, m, h, u, part: str = FULL, C: float = 2.0, bname: str = LAGRANGE) -> np.ndarray:
    """v = A u for a canonical vector u of ncells * n^3 values."""
    return assemble(p, m, h, part, C, bname) @ np.asarray(u, dtype=np.float64)


def cell_apply(p: int, m, h, u, cells, part: str = FULL, C: float = 2.0, bname: str = LAGRANGE) -> np.ndarray:
    """(A u) restricted to the given cells, from their row blocks only (for
    meshes too large to assemble): u is the canonical vector, returns
    (len(cells), n^3)."""
    n3 = (p + 1) ** 3
    u = np.asarray(u, dtype=np.float64).reshape(-1, n3)
    out = np.zeros((len(cells), n3))
    for r, c in enumerate(cells):
        for nb, blk in cell_row_blocks(p, m, h, int(c), part, C, bname):
            out[r] += blk @ u[nb]
    return out


def mass(p: int, m, h, bname: str = LAGRANGE) -> sp.csr_matrix:
    """Global (block-diagonal) mass matrix."""
    ncell = int(m[0] * m[1] * m[2])
    M = ref_data(p, bname)[0]
    Mc = np.kron(np.kron(h[0] * M, h[1] * M), h[2] * M)
    return sp.block_diag([Mc] * ncell, format="csr")


def cell_block(p: int, h, C: float = 2.0, bname: str = LAGRANGE) -> np.ndarray:
    """The cell block of eq. (cell_block): the Kronecker sum of (h_d M_hat,
    A_hat / h_d), A_hat = K_hat + the own-side blocks of both faces."""
    M, K, (e0, g0, e1, g1) = ref_data(p, bname)
    N = basis.face_blocks(e0, g0, e1, g1, basis.penalty_reference(p, C))
    A = K + N["--"] + N["++"]
    return dense.kronecker_sum([(float(hd) * M, A / float(hd)) for hd in h])


def block_jacobi(p: int, m, h, r, C: float = 2.0, bname: str = LAGRANGE) -> np.ndarray:
    """z = D^{-1} r with D the cell-diagonal blocks of Sec. 5.2: the cell block
    of eq. (cell_block) on every cell, boundary cells included (the paper
    keeps the interior stencil there), each solved densely."""
    n3 = (p + 1) ** 3
    ncell = int(m[0] * m[1] * m[2])
    r = np.asarray(r, dtype=np.float64).reshape(ncell, n3)
    D = cell_block(p, h, C, bname)
    return np.linalg.solve(D, r.T).T.reshape(-1)


def pcg(A, b, prec, rtol: float, maxit: int, x0=None, criterion: str = "residual"):
    """Textbook preconditioned conjugate gradients for the SPD system A x = b
    (Hestenes-Stiefel recurrences).  criterion "residual": stop when
    ||b - A x||_2 <= rtol ||b||_2 with the recursively updated residual;
    "preconditioned": stop when the preconditioned residual norm
    <r, z>^{1/2} has decreased by the factor rtol from its initial value
    (the rule of Sec. 6.1).  prec(r) applies the preconditioner.  Returns
    (x, iterations, ||r||_2 / ||b||_2)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.zeros_like(b), 0, 0.0
    z = prec(r)
    pdir = z.copy()
    rz = r @ z
    rz0 = rz
    it = 0

    def converged():
        if criterion == "preconditioned":
            return np.sqrt(rz) <= rtol * np.sqrt(rz0)
        return np.linalg.norm(r) <= rtol * nb

    while not converged() and it < maxit:
        q = A @ pdir
        alpha = rz / (pdir @ q)
        x += alpha * pdir
        r -= alpha * q
        z = prec(r)
        rz_new = r @ z
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
        it += 1
    return x, it, float(np.linalg.norm(r) / nb)
