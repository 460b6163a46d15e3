"""Vertex-patch blocks: the SIPG operator restricted to the 2 x 2 x 2 cells
around a mesh vertex, as one tensor-product block of n = 2(p+1) points per
direction.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed:

* Sec. 6.1 (comparison with a vertex-patch smoother): a patch of cells
  around a vertex is solved as one local problem; on a Cartesian mesh its
  operator keeps the tensor-product structure.
* Sec. 5.2, eq. (cell_block) and eq. (face_coupling): along one direction a
  patch holds two cells of the same length h; its 1D operator has the cell
  block A_hat (stiffness plus the own-side blocks of both faces, i.e. the
  interior stencil on every face, as for the block-Jacobi cells) on each
  cell and the coupling blocks N^{-+}, N^{+-} of the face between them; the
  mass is block-diagonal, one cell mass per cell.

Patch-local DoF order per direction: cell 0's n_c points, then cell 1's.
Pins (tests/test_oracle_patch.py): the patch block equals the rows and
columns of the assembled mesh operator (sipg.assemble) for the eight cells
of an interior patch, for the full operator and for its volume part, with
anisotropic lengths; symmetry, definiteness and the reflection symmetry of
the 1D factors.
"""
from __future__ import annotations

import numpy as np

from . import basis, dense


def patch_factors(p: int, C: float = 2.0):
    """(M_p, K_p, A_p): the reference 1D mass, broken stiffness and patch
    operator of two adjacent cells of degree p, each (2(p+1))^2."""
    M, K = basis.mass_stiffness(p)
    A = basis.penalized_stiffness(p, C)
    e0, g0, e1, g1 = basis.endpoint_vectors(p)
    N = basis.face_blocks(e0, g0, e1, g1, basis.penalty_reference(p, C))
    n = p + 1
    Z = np.zeros((n, n))
    Mp = np.block([[M, Z], [Z, M]])
    Kp = np.block([[K, Z], [Z, K]])
    # cell 0 is the '-' side of the shared face (its right end), cell 1 the '+'
    Ap = np.block([[A, N["-+"]], [N["+-"], A]])
    return Mp, Kp, Ap


def patch_operator(p: int, h, op: str = dense.CELL, C: float = 2.0) -> np.ndarray:
    """The (2(p+1))^3 block of one patch of cells with lengths h: Kronecker
    sum of (h_d M_p, P_p / h_d) with P_p the patch operator (CELL) or the
    broken stiffness (NEUMANN, the cells' volume operators)."""
    Mp, Kp, Ap = patch_factors(p, C)
    P = Ap if op == dense.CELL else Kp
    return dense.kronecker_sum([(float(hd) * Mp, P / float(hd)) for hd in h])


def patch_dofs(p: int, m, corner):
    """Global DoF indices (canonical mesh order) of the patch whose lowest
    cell is `corner`, listed in patch-local order."""
    n = p + 1
    n3 = n ** 3
    out = []
    for X in range(2 * n):
        for Y in range(2 * n):
            for Z in range(2 * n):
                cx, ix = corner[0] + X // n, X % n
                cy, iy = corner[1] + Y // n, Y % n
                cz, iz = corner[2] + Z // n, Z % n
                c = (cx * m[1] + cy) * m[2] + cz
                out.append(c * n3 + (ix * n + iy) * n + iz)
    return np.array(out)
