"""Sum-factorized CPU reference for whole batches at full size.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Not the oracle of the
method: it computes the same results as ``dense`` by the factorized route
(successive 1D contractions along z, y, x and, for the inverse, the
generalized eigen-decomposition of each direction), which is what makes it
fast enough to check every block of a full-size batch.  It is pinned against
``dense`` (the plain definition) on samples in tests/test_oracle_sumfact.py,
and it shares no code with the HIP library: the 1D data come from
``basis`` (product-form Lagrange basis, Gauss-Legendre quadrature) and the
eigen-decomposition from LAPACK (``scipy.linalg.eigh``), where the library
builds its own tables with a barycentric basis and a Cholesky + Jacobi
eigen-solver.

Paper passages followed:

* Sec. 3.1, eq. (eval_pipeline): the volume operator of a Cartesian cell is
  the Kronecker sum K (x) M (x) M + M (x) K (x) M + M (x) M (x) K of 1D
  factors scaled by the cell size, evaluated as 1D contractions
  (seven of them: t = M_z u, w = K_z u, a = M_y t, c = K_y t + M_y w,
  v = K_x a + M_x c).
* Sec. 5.2, eq. (cell_block) and the fast diagonalization that follows it:
  with per-direction generalized eigenpairs P_d S_d = M_d S_d Lambda_d,
  S_d^T M_d S_d = I, the inverse of the cell block is
  (S_x (x) S_y (x) S_z) diag(1/(lx_i + ly_j + lz_k)) (S_x (x) S_y (x) S_z)^T,
  six contractions and one diagonal scaling.  For a box of lengths h_d the
  pair (P_hat/h_d, h_d M_hat) has S_d = S_hat/sqrt(h_d) and
  lambda_d = lambda_hat/h_d^2.

Vectors are (nblocks, n^3) in the canonical order q = (i_x n + i_y) n + i_z.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import dense


def _blocks(u, n):
    return np.asarray(u, dtype=np.float64).reshape(-1, n, n, n)


def apply(p: int, h_all, u_all, op: str = dense.NEUMANN, C: float = 2.0) -> np.ndarray:
    """v_b = A_b u_b by seven 1D contractions per block (eq. (eval_pipeline))."""
    n = p + 1
    M, P = dense.reference_pair(p, op, C)
    h = np.asarray(h_all, dtype=np.float64).reshape(-1, 3)
    hx, hy, hz = (h[:, d][:, None, None, None] for d in range(3))
    u = _blocks(u_all, n)
    # contractions along z (last index), then y, then x, with the physical
    # factors M_d = h_d M_hat and P_d = P_hat / h_d
    t = np.einsum("kc,bijc->bijk", M, u) * hz
    w = np.einsum("kc,bijc->bijk", P, u) / hz
    a = np.einsum("jc,bick->bijk", M, t) * hy
    c = np.einsum("jc,bick->bijk", P, t) / hy + np.einsum("jc,bick->bijk", M, w) * hy
    v = np.einsum("ic,bcjk->bijk", P, a) / hx + np.einsum("ic,bcjk->bijk", M, c) * hx
    return v.reshape(u.shape[0], n ** 3)


def eigenpairs(p: int, op: str = dense.CELL, C: float = 2.0):
    """(S_hat, lambda_hat): P_hat S = M_hat S diag(lambda), S^T M_hat S = I (LAPACK)."""
    M, P = dense.reference_pair(p, op, C)
    lam, S = scipy.linalg.eigh(0.5 * (P + P.T), M)
    return S, lam


def inverse(p: int, h_all, r_all, op: str = dense.CELL, C: float = 2.0) -> np.ndarray:
    """x_b = D_b^{-1} r_b by fast diagonalization (Sec. 5.2): six 1D
    contractions and the scaling by the reciprocal eigenvalue sums."""
    n = p + 1
    S, lam = eigenpairs(p, op, C)
    h = np.asarray(h_all, dtype=np.float64).reshape(-1, 3)
    r = _blocks(r_all, n)
    sx, sy, sz = (1.0 / np.sqrt(h[:, d])[:, None, None, None] for d in range(3))
    # y = (S_x (x) S_y (x) S_z)^T r
    y = np.einsum("ck,bijc->bijk", S, r) * sz
    y = np.einsum("cj,bick->bijk", S, y) * sy
    y = np.einsum("ci,bcjk->bijk", S, y) * sx
    lx = lam[None, :] / h[:, 0:1] ** 2
    ly = lam[None, :] / h[:, 1:2] ** 2
    lz = lam[None, :] / h[:, 2:3] ** 2
    y = y / (lx[:, :, None, None] + ly[:, None, :, None] + lz[:, None, None, :])
    # x = (S_x (x) S_y (x) S_z) y
    x = np.einsum("ic,bcjk->bijk", S, y) * sx
    x = np.einsum("jc,bick->bijk", S, x) * sy
    x = np.einsum("kc,bijc->bijk", S, x) * sz
    return x.reshape(r.shape[0], n ** 3)
