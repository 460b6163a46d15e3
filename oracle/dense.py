"""Dense per-block operators: plain definitions, no sum factorization.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed:

* Sec. 3.1, eq. (eval_pipeline): on a Cartesian cell the volume operator is
  the Kronecker sum K (x) M (x) M + M (x) K (x) M + M (x) M (x) K, with 1D
  factors scaled by the cell size.  For an axis-aligned box with edge
  lengths (h_x, h_y, h_z) the factors are M_d = h_d M_hat and K_d = K_hat/h_d;
  for a cube this is the h^{d-2} prefactor of the equation.
* Sec. 5.2, eq. (cell_block): the cell block D_K has the same Kronecker-sum
  form with K replaced by A_hat = stiffness + own-side face blocks, scaled
  as A_d = A_hat / h_d.  It is symmetric positive definite.
* Sec. 2 (blocked storage): a block's DoFs are indexed (i_x, i_y, i_z); here
  the canonical flat index is q = (i_x n + i_y) n + i_z, so x is the slowest
  index and the first Kronecker slot acts on x.

apply  = dense matrix-vector product with the n^3 x n^3 matrix.
solve  = LAPACK dense solve followed by refinement steps whose residual is
         formed in numpy long double (80-bit on x86), so the result is the
         exact solution up to a few FP64 ulps even at condition numbers ~1e3.

Pins: A 1 = 0 for the Neumann block; symmetry and definiteness; the energy
u^T A u of interpolated polynomials equals the exact Dirichlet integral on an
anisotropic box; isotropic scaling A(h) = h A(1); the generalized eigenvalues
of (D, M (x) M (x) M) are the sums of the 1D ones; brute-force 3D/2D
quadrature assembly of the volume and face integrals with an independently
built basis; the long-double residual of the solve.
"""
from __future__ import annotations

import numpy as np

from . import basis

NEUMANN = "neumann"     # 1D factor K: pure stiffness, the volume operator
CELL = "cell"           # 1D factor A_hat: the SIPG cell block of eq. (cell_block)


def reference_pair(p: int, op: str, C: float = 2.0):
    """(M_hat, P_hat) with P_hat = K_hat (Neumann) or A_hat (cell block)."""
    M, K = basis.mass_stiffness(p)
    if op == NEUMANN:
        return M, K
    if op == CELL:
        return M, basis.penalized_stiffness(p, C)
    raise ValueError(f"unknown operator {op!r}")


def direction_factors(p: int, h, op: str, C: float = 2.0):
    """Per-direction physical 1D factors [(M_x, P_x), (M_y, P_y), (M_z, P_z)]."""
    M, P = reference_pair(p, op, C)
    return [(float(hd) * M, P / float(hd)) for hd in h]


def kronecker_sum(pairs) -> np.ndarray:
    """P_x(x)M_y(x)M_z + M_x(x)P_y(x)M_z + M_x(x)M_y(x)P_z for explicit
    per-direction pairs [(M_x, P_x), (M_y, P_y), (M_z, P_z)] (the form of
    eq. (eval_pipeline) and eq. (cell_block) with per-cell factors)."""
    (Mx, Px), (My, Py), (Mz, Pz) = pairs
    return (np.kron(np.kron(Px, My), Mz)
            + np.kron(np.kron(Mx, Py), Mz)
            + np.kron(np.kron(Mx, My), Pz))


def dense_operator(p: int, h, op: str = NEUMANN, C: float = 2.0) -> np.ndarray:
    """The n^3 x n^3 block matrix P_x(x)M_y(x)M_z + M_x(x)P_y(x)M_z + M_x(x)M_y(x)P_z."""
    return kronecker_sum(direction_factors(p, h, op, C))


def dense_mass(p: int, h) -> np.ndarray:
    """M_x (x) M_y (x) M_z, the block mass matrix."""
    M, _ = basis.mass_stiffness(p)
    return np.kron(np.kron(h[0] * M, h[1] * M), h[2] * M)


def apply(p: int, h_all, u_all, op: str = NEUMANN, C: float = 2.0) -> np.ndarray:
    """v_b = A_b u_b for every block b; u_all is (nblocks, n^3), h_all is (nblocks, 3)."""
    h_all = np.asarray(h_all, dtype=np.float64).reshape(-1, 3)
    u_all = np.asarray(u_all, dtype=np.float64)
    out = np.empty_like(u_all)
    for b in range(u_all.shape[0]):
        out[b] = dense_operator(p, h_all[b], op, C) @ u_all[b]
    return out


def solve_block(D: np.ndarray, r: np.ndarray, refine: int = 2) -> np.ndarray:
    """x with D x = r: LAPACK solve, then ``refine`` steps of iterative
    refinement with the residual r - D x accumulated in long double."""
    x = np.linalg.solve(D, r)
    if refine:
        D_ld = D.astype(np.longdouble)
        r_ld = np.asarray(r).astype(np.longdouble)
        for _ in range(refine):
            res = r_ld - D_ld @ x.astype(np.longdouble)
            x = x + np.linalg.solve(D, res.astype(np.float64))
    return x


def solve(p: int, h_all, r_all, op: str = CELL, C: float = 2.0, refine: int = 2) -> np.ndarray:
    """x_b = D_b^{-1} r_b for every block (dense solve, the plain definition of
    the cell-block inverse of Sec. 5.2)."""
    h_all = np.asarray(h_all, dtype=np.float64).reshape(-1, 3)
    r_all = np.asarray(r_all, dtype=np.float64)
    out = np.empty_like(r_all)
    for b in range(r_all.shape[0]):
        out[b] = solve_block(dense_operator(p, h_all[b], op, C), r_all[b], refine)
    return out


def condition_number(p: int, h, op: str = CELL, C: float = 2.0) -> float:
    """2-norm condition number of the dense block matrix."""
    return float(np.linalg.cond(dense_operator(p, h, op, C)))


def apply_factors(M_all, P_all, u_all) -> np.ndarray:
    """v_b = A_b u_b with explicit per-block, per-direction factors:
    M_all and P_all are (nblocks, 3, n, n), u_all is (nblocks, n^3)."""
    u_all = np.asarray(u_all, dtype=np.float64)
    out = np.empty_like(u_all)
    for b in range(u_all.shape[0]):
        pairs = [(np.asarray(M_all[b][d], dtype=np.float64), np.asarray(P_all[b][d], dtype=np.float64))
                 for d in range(3)]
        out[b] = kronecker_sum(pairs) @ u_all[b]
    return out


def solve_factors(M_all, P_all, r_all, refine: int = 2) -> np.ndarray:
    """x_b = A_b^{-1} r_b with explicit per-block factors (dense solve)."""
    r_all = np.asarray(r_all, dtype=np.float64)
    out = np.empty_like(r_all)
    for b in range(r_all.shape[0]):
        pairs = [(np.asarray(M_all[b][d], dtype=np.float64), np.asarray(P_all[b][d], dtype=np.float64))
                 for d in range(3)]
        out[b] = solve_block(kronecker_sum(pairs), r_all[b], refine)
    return out


# --------------------------------------------------------------------------
# Whole-batch forms of the same dense operators, for checks at full size.
#
# For a block of lengths (h_x, h_y, h_z) every term of the Kronecker sum is a
# scalar multiple of a reference term, e.g.
#   kron(P_hat/h_x, h_y M_hat, h_z M_hat) = (h_y h_z / h_x) kron(P_hat, M_hat, M_hat),
# so the dense n^3 x n^3 block matrix is s_x T_x + s_y T_y + s_z T_z with the
# three reference Kronecker products T_d (eq. (eval_pipeline), eq. (cell_block))
# and s_x = h_y h_z / h_x, s_y = h_x h_z / h_y, s_z = h_x h_y / h_z.  These
# functions form exactly that matrix (never a sum-factorized or diagonalized
# form); only the per-block scalars are pulled out of the products.

def reference_terms(p: int, op: str, C: float = 2.0):
    """(T_x, T_y, T_z) = kron(P,M,M), kron(M,P,M), kron(M,M,P) of the reference pair."""
    M, P = reference_pair(p, op, C)
    return (np.kron(np.kron(P, M), M), np.kron(np.kron(M, P), M), np.kron(np.kron(M, M), P))


def term_scales(h_all) -> np.ndarray:
    """(nblocks, 3) array of (s_x, s_y, s_z) for lengths (nblocks, 3)."""
    h = np.asarray(h_all, dtype=np.float64).reshape(-1, 3)
    hx, hy, hz = h[:, 0], h[:, 1], h[:, 2]
    return np.stack([hy * hz / hx, hx * hz / hy, hx * hy / hz], axis=1)


def apply_batch(p: int, h_all, u_all, op: str = NEUMANN, C: float = 2.0, absolute: bool = False) -> np.ndarray:
    """v_b = A_b u_b for every block as three dense products over the whole
    batch.  With absolute=True the entries of every T_d are replaced by their
    absolute values (|A_b| u_b, a scale for error bounds)."""
    T = reference_terms(p, op, C)
    if absolute:
        T = tuple(np.abs(t) for t in T)
    s = term_scales(h_all)
    u = np.asarray(u_all, dtype=np.float64)
    return s[:, 0:1] * (u @ T[0].T) + s[:, 1:2] * (u @ T[1].T) + s[:, 2:3] * (u @ T[2].T)


def residual_batch(p: int, h_all, x_all, r_all, op: str = CELL, C: float = 2.0) -> np.ndarray:
    """r_b - D_b x_b for every block (FP64 dense products)."""
    return np.asarray(r_all, dtype=np.float64) - apply_batch(p, h_all, x_all, op, C)


def solve_batch(p: int, h_all, r_all, op: str = CELL, C: float = 2.0, refine: int = 2,
                chunk: int = 64) -> np.ndarray:
    """x_b = D_b^{-1} r_b for every block: the dense matrices of a chunk of
    blocks, a batched LAPACK solve, and ``refine`` refinement steps with the
    residual accumulated in long double (as ``solve_block``).  r_all may be
    (nblocks, n^3) or (nblocks, n^3, k) for k right-hand sides per block."""
    T = reference_terms(p, op, C)
    s = term_scales(h_all)
    r_all = np.asarray(r_all, dtype=np.float64)
    multi = r_all.ndim == 3
    R = r_all if multi else r_all[:, :, None]
    out = np.empty_like(R)
    T_ld = tuple(t.astype(np.longdouble) for t in T)
    for c0 in range(0, R.shape[0], chunk):
        c1 = min(R.shape[0], c0 + chunk)
        sc = s[c0:c1]
        D = (sc[:, 0, None, None] * T[0] + sc[:, 1, None, None] * T[1] + sc[:, 2, None, None] * T[2])
        x = np.linalg.solve(D, R[c0:c1])
        if refine:
            D_ld = (sc[:, 0, None, None].astype(np.longdouble) * T_ld[0]
                    + sc[:, 1, None, None].astype(np.longdouble) * T_ld[1]
                    + sc[:, 2, None, None].astype(np.longdouble) * T_ld[2])
            r_ld = R[c0:c1].astype(np.longdouble)
            for _ in range(refine):
                res = r_ld - np.matmul(D_ld, x.astype(np.longdouble))
                x = x + np.linalg.solve(D, res.astype(np.float64))
        out[c0:c1] = x
    return out if multi else out[:, :, 0]
