"""Geometric multigrid for the coupled SIPG operator on uniform box meshes:
Chebyshev-accelerated block-Jacobi smoothing, level transfers by polynomial
embedding, a dense coarse solve, and CG preconditioned by one V-cycle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed:

* Sec. 5.2 (block-Jacobi smoother): the cell blocks of eq. (cell_block) with
  the interior stencil on every cell (``sipg.block_jacobi``).
* Sec. 5.2, eq. (chebyshev_weights) and eq. (chebyshev_richardson): one
  smoothing application is three Richardson updates
  u <- u + omega_j D^{-1} (b - A u) with omega_j = 1 / (c - d cos((2j-1) pi / 6)),
  c = (a+b)/2, d = (b-a)/2, on the interval [a, b] = [0.2, 2] of Sec. 6.1.
* Sec. 5 (level transfers): on uniform refinement a coarse cell's polynomial
  is embedded into its 2^3 children (prolongation); restriction is the
  transpose.
* Sec. 6.1: one pre- and one post-smoothing application per level, the
  coarsest level solved exactly by a dense factorization, CG preconditioned
  by one V-cycle.

Levels of an m-cell-per-side unit cube: m, m/2, ... while even; the
coarsest has the odd part of m cells per side (1 for powers of two).  Every
level is rediscretized with its own cell size (and penalty).

Optional degree-coarsened coarsest level (``coarse_degree``; a reading, not
the paper's configuration, whose meshes halve down to one cell): one more
level on the coarsest cells with the polynomial degree lowered to
``coarse_degree``, reached by the cellwise embedding E of Q_pc into Q_p
(Sec. 5's level transfers with the degree in place of the cell size), with
the Galerkin operator E^T A E.  For nested spaces with exact quadrature this
is the degree-pc SIPG form with the fine level's penalty C p (p+1) / h, which
the pins check.
Pins (tests/test_oracle_mg.py): the Chebyshev error polynomial of
eq. (chebyshev_error_polynomial) in closed form, exact prolongation of
polynomials, P^T M_fine P = M_coarse, the smoother's error propagator, the
V-cycle's symmetry, and CG iteration counts in the range the paper reports.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import basis, hermite, sipg

INTERVAL = (0.2, 2.0)


def chebyshev_weights(a: float = INTERVAL[0], b: float = INTERVAL[1], degree: int = 3):
    """omega_j = 1 / (c - d cos((2j-1) pi / (2 degree))), j = 1..degree."""
    c = 0.5 * (a + b)
    d = 0.5 * (b - a)
    return [1.0 / (c - d * math.cos((2 * j - 1) * math.pi / (2 * degree))) for j in range(1, degree + 1)]


def levels(m):
    """Cells of every level, finest first: m (an int for a cube, or the
    three counts of a box), halved in every direction while all counts are
    even."""
    if np.isscalar(m):
        out = [int(m)]
        while out[-1] % 2 == 0:
            out.append(out[-1] // 2)
        return out
    out = [tuple(int(v) for v in m)]
    while all(v % 2 == 0 for v in out[-1]):
        out.append(tuple(v // 2 for v in out[-1]))
    return out


def prolongation_1d(p: int, bname: str = sipg.LAGRANGE):
    """(P_0, P_1): P_c[i, j] = l_j((x_i + c) / 2), the coarse basis function j
    at node i of child c (left c = 0, right c = 1) in the parent's
    coordinates; in the Hermite-type basis the child's coefficients of the
    same function."""
    if bname == sipg.HERMITE:
        return hermite.prolongation_1d(p)
    x = basis.gll_nodes(p)
    return tuple(basis.lagrange_values(x, (x + c) / 2.0) for c in (0, 1))


def prolongation(p: int, mc, bname: str = sipg.LAGRANGE) -> sp.csr_matrix:
    """Fine (2 mc cells per direction) <- coarse (mc) embedding, canonical
    orders; mc an int for a cube or the three counts of a box."""
    mc = (int(mc),) * 3 if np.isscalar(mc) else tuple(int(v) for v in mc)
    n3 = (p + 1) ** 3
    P1 = prolongation_1d(p, bname)
    mf = tuple(2 * v for v in mc)
    rows, cols, vals = [], [], []
    li = np.repeat(np.arange(n3), n3)
    lj = np.tile(np.arange(n3), n3)
    for f in range(mf[0] * mf[1] * mf[2]):
        fx, fy, fz = sipg.cell_coords(mf, f)
        c = sipg.cell_index(mc, fx // 2, fy // 2, fz // 2)
        blk = np.kron(np.kron(P1[fx % 2], P1[fy % 2]), P1[fz % 2])
        rows.append(f * n3 + li)
        cols.append(c * n3 + lj)
        vals.append(blk.reshape(-1))
    N = mf[0] * mf[1] * mf[2] * n3
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, mc[0] * mc[1] * mc[2] * n3)).tocsr()


def degree_embedding_1d(p: int, pc: int) -> np.ndarray:
    """E[i, j] = l^pc_j(x^p_i): the degree-pc Lagrange function j (Gauss-Lobatto
    nodes of [0, 1]) at node i of the degree-p basis; E c holds the degree-p
    nodal values of the degree-pc polynomial with nodal values c."""
    return basis.lagrange_values(basis.gll_nodes(pc), basis.gll_nodes(p))


def degree_embedding(p: int, pc: int, cells) -> sp.csr_matrix:
    """Cellwise embedding of Q_pc into Q_p on the same cells (canonical
    orders): block diagonal, each block the Kronecker cube of the 1D one."""
    E1 = degree_embedding_1d(p, pc)
    blk = sp.csr_matrix(np.kron(np.kron(E1, E1), E1))
    ncell = int(np.prod(cells))
    return sp.block_diag([blk] * ncell, format="csr")


class Hierarchy:
    """Level operators, transfers and the coarse inverse of a unit cube with
    m cells per side, or of a box with cells m = (mx, my, mz) of lengths h
    (each level doubles the lengths).  With coarse_degree (Lagrange basis,
    1 <= coarse_degree < p) one more level of that degree on the coarsest
    cells, with the Galerkin operator E^T A E, is the one solved exactly."""

    def __init__(self, p: int, m, C: float = 2.0, bname: str = sipg.LAGRANGE, h=None, coarse_degree=None):
        self.p = p
        self.bname = bname
        self.ms = levels(m)
        box = not np.isscalar(m)
        self.cells = [ml if box else (ml,) * 3 for ml in self.ms]
        if box:
            h0 = tuple(float(v) for v in h)
            self.hs = [tuple(v * 2 ** k for v in h0) for k in range(len(self.ms))]
        else:
            self.hs = [(1.0 / ml,) * 3 for ml in self.ms]
        self.A = [sipg.assemble(p, c, hl, sipg.FULL, C, bname) for c, hl in zip(self.cells, self.hs)]
        self.P = [prolongation(p, self.ms[k + 1], bname) for k in range(len(self.ms) - 1)]
        self.degrees = [p] * len(self.ms)
        if coarse_degree is not None:
            if bname != sipg.LAGRANGE or not 1 <= coarse_degree < p:
                raise ValueError("coarse_degree needs the Lagrange basis and 1 <= coarse_degree < p")
            E = degree_embedding(p, coarse_degree, self.cells[-1])
            self.ms.append(self.ms[-1])
            self.cells.append(self.cells[-1])
            self.hs.append(self.hs[-1])
            self.A.append((E.T @ self.A[-1] @ E).tocsr())
            self.P.append(E)
            self.degrees.append(coarse_degree)
        self.coarse = np.linalg.inv(self.A[-1].toarray())
        self.omega = chebyshev_weights()
        self.C = C

    def smooth(self, k: int, u, b):
        """One Chebyshev application (three Richardson updates) on level k."""
        for w in self.omega:
            u = u + w * sipg.block_jacobi(self.p, self.cells[k], self.hs[k], b - self.A[k] @ u, self.C, self.bname)
        return u

    def vcycle(self, b, k: int = 0):
        """Approximate A_k^{-1} b by one V-cycle from level k (0 = finest)."""
        if k == len(self.ms) - 1:
            return self.coarse @ b
        u = self.smooth(k, np.zeros_like(b), b)
        r = b - self.A[k] @ u
        u = u + self.P[k] @ self.vcycle(self.P[k].T @ r, k + 1)
        return self.smooth(k, u, b)


def mg_pcg(p: int, m: int, b, rtol: float, maxit: int = 200, bname: str = sipg.LAGRANGE,
           criterion: str = "residual"):
    """CG on the finest level preconditioned by one V-cycle; returns
    (x, iterations, relative residual)."""
    H = Hierarchy(p, m, bname=bname)
    return sipg.pcg(H.A[0], b, H.vcycle, rtol, maxit, criterion=criterion)
