"""Seeded synthetic inputs: block degrees, cell lengths and vectors.

This module only draws random numbers and arranges them; it holds none of the
method's arithmetic.  The oracle and the HIP path consume the same host arrays
it returns.

Draw order for one workload (numpy ``default_rng(seed)``, PCG64):
  1. degrees, one per block (only when the workload mixes degrees);
  2. cell edge lengths ``h`` as a (nblocks, 3) array (x, y, z), unless fixed;
  3. the vector ``u`` (and then ``b`` when a right-hand side is requested),
     all blocks in block order, each block's n^3 values in canonical order
     q = (i_x n + i_y) n + i_z.

The shapes follow the paper's workloads: uniform Cartesian meshes of
unit-cube cells at p = 3 measured from 16^3 to 128^3 cells (Sec. 6.5), plus
anisotropic boxes, degree mixes and low-precision cases that exercise the
same operators.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Group:
    """All blocks of one degree, in the order they appear in the workload."""
    p: int
    h: np.ndarray            # (nblocks, 3) float64
    u: np.ndarray            # (nblocks, n^3) float64
    block_ids: np.ndarray    # (nblocks,) int64, positions in the workload
    b: np.ndarray | None = None

    @property
    def n(self) -> int:
        return self.p + 1

    @property
    def nblocks(self) -> int:
        return int(self.h.shape[0])

    @property
    def ndof(self) -> int:
        return self.nblocks * self.n ** 3


@dataclass
class Workload:
    name: str
    groups: list = field(default_factory=list)
    description: str = ""

    @property
    def ndof(self) -> int:
        return sum(g.ndof for g in self.groups)

    @property
    def nblocks(self) -> int:
        return sum(g.nblocks for g in self.groups)


def _uniform_degree_workload(name, nblocks, p, seed, h_fixed=None, h_range=None,
                             with_rhs=False, description=""):
    rng = np.random.default_rng(seed)
    n = p + 1
    if h_fixed is not None:
        h = np.full((nblocks, 3), float(h_fixed))
    else:
        h = rng.uniform(h_range[0], h_range[1], size=(nblocks, 3))
    u = rng.uniform(-1.0, 1.0, size=(nblocks, n ** 3))
    b = rng.uniform(-1.0, 1.0, size=(nblocks, n ** 3)) if with_rhs else None
    g = Group(p=p, h=h, u=u, block_ids=np.arange(nblocks, dtype=np.int64), b=b)
    return Workload(name=name, groups=[g], description=description)


def mixed_degree_workload(name, nblocks, degrees, h_range, seed, with_rhs=False,
                          description=""):
    """Blocks whose degree is drawn uniformly from ``degrees``; one Group per degree."""
    rng = np.random.default_rng(seed)
    deg = rng.choice(np.asarray(degrees, dtype=np.int64), size=nblocks)
    h = rng.uniform(h_range[0], h_range[1], size=(nblocks, 3))
    sizes = (deg + 1) ** 3
    flat = rng.uniform(-1.0, 1.0, size=int(sizes.sum()))
    flat_b = rng.uniform(-1.0, 1.0, size=int(sizes.sum())) if with_rhs else None
    starts = np.concatenate(([0], np.cumsum(sizes)[:-1]))
    groups = []
    for p in sorted(set(int(d) for d in degrees)):
        ids = np.nonzero(deg == p)[0].astype(np.int64)
        n3 = (p + 1) ** 3
        idx = starts[ids][:, None] + np.arange(n3)[None, :]
        u = flat[idx] if len(ids) else np.zeros((0, n3))
        b = (flat_b[idx] if len(ids) else np.zeros((0, n3))) if with_rhs else None
        groups.append(Group(p=p, h=h[ids], u=u, block_ids=ids, b=b))
    return Workload(name=name, groups=groups, description=description)


def small_p2(with_rhs=False):
    """8x8x8 unit-cube cells of size 1/8, p=2, u ~ U[-1,1], seed 0."""
    return _uniform_degree_workload("p2_8cube_h1/8", 512, 2, seed=0, h_fixed=1.0 / 8,
                                    with_rhs=with_rhs,
                                    description="512 cells, p=2, h=1/8, FP64")


def large_p2(with_rhs=False):
    """128^3 cells of size 1/128, p=2, seed 0 (large enough to stream from HBM)."""
    return _uniform_degree_workload("p2_128cube", 128 ** 3, 2, seed=0, h_fixed=1.0 / 128,
                                    with_rhs=with_rhs,
                                    description="2,097,152 cells, p=2, FP64")


def affine_p3(nblocks=64 ** 3, with_rhs=False):
    """64^3 affine cells, p=3, edge lengths ~ U[0.5, 2] per cell and axis, seed 1."""
    return _uniform_degree_workload("p3_64cube_affine", nblocks, 3, seed=1,
                                    h_range=(0.5, 2.0), with_rhs=with_rhs,
                                    description=f"{nblocks} cells, p=3, h~U[0.5,2]")


def mixed_precision_p7(nblocks=32 ** 3, with_rhs=True):
    """32^3 cells, p=7, edge lengths ~ U[0.5, 4], seed 2 (b for refinement)."""
    return _uniform_degree_workload("p7_32cube_aniso", nblocks, 7, seed=2,
                                    h_range=(0.5, 4.0), with_rhs=with_rhs,
                                    description=f"{nblocks} cells, p=7, h~U[0.5,4]")


def uneven_degrees(nblocks=20000, with_rhs=True):
    """20000 independent blocks, degree ~ U{2,3,7}, h ~ U[0.5, 2], seed 3."""
    return mixed_degree_workload("uneven_p237_20000", nblocks, (2, 3, 7), (0.5, 2.0),
                                 seed=3, with_rhs=with_rhs,
                                 description=f"{nblocks} blocks, p~U{{2,3,7}}, h~U[0.5,2]")


def random_blocks(p, nblocks, seed, h_range=(0.5, 2.0), with_rhs=False):
    """Generic seeded case used by tests (ragged sizes, edge cases)."""
    return _uniform_degree_workload(f"p{p}_n{nblocks}_s{seed}", nblocks, p, seed=seed,
                                    h_range=h_range, with_rhs=with_rhs)


@dataclass
class BoxMesh:
    """A uniform Cartesian box mesh (the paper's uniformly refined unit cube
    of Sec. 6.5): cells per direction, cell lengths, degree and a vector in
    mesh order (cell c = (cx m_y + cy) m_z + cz, canonical DoFs per cell)."""
    name: str
    p: int
    cells: tuple
    h: tuple
    u: np.ndarray            # (ncells * n^3,) float64
    b: np.ndarray | None = None

    @property
    def n(self) -> int:
        return self.p + 1

    @property
    def ncells(self) -> int:
        return self.cells[0] * self.cells[1] * self.cells[2]

    @property
    def ndof(self) -> int:
        return self.ncells * self.n ** 3


def unit_cube_mesh(p: int, m: int, seed: int, with_rhs: bool = False) -> BoxMesh:
    """m^3 cells of length 1/m on the unit cube; u (and b) ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    nd = m ** 3 * (p + 1) ** 3
    u = rng.uniform(-1.0, 1.0, nd)
    b = rng.uniform(-1.0, 1.0, nd) if with_rhs else None
    return BoxMesh(f"sipg_p{p}_{m}cube", p, (m, m, m), (1.0 / m,) * 3, u, b)
