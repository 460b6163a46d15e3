"""GPU parity of the grouped tile order of the one-cell-per-lane mesh
kernels (Lagrange basis, x-planes of 8 MiB or more: each XCD visits its
tiles in groups of 8 carried through the x-planes).  The boxes are chosen
so that the order is active, with whole groups per row, with a narrower
last group (tiles per plane not a multiple of 8) and with a tail of
plain-order tiles past the last whole row.  The output starts as NaN, so a
tile the order skipped shows up; sampled cells (corners, edges, random)
are checked against the oracle's row blocks, and an MG-preconditioned CG
solve on a box whose finest level takes the grouped order in the operator,
the smoother and the CG operator is checked by the oracle's true residual
rows."""
import numpy as np
import pytest

from oracle import sipg
from paper_2609_04534_amd import tpfdm

from .gpu_util import from_blocked, to_blocked

pytestmark = pytest.mark.gpu

TOL = {tpfdm.F64: 1e-12, tpfdm.F32: 2e-6}


def _torch():
    import torch
    return torch


def _grouped(cells, n, dt):
    """Whether the kernels take the grouped order on this machine (mirrors the
    rule stated above: whole 64-cell tiles per plane, planes of at least
    8 MiB, at least two whole planes per XCD range)."""
    plane = cells[1] * cells[2]
    if plane % 64 or plane * n ** 3 * (8 if dt == tpfdm.F64 else 4) < 8 << 20:
        return False
    nwg = -(-cells[0] * plane // 64)
    return nwg % 8 == 0 and (nwg // 8) // (plane // 64) >= 2


def _sample(cells, rng, k=40):
    mx, my, mz = cells
    corners = [sipg.cell_index(cells, a, b, c) for a in (0, mx - 1) for b in (0, my - 1) for c in (0, mz - 1)]
    edges = [sipg.cell_index(cells, mx // 2, 0, 0), sipg.cell_index(cells, 0, my // 2, mz - 1),
             sipg.cell_index(cells, mx - 1, my - 1, mz // 3), sipg.cell_index(cells, 1, 64 % my, 63 % mz)]
    return sorted(set(corners + edges + rng.choice(mx * my * mz, k, replace=False).tolist()))


# (cells, dtype): 20 x 129 x 128 has 258 tiles per plane (32 whole groups
# of 8 and one of 2) and 129 tiles per XCD past its two whole planes
BOXES = [((16, 128, 128), tpfdm.F64), ((20, 129, 128), tpfdm.F64), ((16, 256, 128), tpfdm.F32)]


@pytest.mark.parametrize("cells,dt", BOXES)
def test_sipg_grouped_tile_order(cells, dt):
    torch = _torch()
    n, p = 4, 3
    assert _grouped(cells, n, dt)
    h = (0.05, 1.0 / cells[1], 0.75 / cells[2])
    ncell = int(np.prod(cells))
    print(f"cells={cells} dtype={tpfdm.DTYPE_NAMES[dt]}", flush=True)
    u = np.random.default_rng(ncell).uniform(-1, 1, ncell * n ** 3)
    with tpfdm.Plan.mesh(n, cells, h) as plan:
        bu = to_blocked(plan, u, dt)
        bv = torch.full_like(bu, float("nan"))
        plan.apply(bu, bv, tpfdm.OP_SIPG)
        assert not torch.isnan(bv).any().item()
        v = from_blocked(plan, bv, dt).reshape(ncell, n ** 3)
        del bu, bv
    if dt == tpfdm.F32:
        u = u.astype(np.float32).astype(np.float64)
    sample = _sample(cells, np.random.default_rng(7))
    ref = sipg.cell_apply(p, cells, h, u, sample)
    ub = np.abs(u).reshape(ncell, n ** 3)
    scale = max(float(np.max(sum(np.abs(blk) @ ub[nb] for nb, blk in sipg.cell_row_blocks(p, cells, h, c))))
                for c in sample)
    err = np.max(np.abs(v[sample] - ref)) / scale
    print(f"  sampled={len(sample)} err={err:.2e}")
    assert err < TOL[dt]


def test_mg_pcg_grouped_tile_order():
    """32 x 128 x 128 cubic cells at p = 3 (five levels down to 1 x 4 x 4):
    the finest level's operator, smoother and CG operator take the grouped
    order, the coarser ones the plain order.  The cells are cubes, as on the
    unit-cube meshes whose iteration counts bound this one (cells stretched
    4:1 took three times the iterations with this block smoother)."""
    torch = _torch()
    cells, n, p = (32, 128, 128), 4, 3
    assert _grouped(cells, n, tpfdm.F64)
    h = (1.0 / 128,) * 3
    ncell = int(np.prod(cells))
    b = np.random.default_rng(3).uniform(-1, 1, ncell * n ** 3)
    with tpfdm.Plan.mesh(n, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        with tpfdm.MG(plan) as V, tpfdm.PCG(plan) as solver:
            solver.set_multigrid(V)
            bb = to_blocked(plan, b, tpfdm.F64)
            bx = torch.full_like(bb, float("nan"))
            s = solver.solve(bb, bx, rtol=1e-8, maxit=100, check_every=4)
            x = from_blocked(plan, bx, tpfdm.F64)
            del bb, bx
    print(f"  {s}")
    assert s["converged"] and s["relres"] <= 1e-8
    assert s["iterations"] <= 16
    assert np.isfinite(x).all()
    sample = _sample(cells, np.random.default_rng(5), k=24)
    rows = b.reshape(ncell, -1)[sample] - sipg.cell_apply(p, cells, h, x, sample)
    assert np.linalg.norm(rows) <= 1e-7 * np.linalg.norm(b)
