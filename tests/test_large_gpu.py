"""Vectors of more than 2^31 elements: every offset in the kernels is 64-bit.

A plan whose vectors hold more than 2^31 values (17 GB in FP64) is applied
and inverted on the lane (p = 3, layout B = 64), wave (p = 7, B = 1) and
matrix-core (p = 7, FP16) paths.  Checked over every element on the GPU:
the Neumann operator annihilates constants (A 1 = 0), and the cell-block
inverse undoes the cell-block operator (D^{-1} D u = u); blocks beyond the
2^31-th element are compared with the dense oracle on the host.
"""
import numpy as np
import pytest

from oracle import dense
from paper_2609_04534_amd import tpfdm

pytestmark = pytest.mark.gpu

LIMIT = 2 ** 31


def _torch():
    import torch
    return torch


def _plan(p, B, nblocks, seed):
    h = np.random.default_rng(seed).uniform(0.5, 2.0, (nblocks, 3))
    plan = tpfdm.Plan([tpfdm.GroupSpec(p + 1, B, h)])
    plan.setup_inverse(tpfdm.OP_CELL)
    return plan, h


def _block_values(vec, B, n3, g):
    """Host copy of block g of a vector in layout [tile][n^3][B]."""
    torch = _torch()
    t, lane = divmod(g, B)
    idx = torch.arange(n3, device=vec.device, dtype=torch.int64) * B + (t * n3 * B + lane)
    return vec[idx].double().cpu().numpy()


def _valid_parts(vec, B, n3, nblocks):
    """The elements of real blocks: every full tile, then the valid lanes of a
    ragged last tile (its padding lanes are never written)."""
    full = nblocks // B
    parts = [vec[: full * n3 * B]]
    if nblocks % B:
        parts.append(vec[full * n3 * B: (full + 1) * n3 * B].view(n3, B)[:, : nblocks % B])
    return parts


def _max_abs(parts):
    return max(float(p.abs().max()) for p in parts)


# (degree, layout B, storage, sampled-block tolerance of apply, of inverse)
CASES = [(3, 64, tpfdm.F64, 1e-12, 1e-11), (7, 1, tpfdm.F64, 1e-12, 1e-11), (7, 1, tpfdm.F16, 1e-2, 8e-2)]


@pytest.mark.parametrize("p,B,dt,tol_apply,tol_inv", CASES)
def test_vectors_beyond_2_31_elements(p, B, dt, tol_apply, tol_inv):
    torch = _torch()
    n3 = (p + 1) ** 3
    tdt = {tpfdm.F64: torch.float64, tpfdm.F16: torch.float16}[dt]
    nblocks = LIMIT // n3 + 3 * B + 5      # past 2^31 elements, ragged last tile
    plan, h = _plan(p, B, nblocks, seed=p)
    E = plan.vector_elems
    assert E > LIMIT
    print(f"p={p} B={B} dtype={tpfdm.DTYPE_NAMES[dt]} nblocks={nblocks} elems={E}", flush=True)
    try:
        gen = torch.Generator(device="cuda").manual_seed(5)
        u = (torch.rand(E, dtype=torch.float32, device="cuda", generator=gen) * 2 - 1).to(tdt)
        v = torch.full_like(u, float("nan"))
        x = torch.full_like(u, float("nan"))
        err_const = None
        if dt == tpfdm.F64:
            # A 1 = 0 for the Neumann operator, in every element of every block
            plan.apply(torch.ones_like(u), v, tpfdm.OP_NEUMANN)
            torch.cuda.synchronize()
            err_const = _max_abs([torch.nan_to_num(q, nan=1e30) for q in _valid_parts(v, B, n3, nblocks)])
            v.fill_(float("nan"))
        plan.apply(u, v, tpfdm.OP_CELL)
        plan.apply_inverse(v, x)
        torch.cuda.synchronize()
        # every element of every block written and finite
        for q in _valid_parts(v, B, n3, nblocks) + _valid_parts(x, B, n3, nblocks):
            assert bool(torch.isfinite(q).all())
        if err_const is not None:
            scale = _max_abs(_valid_parts(v, B, n3, nblocks))
            print(f"  max |A 1| = {err_const:.2e} (max |D u| = {scale:.2e})", flush=True)
            assert err_const <= 1e-13 * scale
        if dt == tpfdm.F64:
            # D^{-1} D u = u over every element of every block
            diffs = [a - b for a, b in zip(_valid_parts(x, B, n3, nblocks), _valid_parts(u, B, n3, nblocks))]
            err = _max_abs(diffs) / _max_abs(_valid_parts(u, B, n3, nblocks))
            del diffs
            print(f"  max |D^-1 D u - u| / max |u| = {err:.2e}", flush=True)
            assert err <= 1e-12
            # the block-local solve of D x = D u from x = 0, FP64 inner
            x.zero_()
            summ = plan.solve(v, x, inner=tpfdm.F64, rtol=1e-10, maxit=10)
            diffs = [a - b for a, b in zip(_valid_parts(x, B, n3, nblocks), _valid_parts(u, B, n3, nblocks))]
            err = _max_abs(diffs) / _max_abs(_valid_parts(u, B, n3, nblocks))
            del diffs
            print(f"  solve {summ}, max |x - u| / max |u| = {err:.2e}", flush=True)
            assert summ["n_failed"] == 0 and summ["max_relres"] <= 1e-10 and err <= 1e-9
        # blocks whose elements lie past 2^31 against the dense oracle
        for g in (nblocks - 1, nblocks - B - 1, LIMIT // n3 + 1):
            ub = _block_values(u, B, n3, g)
            vb = _block_values(v, B, n3, g)
            xb = _block_values(x, B, n3, g)
            ref_v = dense.apply_batch(p, h[g:g + 1], ub[None, :], dense.CELL)[0]
            ref_x = dense.solve_batch(p, h[g:g + 1], vb[None, :])[0]
            ev = np.linalg.norm(vb - ref_v) / np.linalg.norm(ref_v)
            ex = np.linalg.norm(xb - ref_x) / np.linalg.norm(ref_x)
            print(f"  block {g}: apply {ev:.2e}, inverse {ex:.2e} (rel. 2-norm vs dense)", flush=True)
            assert ev <= tol_apply and ex <= tol_inv
    finally:
        plan.destroy()
        torch.cuda.empty_cache()


@pytest.mark.parametrize("p,cells,basis", [(3, (320, 322, 328), tpfdm.BASIS_LAGRANGE),
                                           (3, (320, 322, 328), tpfdm.BASIS_HERMITE),
                                           (7, (160, 162, 164), tpfdm.BASIS_LAGRANGE)])
def test_sipg_operator_beyond_2_31_elements(p, cells, basis):
    """The coupled operator on a mesh whose vectors exceed 2^31 elements:
    rows of sampled cells (corners, faces, interior, the last cells) against
    the oracle's row blocks of the same cells, their neighbours' blocks read
    back from the GPU."""
    from oracle import sipg
    torch = _torch()
    n = p + 1
    n3 = n ** 3
    h = tuple(1.0 / c for c in cells)
    ncell = cells[0] * cells[1] * cells[2]
    bname = sipg.HERMITE if basis == tpfdm.BASIS_HERMITE else sipg.LAGRANGE
    with tpfdm.Plan.mesh(n, cells, h, basis=basis) as plan:
        E = plan.vector_elems
        assert E > LIMIT
        B = tpfdm.default_layout_B(n)
        print(f"p={p} cells={cells} basis={bname} elems={E}", flush=True)
        gen = torch.Generator(device="cuda").manual_seed(7)
        u = torch.rand(E, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1
        v = torch.full_like(u, float("nan"))
        plan.apply(u, v, tpfdm.OP_SIPG)
        torch.cuda.synchronize()
        for q in _valid_parts(v, B, n3, ncell):
            assert bool(torch.isfinite(q).all())
        mx, my, mz = cells
        sample = {sipg.cell_index(cells, a, b_, c) for a in (0, mx - 1) for b_ in (0, my - 1) for c in (0, mz - 1)}
        sample |= {ncell - 1, ncell - 2, ncell - mz, sipg.cell_index(cells, mx - 1, my // 2, mz // 2),
                   LIMIT // n3 + 7}
        worst = 0.0
        for c in sorted(sample):
            row = np.zeros(n3)
            scale = np.zeros(n3)
            for nb, blk in sipg.cell_row_blocks(p, cells, h, int(c), sipg.FULL, 2.0, bname):
                ub = _block_values(u, B, n3, nb)
                row += blk @ ub
                scale += np.abs(blk) @ np.abs(ub)
            got = _block_values(v, B, n3, int(c))
            worst = max(worst, float(np.max(np.abs(got - row) / np.max(scale))))
        print(f"  {len(sample)} sampled rows: max error / row scale {worst:.2e}", flush=True)
        assert worst <= 1e-13
        del u, v
    torch.cuda.empty_cache()
