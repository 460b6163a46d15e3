"""GPU parity of vertex-patch blocks (plans with TP_BLOCKS_PATCHES): each
block is the 2 x 2 x 2 cells of degree p around a vertex, n = 2(p+1) points
per direction, served by the same kernels as cell blocks of that n.  Apply
(patch operator and broken volume operator), the exact patch inverse (FDM,
SCALED and GENERAL) and the block-local solve against the oracle's patch
blocks, which are pinned to the assembled mesh operator."""
import numpy as np
import pytest

from oracle import dense, patch
from paper_2609_04534_amd import tpfdm

from .gpu_util import from_blocked, rel_err_blocks, to_blocked

pytestmark = pytest.mark.gpu

TOL_APPLY = {tpfdm.F64: 1e-12, tpfdm.F32: 2e-6, tpfdm.F16: 5e-3}


def _torch():
    import torch
    return torch


def _patches(p, nb, seed):
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.5, 2.0, (nb, 3))
    u = rng.uniform(-1, 1, (nb, (2 * (p + 1)) ** 3))
    return h, u


def _plan(p, h, B=None, **kw):
    n = 2 * (p + 1)
    g = tpfdm.GroupSpec(n, tpfdm.default_layout_B(n) if B is None else B, h)
    return tpfdm.Plan([g], blocks=tpfdm.BLOCKS_PATCHES, **kw)


def _ref(p, h, u, op, inverse=False):
    out = np.empty_like(u)
    for b in range(len(h)):
        D = patch.patch_operator(p, h[b], op)
        out[b] = dense.solve_block(D, u[b]) if inverse else D @ u[b]
    return out


CASES = [(1, 130, None), (2, 65, None), (3, 63, None), (3, 20, 4), (2, 70, 64)]


@pytest.mark.parametrize("p,nb,B", CASES)
@pytest.mark.parametrize("op", [tpfdm.OP_CELL, tpfdm.OP_NEUMANN])
def test_patch_apply_matches_oracle(p, nb, B, op):
    torch = _torch()
    h, u = _patches(p, nb, 10 * p + nb)
    dop = dense.CELL if op == tpfdm.OP_CELL else dense.NEUMANN
    ref = _ref(p, h, u, dop)
    print(f"p={p} nb={nb} B={B} op={op}", flush=True)
    with _plan(p, h, B) as plan:
        bu = to_blocked(plan, u.reshape(-1), tpfdm.F64)
        bv = torch.full_like(bu, float("nan"))
        plan.apply(bu, bv, op)
        got = from_blocked(plan, bv, tpfdm.F64).reshape(nb, -1)
    if op == tpfdm.OP_NEUMANN:
        # near-null outputs on constants: absolute error against |A||u|
        scale = max(np.abs(r).max() for r in ref) + 1e-300
        assert np.abs(got - ref).max() <= 1e-12 * max(scale, np.abs(u).max() * 10)
    else:
        assert rel_err_blocks(got, ref) < TOL_APPLY[tpfdm.F64]


@pytest.mark.parametrize("dt", [tpfdm.F32, tpfdm.F16])
def test_patch_apply_low_precision(dt):
    """p = 3 patches (n = 8): the FP32 wave kernel and the FP16 MFMA kernel."""
    torch = _torch()
    p, nb = 3, 70
    h, u = _patches(p, nb, 5)
    ref = _ref(p, h, u, dense.CELL)
    with _plan(p, h) as plan:
        bu = to_blocked(plan, u.reshape(-1), dt)
        bv = torch.empty_like(bu)
        plan.apply(bu, bv, tpfdm.OP_CELL)
        got = from_blocked(plan, bv, dt).reshape(nb, -1)
    err = rel_err_blocks(got, ref)
    print(f"dt={tpfdm.DTYPE_NAMES[dt]} err={err:.2e}")
    assert err < TOL_APPLY[dt]


@pytest.mark.parametrize("p,nb", [(1, 130), (2, 65), (3, 63)])
@pytest.mark.parametrize("mode", [None, "general"])
def test_patch_inverse_is_the_exact_local_solve(p, nb, mode):
    """apply_inverse on patch blocks: the patch problem solved exactly (fast
    diagonalization of the patch factors), against a dense solve."""
    torch = _torch()
    h, r = _patches(p, nb, 100 + p)
    ref = _ref(p, h, r, dense.CELL, inverse=True)
    with _plan(p, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL, mode=tpfdm.FACTOR_GENERAL if mode else None)
        br = to_blocked(plan, r.reshape(-1), tpfdm.F64)
        bx = torch.full_like(br, float("nan"))
        plan.apply_inverse(br, bx)
        got = from_blocked(plan, bx, tpfdm.F64).reshape(nb, -1)
    err = rel_err_blocks(got, ref)
    cond = max(np.linalg.cond(patch.patch_operator(p, h[b], dense.CELL)) for b in range(3))
    print(f"p={p} mode={mode} err={err:.2e} cond~{cond:.1e}")
    assert err < 1e-12 * max(1.0, cond / 100)


def test_patch_solve_and_persistent_mixed_degrees():
    """The block-local solve on patches (FP32 inner), and one persistent
    plan over patch groups of every degree."""
    torch = _torch()
    specs, data = [], []
    for p, nb in ((1, 40), (2, 33), (3, 17)):
        h, b = _patches(p, nb, 300 + p)
        n = 2 * (p + 1)
        specs.append(tpfdm.GroupSpec(n, tpfdm.default_layout_B(n), h))
        data.append((p, h, b))
    flat = np.concatenate([b.reshape(-1) for _, _, b in data])
    for persistent in (False, True):
        with tpfdm.Plan(specs, blocks=tpfdm.BLOCKS_PATCHES, persistent=persistent) as plan:
            plan.setup_inverse(tpfdm.OP_CELL)
            bb = to_blocked(plan, flat, tpfdm.F64)
            bx = torch.zeros_like(bb)
            plan.solve(bb, bx, inner=tpfdm.F32, rtol=1e-11, maxit=20)
            x = from_blocked(plan, bx, tpfdm.F64)
        o = 0
        for p, h, b in data:
            k = b.size
            ref = _ref(p, h, b, dense.CELL, inverse=True)
            err = rel_err_blocks(x[o:o + k].reshape(b.shape), ref)
            print(f"persistent={persistent} p={p} err={err:.2e}")
            assert err < 1e-9
            o += k
