"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (default layouts and mappings, one call over the whole batch): sampled
blocks are checked one by one against the dense oracle, and the solve's
per-block residual bound is checked for every block (it holds at any size)."""
import numpy as np
import pytest

from oracle import dense
from paper_2609_04534_amd import tpfdm, workloads
from tests.gpu_util import canon, from_blocked, rel_err_blocks, split, to_blocked

pytestmark = pytest.mark.gpu

TOL_APPLY = {tpfdm.F64: 1e-12, tpfdm.F32: 2e-6, tpfdm.F16: 5e-3, tpfdm.BF16: 4e-2}
TOL_INV = {tpfdm.F64: 1e-12, tpfdm.F32: 5e-6, tpfdm.F16: 2e-2, tpfdm.BF16: 1e-1}

WORKLOADS = {
    "p2_128cube": lambda: workloads.large_p2(with_rhs=True),
    "p3_64cube_affine": lambda: workloads.affine_p3(with_rhs=True),
    "p7_32cube_aniso": lambda: workloads.mixed_precision_p7(with_rhs=True),
    "uneven_p237_20000": lambda: workloads.uneven_degrees(with_rhs=True),
}
_cache = {}


def _workload(name):
    if name not in _cache:
        _cache.clear()
        _cache[name] = WORKLOADS[name]()
    return _cache[name]


def _samples(nblocks, seed, k=40):
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(nblocks, size=min(k, nblocks), replace=False).tolist())
    idx.update({0, nblocks - 1})
    return np.array(sorted(idx))


CASES = [("p2_128cube", tpfdm.F64, False), ("p3_64cube_affine", tpfdm.F64, False),
         ("p3_64cube_affine", tpfdm.F32, False), ("p3_64cube_affine", tpfdm.F16, False),
         ("p3_64cube_affine", tpfdm.BF16, False), ("p7_32cube_aniso", tpfdm.F64, False),
         ("p7_32cube_aniso", tpfdm.F32, False), ("p7_32cube_aniso", tpfdm.F16, False),
         ("p7_32cube_aniso", tpfdm.BF16, False), ("uneven_p237_20000", tpfdm.F32, False),
         ("uneven_p237_20000", tpfdm.F32, True)]


@pytest.mark.parametrize("name,dt,persistent", CASES)
def test_fullsize_step_sampled_blocks(name, dt, persistent):
    """The bench step (apply with the Neumann operator, then apply_inverse of
    the cell block on apply's output) over the whole workload."""
    import torch
    wl = _workload(name)
    print(f"workload={name} dtype={tpfdm.DTYPE_NAMES[dt]} persistent={persistent} ndof={wl.ndof}", flush=True)
    with tpfdm.Plan(tpfdm.groups_for_workload(wl), persistent=persistent) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bu = to_blocked(plan, canon([g.u for g in wl.groups]), dt)
        bv = torch.empty_like(bu)
        bx = torch.empty_like(bu)
        plan.apply(bu, bv, tpfdm.OP_NEUMANN)
        plan.apply_inverse(bv, bx)
        v = split(from_blocked(plan, bv, dt), wl.groups)
        x = split(from_blocked(plan, bx, dt), wl.groups)
    for gi, g in enumerate(wl.groups):
        s = _samples(g.nblocks, seed=gi)
        ref_v = dense.apply(g.p, g.h[s], g.u[s], dense.NEUMANN)
        # the inverse is checked on the vector it was given (apply's output
        # as stored in dt), so the two tolerances do not compound
        ref_x = dense.solve(g.p, g.h[s], v[gi][s])
        scale = np.abs(dense.apply(g.p, g.h[s], np.abs(g.u[s]), dense.NEUMANN)).max(axis=1, keepdims=True)
        ea = float(np.max(np.abs(v[gi][s] - ref_v) / scale))
        ei = rel_err_blocks(x[gi][s], ref_x)
        print(f"  p={g.p} blocks={g.nblocks} sampled={len(s)} apply_err={ea:.2e} inverse_err={ei:.2e}")
        assert ea < TOL_APPLY[dt]
        assert ei < TOL_INV[dt] * (4 if dt != tpfdm.F64 else 1)


@pytest.mark.parametrize("name,inner", [("p3_64cube_affine", tpfdm.F32), ("p3_64cube_affine", tpfdm.F64),
                                        ("p7_32cube_aniso", tpfdm.F16), ("p2_128cube", tpfdm.F32),
                                        ("uneven_p237_20000", tpfdm.F32)])
def test_fullsize_solve(name, inner):
    import torch
    wl = _workload(name)
    print(f"workload={name} inner={tpfdm.DTYPE_NAMES[inner]} ndof={wl.ndof}", flush=True)
    with tpfdm.Plan(tpfdm.groups_for_workload(wl)) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bb = to_blocked(plan, canon([g.b for g in wl.groups]), tpfdm.F64)
        bx = torch.zeros_like(bb)
        relres = torch.full((plan.nblocks,), -1.0, dtype=torch.float64, device="cuda")
        s = plan.solve(bb, bx, inner=inner, rtol=1e-10, maxit=50, relres=relres)
        rr = relres.cpu().numpy()
        x = split(from_blocked(plan, bx, tpfdm.F64), wl.groups)
    print(f"  summary={s}")
    assert s["n_failed"] == 0 and s["max_relres"] <= 1e-10
    assert np.all((rr >= 0) & (rr <= 1e-10))      # every block, at full size
    for gi, g in enumerate(wl.groups):
        smp = _samples(g.nblocks, seed=10 + gi, k=16)
        ref = dense.solve(g.p, g.h[smp], g.b[smp])
        kappa = max(dense.condition_number(g.p, h) for h in g.h[smp[:3]])
        assert rel_err_blocks(x[gi][smp], ref) < 4e-10 * kappa
