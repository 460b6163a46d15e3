"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Tolerances (per block, ||y - y*||_2 / ||y*||_2, max over blocks):
  FP64 apply and inverse: 1e-12.
  Mixed forms, against the FP64 oracle on the FP64 input (so the input's
  rounding to the storage type is included): derived from unit roundoff u of
  the storage type times the growth of the contraction chain (three 1D
  contractions per Kronecker term, a few u each, with margin):
      FP32  apply 2e-6,  inverse 5e-6
      FP16  apply 5e-3,  inverse 2e-2
      BF16  apply 4e-2,  inverse 1e-1
"""
import numpy as np
import pytest

from oracle import dense
from paper_2609_04534_amd import tpfdm, workloads

from .gpu_util import canon, from_blocked, gpu_apply, gpu_inverse, rel_err_blocks, split, to_blocked

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
TOL_APPLY = {tpfdm.F32: 2e-6, tpfdm.F16: 5e-3, tpfdm.BF16: 4e-2}
TOL_INV = {tpfdm.F32: 5e-6, tpfdm.F16: 2e-2, tpfdm.BF16: 1e-1}


def _torch():
    import torch
    return torch


def make_plan(wl, layout_B=None, **kw):
    return tpfdm.Plan(tpfdm.groups_for_workload(wl, layout_B), **kw)


def oracle_apply(wl, op=dense.NEUMANN, which=None):
    out = []
    for g in wl.groups:
        u = g.u if which is None else which(g)
        out.append(dense.apply(g.p, g.h, u, op))
    return out


CASES = [(p, nb) for p in (1, 2, 3, 4, 5, 6, 7) for nb in (1, 63, 65, 130)]


# ------------------------------------------------------------------ layout
@pytest.mark.parametrize("dt", [tpfdm.F64, tpfdm.F32, tpfdm.F16, tpfdm.BF16])
@pytest.mark.parametrize("p,B", [(2, 64), (3, 1), (3, 8), (7, 1), (7, 16), (1, 1024)])
def test_pack_unpack_roundtrip_bit_exact(dt, p, B):
    torch = _torch()
    wl = workloads.random_blocks(p, 77, seed=5)
    with make_plan(wl, B) as plan:
        flat = canon([g.u for g in wl.groups])
        cu = torch.from_numpy(flat).cuda().to(
            {tpfdm.F64: torch.float64, tpfdm.F32: torch.float32, tpfdm.F16: torch.float16,
             tpfdm.BF16: torch.bfloat16}[dt])
        bu = torch.full((plan.vector_elems,), 7.0, dtype=cu.dtype, device="cuda")
        plan.pack(cu, bu)
        back = torch.empty_like(cu)
        plan.unpack(bu, back)
        torch.cuda.synchronize()
        assert torch.equal(back.view(torch.int16 if cu.element_size() == 2 else
                                     (torch.int32 if cu.element_size() == 4 else torch.int64)),
                           cu.view(torch.int16 if cu.element_size() == 2 else
                                   (torch.int32 if cu.element_size() == 4 else torch.int64)))
        # padding lanes are zero after pack
        n3 = (p + 1) ** 3
        tiles = (77 + B - 1) // B
        blk = bu[:tiles * n3 * B].view(tiles, n3, B)
        if tiles * B > 77:
            assert torch.all(blk[-1, :, 77 - (tiles - 1) * B:] == 0)


# ------------------------------------------------------------------ FP64 apply
@pytest.mark.parametrize("op", [tpfdm.OP_NEUMANN, tpfdm.OP_CELL])
@pytest.mark.parametrize("p,nb", CASES)
def test_apply_f64_matches_oracle(p, nb, op):
    wl = workloads.random_blocks(p, nb, seed=100 + p * 7 + nb)
    with make_plan(wl) as plan:
        got, _ = gpu_apply(plan, canon([g.u for g in wl.groups]), tpfdm.F64, op)
    ref = oracle_apply(wl, dense.NEUMANN if op == tpfdm.OP_NEUMANN else dense.CELL)
    assert rel_err_blocks(split(got, wl.groups)[0], ref[0]) < F64_TOL


@pytest.mark.parametrize("p,B", [(2, 1), (2, 8), (3, 16), (3, 1024), (4, 1), (7, 8), (5, 64)])
def test_apply_f64_any_layout(p, B):
    wl = workloads.random_blocks(p, 70, seed=9)
    with make_plan(wl, B) as plan:
        got, _ = gpu_apply(plan, canon([g.u for g in wl.groups]))
    assert rel_err_blocks(split(got, wl.groups)[0], oracle_apply(wl)[0]) < F64_TOL


@pytest.mark.parametrize("p", [2, 3, 7])
def test_apply_never_writes_padding(p):
    torch = _torch()
    wl = workloads.random_blocks(p, 70, seed=4)
    B = 64
    with make_plan(wl, B) as plan:
        _, bv = gpu_apply(plan, canon([g.u for g in wl.groups]), sentinel=True)
        torch.cuda.synchronize()
        n3 = (p + 1) ** 3
        blk = bv.view(-1, n3, B)
        assert torch.all(torch.isnan(blk[-1, :, 70 - 64:]))
        assert not torch.any(torch.isnan(blk[0]))


@pytest.mark.parametrize("p", [1, 2, 3, 7])
def test_neumann_annihilates_constants(p):
    wl = workloads.random_blocks(p, 65, seed=2)
    with make_plan(wl) as plan:
        ones = np.ones(plan.ndof)
        got, _ = gpu_apply(plan, ones)
        u = np.random.default_rng(1).uniform(-1, 1, plan.ndof)
        ref, _ = gpu_apply(plan, u)
    scale = np.abs(ref).max()
    assert np.abs(got).max() < 1e-13 * scale


@pytest.mark.parametrize("p", [2, 3, 7])
@pytest.mark.parametrize("op", [tpfdm.OP_NEUMANN, tpfdm.OP_CELL])
def test_symmetry_on_gpu_outputs(p, op):
    wl = workloads.random_blocks(p, 40, seed=3)
    rng = np.random.default_rng(7)
    with make_plan(wl) as plan:
        u = rng.uniform(-1, 1, plan.ndof)
        w = rng.uniform(-1, 1, plan.ndof)
        Au, _ = gpu_apply(plan, u, op=op)
        Aw, _ = gpu_apply(plan, w, op=op)
    n3 = (p + 1) ** 3
    lhs = (w.reshape(-1, n3) * Au.reshape(-1, n3)).sum(1)
    rhs = (u.reshape(-1, n3) * Aw.reshape(-1, n3)).sum(1)
    scale = np.abs(w.reshape(-1, n3)) @ np.ones(n3) * np.abs(Au.reshape(-1, n3)).max(1)
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-13


# ------------------------------------------------------------------ FP64 inverse
@pytest.mark.parametrize("p,nb", CASES)
def test_inverse_f64_matches_dense_solve(p, nb):
    wl = workloads.random_blocks(p, nb, seed=200 + p * 5 + nb, h_range=(0.5, 4.0))
    with make_plan(wl) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        got, _ = gpu_inverse(plan, canon([g.u for g in wl.groups]))
    g = wl.groups[0]
    ref = dense.solve(g.p, g.h, g.u)
    assert rel_err_blocks(split(got, wl.groups)[0], ref) < F64_TOL


@pytest.mark.parametrize("p", [1, 2, 3, 4, 7])
def test_apply_of_inverse_is_identity(p):
    """D (D^{-1} r) = r with both factors computed on the GPU (A A^{-1} = I)."""
    torch = _torch()
    wl = workloads.random_blocks(p, 65, seed=31, h_range=(0.5, 4.0))
    with make_plan(wl) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        r = canon([g.u for g in wl.groups])
        br = to_blocked(plan, r, tpfdm.F64)
        bx = torch.empty_like(br)
        by = torch.empty_like(br)
        plan.apply_inverse(br, bx)
        plan.apply(bx, by, tpfdm.OP_CELL)
        y = from_blocked(plan, by, tpfdm.F64)
    n3 = (p + 1) ** 3
    assert rel_err_blocks(y.reshape(-1, n3), r.reshape(-1, n3)) < 1e-12


@pytest.mark.parametrize("p", [2, 3, 7])
def test_inverse_of_unit_vectors(p):
    """Every column of D^{-1}: r = e_j for all j in one batch of blocks."""
    n3 = (p + 1) ** 3
    h = np.tile([[0.6, 1.7, 0.9]], (n3, 1))
    E = np.eye(n3)
    with tpfdm.Plan([tpfdm.GroupSpec(p + 1, tpfdm.default_layout_B(p + 1), h)]) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        X, _ = gpu_inverse(plan, E.reshape(-1))
    D = dense.dense_operator(p, h[0], dense.CELL)
    assert np.abs(X.reshape(n3, n3) @ D.T - E).max() < 1e-12


# ------------------------------------------------------------------ errors
def test_inverse_requires_setup_and_rejects_neumann():
    torch = _torch()
    wl = workloads.random_blocks(3, 10, seed=1)
    with make_plan(wl) as plan:
        buf = torch.zeros(plan.vector_elems, dtype=torch.float64, device="cuda")
        out = torch.zeros_like(buf)
        with pytest.raises(tpfdm.TpfdmError) as e:
            plan.apply_inverse(buf, out)
        assert e.value.status == -9
        with pytest.raises(tpfdm.TpfdmError) as e:
            plan.setup_inverse(tpfdm.OP_NEUMANN)
        assert e.value.status == -4
        with pytest.raises(tpfdm.TpfdmError) as e:
            plan.apply(buf, buf)
        assert e.value.status == -1


def test_h_validation_on_device_input():
    torch = _torch()
    h = torch.ones((5, 3), dtype=torch.float64, device="cuda")
    h[2, 1] = 0.0
    with pytest.raises(tpfdm.TpfdmError) as e:
        tpfdm.Plan([tpfdm.GroupSpec(3, 64, h)])
    assert e.value.status == -1
    h[2, 1] = float("inf")
    with pytest.raises(tpfdm.TpfdmError):
        tpfdm.Plan([tpfdm.GroupSpec(3, 64, h)])


def test_empty_group_and_empty_plan():
    torch = _torch()
    with tpfdm.Plan([tpfdm.GroupSpec(3, 64, np.zeros((0, 3)))]) as plan:
        assert plan.vector_elems == 0 and plan.ndof == 0
        plan.setup_inverse()
        buf = torch.zeros(1, dtype=torch.float64, device="cuda")
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        plan.apply(buf, out)
        plan.apply_inverse(buf, out)
        torch.cuda.synchronize()
    with tpfdm.Plan([]) as plan:
        assert plan.vector_elems == 0


# ------------------------------------------------------------------ invariance
@pytest.mark.parametrize("p", [2, 3, 7])
def test_block_result_independent_of_batch(p):
    """A block's output is bitwise the same alone and inside a batch, at any
    position, and for any layout B (no cross-block arithmetic)."""
    torch = _torch()
    wl = workloads.random_blocks(p, 130, seed=77)
    g = wl.groups[0]
    with make_plan(wl) as plan:
        plan.setup_inverse()
        full_a, _ = gpu_apply(plan, canon([g.u]))
        full_i, _ = gpu_inverse(plan, canon([g.u]))
    n3 = (p + 1) ** 3
    for pick in (0, 64, 129):
        solo = workloads.Group(p=p, h=g.h[pick:pick + 1], u=g.u[pick:pick + 1],
                               block_ids=np.array([0]))
        for B in (1, 64):
            with tpfdm.Plan([tpfdm.GroupSpec(p + 1, B, solo.h)]) as plan:
                plan.setup_inverse()
                a, _ = gpu_apply(plan, solo.u.reshape(-1))
                i, _ = gpu_inverse(plan, solo.u.reshape(-1))
            assert np.array_equal(a, full_a.reshape(-1, n3)[pick])
            assert np.array_equal(i, full_i.reshape(-1, n3)[pick])


def test_repeat_runs_bitwise_identical():
    wl = workloads.random_blocks(3, 300, seed=8)
    with make_plan(wl) as plan:
        plan.setup_inverse()
        a1, _ = gpu_apply(plan, canon([wl.groups[0].u]))
        a2, _ = gpu_apply(plan, canon([wl.groups[0].u]))
        i1, _ = gpu_inverse(plan, canon([wl.groups[0].u]))
        i2, _ = gpu_inverse(plan, canon([wl.groups[0].u]))
    assert np.array_equal(a1, a2) and np.array_equal(i1, i2)


# ------------------------------------------------------------------ mixed precision
@pytest.mark.parametrize("dt", [tpfdm.F32, tpfdm.F16, tpfdm.BF16])
@pytest.mark.parametrize("p", [2, 3, 7])
def test_low_precision_error_vs_f64_oracle(dt, p):
    wl = workloads.random_blocks(p, 65, seed=300 + p, h_range=(0.5, 4.0))
    g = wl.groups[0]
    with make_plan(wl) as plan:
        plan.setup_inverse()
        a, _ = gpu_apply(plan, canon([g.u]), dt, tpfdm.OP_NEUMANN)
        i, _ = gpu_inverse(plan, canon([g.u]), dt)
    ea = rel_err_blocks(split(a, wl.groups)[0], dense.apply(p, g.h, g.u, dense.NEUMANN))
    ei = rel_err_blocks(split(i, wl.groups)[0], dense.solve(p, g.h, g.u))
    print(f"dtype={tpfdm.DTYPE_NAMES[dt]} p={p} apply_err={ea:.3e} inverse_err={ei:.3e}")
    assert ea < TOL_APPLY[dt]
    assert ei < TOL_INV[dt]


# ------------------------------------------------------------------ solve
# iteration caps per inner precision: the inner FDM is exact up to its own
# rounding, so each correction gains about -log10(kappa * u) digits
# (kappa <= 6e2 for h ~ U[0.5, 4]; u = 2^-24, 2^-11, 2^-8)
SOLVE_MAXIT = {tpfdm.F64: 2, tpfdm.F32: 4, tpfdm.F16: 10, tpfdm.BF16: 16}
SOLVE_CASES = ([(inner, p, tpfdm.MAP_AUTO, None) for inner in (tpfdm.F64, tpfdm.F32, tpfdm.F16, tpfdm.BF16)
                for p in (1, 2, 3, 4, 7)]
               + [(inner, p, tpfdm.MAP_LANE, None) for inner in (tpfdm.F64, tpfdm.F32, tpfdm.F16, tpfdm.BF16)
                  for p in (1, 2, 3)]
               + [(inner, p, tpfdm.MAP_WAVE, None) for inner in (tpfdm.F64, tpfdm.F32, tpfdm.BF16) for p in (1, 2, 3)]
               + [(tpfdm.F32, 3, tpfdm.MAP_LANE, 8), (tpfdm.F64, 2, tpfdm.MAP_LANE, 1)])


@pytest.mark.parametrize("inner,p,mapping,layout_B", SOLVE_CASES)
def test_solve_matches_dense_solve(inner, p, mapping, layout_B):
    torch = _torch()
    wl = workloads.random_blocks(p, 65, seed=400 + p, h_range=(0.5, 4.0), with_rhs=True)
    g = wl.groups[0]
    with make_plan(wl, layout_B, mapping=mapping) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bb = to_blocked(plan, canon([g.b]), tpfdm.F64)
        bx = torch.zeros_like(bb)
        iters = torch.full((plan.nblocks,), -1, dtype=torch.int32, device="cuda")
        relres = torch.full((plan.nblocks,), -1.0, dtype=torch.float64, device="cuda")
        s = plan.solve(bb, bx, inner=inner, rtol=1e-10, maxit=30, iters=iters, relres=relres)
        x = from_blocked(plan, bx, tpfdm.F64)
        it = iters.cpu().numpy()
        rr = relres.cpu().numpy()
    ref = dense.solve(p, g.h, g.b)
    print(f"inner={tpfdm.DTYPE_NAMES[inner]} p={p} mapping={mapping} B={layout_B} summary={s}")
    assert s["n_failed"] == 0 and s["max_relres"] <= 1e-10
    assert np.all(rr <= 1e-10) and np.all(it >= 1) and np.all(it <= SOLVE_MAXIT[inner])
    assert s["max_iters"] == it.max()
    # forward error bounded by condition number times the residual tolerance
    kappa = max(dense.condition_number(p, h) for h in g.h[:5])
    assert rel_err_blocks(split(x, wl.groups)[0], ref) < 1e-10 * kappa * 4


@pytest.mark.parametrize("mapping", [tpfdm.MAP_AUTO, tpfdm.MAP_LANE, tpfdm.MAP_WAVE])
def test_solve_zero_rhs_and_initial_guess(mapping):
    torch = _torch()
    wl = workloads.random_blocks(3, 70, seed=12, with_rhs=True)
    g = wl.groups[0]
    b = g.b.copy()
    b[5] = 0.0
    with make_plan(wl, mapping=mapping) as plan:
        plan.setup_inverse()
        bb = to_blocked(plan, canon([b]), tpfdm.F64)
        # start from the exact solution for block 7: zero iterations there
        x0 = np.zeros_like(b)
        x0[7] = dense.solve(3, g.h[7:8], b[7:8])[0]
        x0[5] = 1.0    # nonzero guess for the b = 0 block must become 0
        bx = to_blocked(plan, canon([x0]), tpfdm.F64)
        iters = torch.zeros(plan.nblocks, dtype=torch.int32, device="cuda")
        plan.solve(bb, bx, inner=tpfdm.F32, rtol=1e-10, maxit=20, iters=iters)
        x = from_blocked(plan, bx, tpfdm.F64).reshape(70, -1)
        it = iters.cpu().numpy()
    assert np.all(x[5] == 0.0) and it[5] == 0
    assert it[7] == 0


def test_solve_maxit_reports_not_converged():
    torch = _torch()
    wl = workloads.random_blocks(7, 8, seed=13, h_range=(0.5, 4.0), with_rhs=True)
    with make_plan(wl) as plan:
        plan.setup_inverse()
        bb = to_blocked(plan, canon([wl.groups[0].b]), tpfdm.F64)
        bx = torch.zeros_like(bb)
        s = plan.solve(bb, bx, inner=tpfdm.F32, rtol=1e-14, maxit=1, raise_on_failure=False)
        assert s["status"] == "TP_ERR_NOT_CONVERGED" and s["n_failed"] == 8 and s["max_iters"] == 1
        with pytest.raises(tpfdm.TpfdmError) as e:
            plan.solve(bb, bx, inner=tpfdm.F32, rtol=1e-14, maxit=1)
        assert e.value.status == -5


def test_solve_summaries_of_consecutive_calls():
    """Each call's summary is its own: calls whose outcomes differ alternate,
    and every returned summary equals the expected outcome and the summary
    read back from the plan's device copy."""
    torch = _torch()
    wl = workloads.random_blocks(7, 8, seed=13, h_range=(0.5, 4.0), with_rhs=True)
    with make_plan(wl) as plan:
        plan.setup_inverse()
        bb = to_blocked(plan, canon([wl.groups[0].b]), tpfdm.F64)
        bx = torch.zeros_like(bb)
        for k in range(12):
            bx.zero_()
            if k % 2 == 0:
                s = plan.solve(bb, bx, inner=tpfdm.F32, rtol=1e-14, maxit=1, raise_on_failure=False)
                assert s["status"] == "TP_ERR_NOT_CONVERGED" and s["n_failed"] == 8 and s["max_iters"] == 1
            else:
                s = plan.solve(bb, bx, inner=tpfdm.F32, rtol=1e-10, maxit=20)
                assert s["status"] == "TP_OK" and s["n_failed"] == 0 and s["max_iters"] >= 2
                assert s["max_relres"] <= 1e-10
            d = plan.solve_summary()
            assert (d["max_iters"], d["n_failed"], d["max_relres"]) == (s["max_iters"], s["n_failed"],
                                                                       s["max_relres"])


def test_solve_nonfinite_rhs_is_reported():
    torch = _torch()
    wl = workloads.random_blocks(3, 10, seed=14, with_rhs=True)
    b = wl.groups[0].b.copy()
    b[3, 5] = float("nan")
    with make_plan(wl) as plan:
        plan.setup_inverse()
        bb = to_blocked(plan, canon([b]), tpfdm.F64)
        bx = torch.zeros_like(bb)
        s = plan.solve(bb, bx, inner=tpfdm.F32, rtol=1e-10, maxit=5, raise_on_failure=False)
    assert s["status"] == "TP_ERR_NONFINITE"


def test_solve_requires_cell_setup():
    torch = _torch()
    wl = workloads.random_blocks(3, 10, seed=15, with_rhs=True)
    with make_plan(wl) as plan:
        buf = torch.zeros(plan.vector_elems, dtype=torch.float64, device="cuda")
        with pytest.raises(tpfdm.TpfdmError) as e:
            plan.solve(buf, torch.zeros_like(buf))
        assert e.value.status == -9


# ------------------------------------------------------------------ persistent + graphs
MIXED_DEGREES = (1, 2, 3, 4, 5, 6, 7)


def _mixed(nblocks=700, seed=21):
    return workloads.mixed_degree_workload("mixed_test", nblocks, MIXED_DEGREES, (0.5, 2.0), seed=seed,
                                           with_rhs=True)


@pytest.mark.parametrize("dt", [tpfdm.F64, tpfdm.F32, tpfdm.F16, tpfdm.BF16])
def test_persistent_equals_per_group_launches(dt):
    """One persistent launch over all degrees gives bitwise the per-group results."""
    wl = _mixed()
    flat = canon([g.u for g in wl.groups])
    outs = {}
    for persistent in (False, True):
        with make_plan(wl, persistent=persistent) as plan:
            plan.setup_inverse()
            a, _ = gpu_apply(plan, flat, dt, tpfdm.OP_NEUMANN)
            c, _ = gpu_apply(plan, flat, dt, tpfdm.OP_CELL)
            i, _ = gpu_inverse(plan, flat, dt)
            outs[persistent] = (a, c, i)
    for k in range(3):
        assert np.array_equal(outs[False][k], outs[True][k]), k


def test_persistent_mixed_matches_oracle():
    wl = _mixed(nblocks=300, seed=22)
    with make_plan(wl, persistent=True) as plan:
        plan.setup_inverse()
        flat = canon([g.u for g in wl.groups])
        a, _ = gpu_apply(plan, flat, tpfdm.F64, tpfdm.OP_NEUMANN)
        i, _ = gpu_inverse(plan, flat, tpfdm.F64)
    for g, ga, gi in zip(wl.groups, split(a, wl.groups), split(i, wl.groups)):
        assert rel_err_blocks(ga, dense.apply(g.p, g.h, g.u, dense.NEUMANN)) < F64_TOL
        assert rel_err_blocks(gi, dense.solve(g.p, g.h, g.u)) < F64_TOL


@pytest.mark.parametrize("inner,mapping", [(tpfdm.F64, tpfdm.MAP_AUTO), (tpfdm.F32, tpfdm.MAP_AUTO),
                                           (tpfdm.F64, tpfdm.MAP_LANE), (tpfdm.F16, tpfdm.MAP_LANE)])
def test_persistent_solve_mixed(inner, mapping):
    torch = _torch()
    wl = _mixed(nblocks=300, seed=23)
    res = {}
    for persistent in (False, True):
        with make_plan(wl, persistent=persistent, mapping=mapping) as plan:
            plan.setup_inverse()
            bb = to_blocked(plan, canon([g.b for g in wl.groups]), tpfdm.F64)
            bx = torch.zeros_like(bb)
            iters = torch.zeros(plan.nblocks, dtype=torch.int32, device="cuda")
            s = plan.solve(bb, bx, inner=inner, rtol=1e-10, maxit=30, iters=iters)
            res[persistent] = (from_blocked(plan, bx, tpfdm.F64), iters.cpu().numpy(), s)
    if mapping != tpfdm.MAP_LANE:  # the single launch solves on wave tiles, as AUTO does for these sizes
        assert np.array_equal(res[False][0], res[True][0])
        assert np.array_equal(res[False][1], res[True][1])
    assert res[True][2]["n_failed"] == 0 and res[False][2]["n_failed"] == 0
    for g, gx in zip(wl.groups, split(res[True][0], wl.groups)):
        ref = dense.solve(g.p, g.h, g.b)
        kappa = max(dense.condition_number(g.p, h) for h in g.h[:3])
        assert rel_err_blocks(gx, ref) < 4e-10 * kappa


@pytest.mark.parametrize("persistent", [False, True])
def test_graph_replay_matches_eager(persistent):
    """Captured apply / inverse / solve graphs replayed several times, with
    eager work and synchronisations in between, reproduce the eager results
    bitwise on every replay."""
    torch = _torch()
    wl = _mixed(nblocks=400, seed=24)
    with make_plan(wl, persistent=persistent) as plan:
        plan.setup_inverse()
        bu = to_blocked(plan, canon([g.u for g in wl.groups]), tpfdm.F32)
        bb = to_blocked(plan, canon([g.b for g in wl.groups]), tpfdm.F64)
        ref_v = torch.empty_like(bu)
        ref_x = torch.empty_like(bu)
        ref_s = torch.zeros_like(bb)
        plan.apply(bu, ref_v, tpfdm.OP_NEUMANN)
        plan.apply_inverse(bu, ref_x)
        plan.solve(bb, ref_s, inner=tpfdm.F32, rtol=1e-10, maxit=30)
        torch.cuda.synchronize()
        gv, gx, gs = torch.empty_like(bu), torch.empty_like(bu), torch.zeros_like(bb)
        graphs = [plan.graph(tpfdm.GRAPH_APPLY, bu, gv, op=tpfdm.OP_NEUMANN),
                  plan.graph(tpfdm.GRAPH_INVERSE, bu, gx),
                  plan.graph(tpfdm.GRAPH_SOLVE, bb, gs, dtype=tpfdm.F32, rtol=1e-10, maxit=30)]
        for rep in range(4):
            gv.fill_(float("nan"))
            gx.fill_(float("nan"))
            gs.zero_()
            scratch = torch.empty_like(bu)
            plan.apply(bu, scratch, tpfdm.OP_CELL)      # eager work between replays
            torch.cuda.synchronize()
            for g in graphs:
                g.launch()
            torch.cuda.synchronize()
            # compare the blocks' entries (padding lanes are never written)
            for got, ref, dt in ((gv, ref_v, tpfdm.F32), (gx, ref_x, tpfdm.F32), (gs, ref_s, tpfdm.F64)):
                assert np.array_equal(from_blocked(plan, got, dt), from_blocked(plan, ref, dt)), rep
            summ = plan.solve_summary()
            assert summ["n_failed"] == 0 and summ["max_iters"] >= 1
        for g in graphs:
            g.destroy()


# ------------------------------------------------------------------ MFMA (n = 8, FP16 / BF16)
@pytest.mark.parametrize("dt", [tpfdm.F16, tpfdm.BF16])
@pytest.mark.parametrize("nb", [1, 2, 63, 130])
def test_mfma_path_matches_oracle(dt, nb):
    """The matrix-core path (n = 8, 16-bit storage, B = 1) against the FP64
    oracle, for odd and even block counts (tiles hold two blocks)."""
    wl = workloads.random_blocks(7, nb, seed=500 + nb, h_range=(0.5, 4.0))
    g = wl.groups[0]
    with make_plan(wl) as plan:
        plan.setup_inverse()
        a, _ = gpu_apply(plan, canon([g.u]), dt, tpfdm.OP_NEUMANN)
        c, _ = gpu_apply(plan, canon([g.u]), dt, tpfdm.OP_CELL)
        i, _ = gpu_inverse(plan, canon([g.u]), dt)
    ea = rel_err_blocks(a.reshape(nb, -1), dense.apply(7, g.h, g.u, dense.NEUMANN))
    ec = rel_err_blocks(c.reshape(nb, -1), dense.apply(7, g.h, g.u, dense.CELL))
    ei = rel_err_blocks(i.reshape(nb, -1), dense.solve(7, g.h, g.u))
    print(f"MFMA dtype={tpfdm.DTYPE_NAMES[dt]} nb={nb} apply {ea:.2e} cell {ec:.2e} inverse {ei:.2e}")
    assert ea < TOL_APPLY[dt] and ec < TOL_APPLY[dt] and ei < TOL_INV[dt]


@pytest.mark.parametrize("dt", [tpfdm.F16, tpfdm.BF16])
def test_mfma_and_vector_paths_agree(dt):
    """MFMA and the even-odd vector path (mapping = WAVE) compute the same
    operator; their difference stays within the storage precision bound."""
    wl = workloads.random_blocks(7, 40, seed=77, h_range=(0.5, 4.0))
    flat = canon([wl.groups[0].u])
    res = {}
    for mapping in (tpfdm.MAP_AUTO, tpfdm.MAP_WAVE):
        with make_plan(wl, mapping=mapping) as plan:
            plan.setup_inverse()
            res[mapping] = (gpu_apply(plan, flat, dt)[0], gpu_inverse(plan, flat, dt)[0])
    for k, tol in ((0, TOL_APPLY[dt]), (1, TOL_INV[dt])):
        got, ref = res[tpfdm.MAP_AUTO][k].reshape(40, -1), res[tpfdm.MAP_WAVE][k].reshape(40, -1)
        assert rel_err_blocks(got, ref) < 2 * tol


# ------------------------------------------------------------------ autotuning
@pytest.mark.parametrize("dt", [tpfdm.F64, tpfdm.F32, tpfdm.F16])
def test_autotune_then_calls_match_oracle(dt):
    """The kernel chosen per group by tp_plan_autotune computes the same
    operators (checked against the oracle after tuning)."""
    torch = _torch()
    wl = _mixed(nblocks=400, seed=31)
    with make_plan(wl) as plan:
        plan.setup_inverse()
        times = plan.autotune(dt, reps=3)
        assert len(times) == len(wl.groups)
        for gi, g in enumerate(wl.groups):
            if g.nblocks:
                assert times[gi][0] > 0 and times[gi][1] > 0
                assert plan.kernel(gi, 0, dt) in ("lane", "wave", "mfma")
                assert plan.kernel(gi, 2) in ("lane", "wave")
        print("choices", [(g.p, plan.kernel(i, 0, dt), plan.kernel(i, 1, dt), plan.kernel(i, 2)) for i, g in
                          enumerate(wl.groups)], "times", times)
        a, _ = gpu_apply(plan, canon([g.u for g in wl.groups]), dt)
        i, _ = gpu_inverse(plan, canon([g.u for g in wl.groups]), dt)
        bb = to_blocked(plan, canon([g.b for g in wl.groups]), tpfdm.F64)
        bx = torch.zeros_like(bb)
        s = plan.solve(bb, bx, inner=tpfdm.F32, rtol=1e-10, maxit=30)
        x = from_blocked(plan, bx, tpfdm.F64)
    ta = F64_TOL if dt == tpfdm.F64 else TOL_APPLY[dt]
    ti = F64_TOL if dt == tpfdm.F64 else TOL_INV[dt]
    for gx, gv, gs, g in zip(split(a, wl.groups), split(i, wl.groups), split(x, wl.groups), wl.groups):
        if not g.nblocks:
            continue
        scale = np.abs(dense.apply(g.p, g.h, np.abs(g.u), dense.NEUMANN)).max(axis=1, keepdims=True)
        assert np.max(np.abs(gx - dense.apply(g.p, g.h, g.u, dense.NEUMANN)) / scale) < ta
        assert rel_err_blocks(gv, dense.solve(g.p, g.h, g.u)) < ti
        assert rel_err_blocks(gs, dense.solve(g.p, g.h, g.b)) < 1e-8
    assert s["n_failed"] == 0


def test_default_kernel_choices_and_persistent_autotune():
    wl = _mixed(nblocks=200, seed=32)
    with make_plan(wl) as plan:
        for gi, g in enumerate(wl.groups):
            want = "lane" if g.p <= 3 else "wave"
            assert plan.kernel(gi, 0, tpfdm.F64) == want
    # MFMA for n = 8 in FP16 when the group starts 16-byte aligned (offset 0 here)
    with make_plan(workloads.random_blocks(7, 10, seed=33)) as plan:
        assert plan.kernel(0, 0, tpfdm.F16) == "mfma" and plan.kernel(0, 0, tpfdm.F64) == "wave"
    with make_plan(wl, persistent=True) as plan:
        # defaults of the single launch: the lane body for n <= 4 in apply and
        # inverse, wave tiles in the solve, one tile per workgroup, groups in order
        for gi, g in enumerate(wl.groups):
            c = plan.launch_config(gi, 0, tpfdm.F32)
            assert c == {"body": "lane" if g.n <= 4 else "wave", "tiles_per_workgroup": 1, "position": gi}
            c = plan.launch_config(gi, 2, tpfdm.F32)
            assert c["body"] == "wave" and c["grid"] == "full" and c["position"] == gi
