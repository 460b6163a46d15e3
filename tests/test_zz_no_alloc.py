"""tp_solve_static (the solve entry point that allocates nothing) against
tp_solve: the same kernels write their partial summaries to the library's
static device workspace instead of the plan's, so iterates, iteration counts
and summaries must be identical bit for bit.  Two calls in a row, the second
on a smaller plan (the workspace keeps the previous call's contents), a
persistent plan, and the rejection of a plan whose solve may need more
partial summaries than the workspace holds."""
import numpy as np
import pytest

from paper_2609_04534_amd import tpfdm, workloads
from tests.gpu_util import canon, from_blocked, to_blocked

pytestmark = pytest.mark.gpu


def _solve_both(wl, inner, persistent=False):
    import torch
    out = {}
    with tpfdm.Plan(tpfdm.groups_for_workload(wl), persistent=persistent) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bb = to_blocked(plan, canon([g.b for g in wl.groups]), tpfdm.F64)
        for static in (False, True):
            bx = torch.zeros_like(bb)
            iters = torch.full((plan.nblocks,), -1, dtype=torch.int32, device="cuda")
            relres = torch.full((plan.nblocks,), -1.0, dtype=torch.float64, device="cuda")
            s = plan.solve(bb, bx, inner=inner, rtol=1e-10, maxit=30, iters=iters, relres=relres, static=static)
            out[static] = (from_blocked(plan, bx, tpfdm.F64), iters.cpu().numpy(), relres.cpu().numpy(), s)
    return out


def _check_same(out):
    a, b = out[False], out[True]
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
    assert a[3] == b[3]
    assert a[3]["status"] == "TP_OK" and a[3]["n_failed"] == 0


@pytest.mark.parametrize("inner", [tpfdm.F64, tpfdm.F32])
def test_static_solve_equals_plan_solve_twice_smaller_second(inner):
    big = workloads.mixed_degree_workload("static_big", 3000, (2, 3, 7), (0.5, 2.0), seed=51, with_rhs=True)
    small = workloads.mixed_degree_workload("static_small", 200, (1, 3), (0.5, 2.0), seed=52, with_rhs=True)
    first = _solve_both(big, inner)
    _check_same(first)
    second = _solve_both(small, inner)
    _check_same(second)
    print("summaries", first[True][3], second[True][3])


def test_static_solve_persistent_plan():
    wl = workloads.mixed_degree_workload("static_persistent", 1500, (2, 3, 7), (0.5, 2.0), seed=53, with_rhs=True)
    _check_same(_solve_both(wl, tpfdm.F32, persistent=True))


def test_static_solve_rejects_plans_beyond_its_workspace():
    import torch
    # three groups of 131072 blocks of n = 2: up to 8192 solve workgroups each
    groups = [tpfdm.GroupSpec(2, 64, np.full((131072, 3), 0.5), -1) for _ in range(3)]
    with tpfdm.Plan(groups) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bb = torch.ones(plan.vector_elems, dtype=torch.float64, device="cuda")
        bx = torch.full_like(bb, 7.0)
        with pytest.raises(tpfdm.TpfdmError) as e:
            plan.solve(bb, bx, inner=tpfdm.F64, static=True)
        assert e.value.status == -1 and "static workspace" in str(e.value)
        torch.cuda.synchronize()
        assert bool(torch.all(bx == 7.0))          # nothing was launched
        s = plan.solve(bb, bx, inner=tpfdm.F64)   # the plan's own workspace still serves it
        assert s["n_failed"] == 0
