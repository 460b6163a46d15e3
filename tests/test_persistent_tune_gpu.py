"""The autotuned single launch over blocks of uneven degree: after
tp_plan_autotune on a persistent plan, every group's output equals, bit for
bit, that of a per-group launch with the same tile body (lane or wave, as the
tuner chose), the solve gives the same iterates and iteration counts, graphs
captured after tuning replay the tuned launch, and the results match the
oracle."""
import numpy as np
import pytest

from oracle import dense
from paper_2609_04534_amd import tpfdm, workloads
from tests.gpu_util import canon, from_blocked, rel_err_blocks, split, to_blocked

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _mixed(nblocks, seed, degrees=(1, 2, 3, 4, 5, 6, 7)):
    return workloads.mixed_degree_workload("tune_test", nblocks, degrees, (0.5, 2.0), seed=seed, with_rhs=True)


def _run(plan, wl, dt):
    torch = _torch()
    bu = to_blocked(plan, canon([g.u for g in wl.groups]), dt)
    outs = []
    for call in ("neumann", "cell", "inverse"):
        bv = torch.full_like(bu, float("nan"))
        if call == "inverse":
            plan.apply_inverse(bu, bv)
        else:
            plan.apply(bu, bv, tpfdm.OP_NEUMANN if call == "neumann" else tpfdm.OP_CELL)
        outs.append(split(from_blocked(plan, bv, dt), wl.groups))
    return outs


def _single_group(g, body, dt):
    """Apply (Neumann, cell) and inverse of one group alone, per-group launch
    with the given tile body."""
    torch = _torch()
    mapping = tpfdm.MAP_LANE if body == "lane" else tpfdm.MAP_WAVE
    spec = [tpfdm.GroupSpec(g.n, tpfdm.default_layout_B(g.n), g.h, 0)]
    with tpfdm.Plan(spec, mapping=mapping) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bu = to_blocked(plan, g.u.reshape(-1), dt)
        outs = []
        for call in ("neumann", "cell", "inverse"):
            bv = torch.full_like(bu, float("nan"))
            if call == "inverse":
                plan.apply_inverse(bu, bv)
            else:
                plan.apply(bu, bv, tpfdm.OP_NEUMANN if call == "neumann" else tpfdm.OP_CELL)
            outs.append(from_blocked(plan, bv, dt).reshape(g.nblocks, -1))
    return outs


@pytest.mark.parametrize("dt", [tpfdm.F64, tpfdm.F32, tpfdm.BF16])
def test_tuned_single_launch_is_bitwise_the_per_group_launches(dt):
    wl = _mixed(1500, seed=41 + dt)
    with tpfdm.Plan(tpfdm.groups_for_workload(wl), persistent=True) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        times = plan.autotune(dt, reps=30)
        assert times[0][0] > 0 and times[0][1] > 0 and times[0][2] > 0
        cfg = [[plan.launch_config(gi, call, dt) for call in (0, 1)] for gi in range(len(wl.groups))]
        print("tuned", times[0], [(g.p, c[0], c[1]) for g, c in zip(wl.groups, cfg)], flush=True)
        assert sorted(c[0]["position"] for c in cfg) == list(range(len(wl.groups)))
        outs = _run(plan, wl, dt)
    for gi, g in enumerate(wl.groups):
        single_apply = _single_group(g, cfg[gi][0]["body"], dt)
        single_inv = _single_group(g, cfg[gi][1]["body"], dt)
        assert np.array_equal(outs[0][gi], single_apply[0]), (g.p, "neumann")
        assert np.array_equal(outs[1][gi], single_apply[1]), (g.p, "cell")
        assert np.array_equal(outs[2][gi], single_inv[2]), (g.p, "inverse")


@pytest.mark.parametrize("inner", [tpfdm.F64, tpfdm.F32])
def test_tuned_single_launch_solve(inner):
    """The tuned solve (any grid, tiles per workgroup and segment order) gives
    the per-group wave solve's iterates and counts bit for bit."""
    torch = _torch()
    wl = _mixed(900, seed=43)
    res = {}
    for persistent in (False, True):
        kw = {"persistent": True} if persistent else {"mapping": tpfdm.MAP_WAVE}
        with tpfdm.Plan(tpfdm.groups_for_workload(wl), **kw) as plan:
            plan.setup_inverse(tpfdm.OP_CELL)
            if persistent:
                plan.autotune(inner, reps=30)
                print("solve config", [plan.launch_config(gi, 2, inner) for gi in range(len(wl.groups))])
            bb = to_blocked(plan, canon([g.b for g in wl.groups]), tpfdm.F64)
            bx = torch.zeros_like(bb)
            iters = torch.zeros(plan.nblocks, dtype=torch.int32, device="cuda")
            s = plan.solve(bb, bx, inner=inner, rtol=1e-10, maxit=30, iters=iters)
            res[persistent] = (from_blocked(plan, bx, tpfdm.F64), iters.cpu().numpy(), s)
    assert np.array_equal(res[False][0], res[True][0])
    assert np.array_equal(res[False][1], res[True][1])
    assert res[True][2]["n_failed"] == 0
    assert res[True][2]["max_iters"] == res[False][2]["max_iters"]
    for g, gx in zip(wl.groups, split(res[True][0], wl.groups)):
        kappa = max(dense.condition_number(g.p, h) for h in g.h[:3])
        assert rel_err_blocks(gx, dense.solve(g.p, g.h, g.b)) < 4e-10 * kappa


def test_tuned_single_launch_matches_oracle_and_graph_replays():
    """C4's shape (degrees 2, 3, 7) in FP64: tuned results against the dense
    oracle, and a graph captured after tuning replays them bitwise."""
    torch = _torch()
    wl = _mixed(2000, seed=44, degrees=(2, 3, 7))
    with tpfdm.Plan(tpfdm.groups_for_workload(wl), persistent=True) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        plan.autotune(tpfdm.F64, reps=30)
        outs = _run(plan, wl, tpfdm.F64)
        bu = to_blocked(plan, canon([g.u for g in wl.groups]), tpfdm.F64)
        gv = torch.empty_like(bu)
        gr = plan.graph(tpfdm.GRAPH_INVERSE, bu, gv)
        for rep in range(3):
            gv.fill_(float("nan"))
            torch.cuda.synchronize()
            gr.launch()
            torch.cuda.synchronize()
            got = split(from_blocked(plan, gv, tpfdm.F64), wl.groups)
            for a, b in zip(got, outs[2]):
                assert np.array_equal(a, b), rep
        gr.destroy()
    for gi, g in enumerate(wl.groups):
        assert rel_err_blocks(outs[0][gi], dense.apply(g.p, g.h, g.u, dense.NEUMANN)) < 1e-12
        assert rel_err_blocks(outs[1][gi], dense.apply(g.p, g.h, g.u, dense.CELL)) < 1e-12
        assert rel_err_blocks(outs[2][gi], dense.solve(g.p, g.h, g.u)) < 1e-12
