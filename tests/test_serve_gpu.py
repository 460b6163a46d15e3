"""The serving loop (paper_2609_04534_amd/serve.py): solves admitted while
others run give the same result as alone, admission keeps within the memory
budget, and a served solve matches the oracle's direct solution."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import sipg
from paper_2609_04534_amd import serve, tpfdm

pytestmark = pytest.mark.gpu

MIX = [(2, 4), (3, 4), (2, 6), (3, 6), (3, 8), (2, 8), (7, 3)]


def _alone(req, inner, multigrid):
    import torch
    with tpfdm.Plan.mesh(req.p + 1, (req.m,) * 3, (1.0 / req.m,) * 3) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bb = torch.empty(plan.vector_elems, dtype=torch.float64, device="cuda")
        plan.pack(req.b, bb)
        bx = torch.empty_like(bb)
        mg = (tpfdm.MG(plan, serve.mg_storage(req.p, inner))
              if multigrid and serve.uses_multigrid(req.p, req.m) else None)
        with tpfdm.PCG(plan) as solver:
            solver.set_multigrid(mg)
            s = solver.solve(bb, bx, inner=inner, rtol=1e-8, maxit=20000, check_every=4 if mg else 8)
        if mg:
            mg.destroy()
        out = torch.empty(plan.ndof, dtype=torch.float64, device="cuda")
        plan.unpack(bx, out)
        torch.cuda.synchronize()
    return out.cpu().numpy(), s


@pytest.mark.parametrize("multigrid", [False, True])
@pytest.mark.parametrize("inner", [tpfdm.F64, tpfdm.F32])
def test_each_result_is_the_same_alone_and_in_the_mix(inner, multigrid):
    reqs = serve.poisson_requests(rate=5000.0, count=14, mix=MIX, seed=inner + 1)
    srv = serve.Server(hbm_budget=1 << 30, inner=inner, rtol=1e-8, multigrid=multigrid)
    try:
        done = srv.run(reqs)
    finally:
        srv.close()
    print(f"inner={tpfdm.DTYPE_NAMES[inner]} max_concurrent={srv.max_concurrent} {serve.latency_stats(done)}")
    assert srv.max_concurrent >= 3          # the solves did overlap
    for r in done:
        assert r.summary["status"] == 0 and r.summary["converged"]
        x_alone, s_alone = _alone(r, inner, multigrid)
        assert s_alone["iterations"] == r.summary["iterations"]
        # same kernels, same fixed-order reductions: identical bits
        assert np.array_equal(r.x.cpu().numpy(), x_alone), r.rid


@pytest.mark.parametrize("multigrid", [False, True])
def test_admission_keeps_within_the_budget(multigrid):
    import torch
    reqs = serve.poisson_requests(rate=5000.0, count=8, mix=[(3, 8)], seed=4)
    with tpfdm.Plan.mesh(4, (8, 8, 8), (0.125,) * 3) as plan:
        one = serve.slot_bytes(plan, 3, 8, multigrid)
    srv = serve.Server(hbm_budget=2 * one + one // 2, inner=tpfdm.F64, multigrid=multigrid)
    try:
        done = srv.run(reqs)
    finally:
        srv.close()
    assert srv.max_concurrent == 2
    assert all(r.summary["converged"] for r in done)
    # queued requests started only after earlier ones finished
    assert sum(1 for r in done if r.start > r.arrival + 1e-3) >= 4
    torch.cuda.synchronize()


@pytest.mark.parametrize("multigrid", [False, True])
def test_served_solve_matches_direct_solution(multigrid):
    reqs = serve.poisson_requests(rate=1000.0, count=3, mix=[(2, 4), (3, 4)], seed=7)
    srv = serve.Server(hbm_budget=1 << 28, inner=tpfdm.F64, rtol=1e-10, multigrid=multigrid)
    try:
        done = srv.run(reqs)
    finally:
        srv.close()
    for r in done:
        A = sipg.assemble(r.p, (r.m,) * 3, (1.0 / r.m,) * 3)
        b = r.b.cpu().numpy()
        xs = spl.spsolve(A.tocsc(), b)
        x = r.x.cpu().numpy()
        assert np.linalg.norm(b - A @ x) <= 2e-10 * np.linalg.norm(b)
        assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)


def test_oversized_request_is_rejected_and_the_rest_served():
    """A request whose slot alone exceeds the budget leaves the queue as
    rejected; the requests behind it are served as usual."""
    import torch
    budget = 4 * serve.class_slot_bytes(2, 6)
    assert serve.class_slot_bytes(3, 16) > budget
    reqs = serve.poisson_requests(rate=5000.0, count=5, mix=[(2, 4), (2, 6)], seed=9)
    big = torch.zeros(16 ** 3 * 64, dtype=torch.float64, device="cuda")
    reqs.insert(1, serve.Request(99, 3, 16, reqs[0].arrival, big))
    srv = serve.Server(hbm_budget=budget, inner=tpfdm.F64, rtol=1e-8)
    try:
        done = srv.run(reqs)
    finally:
        srv.close()
    assert srv.rejected == 1
    for r in done:
        if r.rid == 99:
            assert r.rejected and r.x is None and r.summary["status"] == "rejected"
        else:
            assert not r.rejected and r.summary["converged"], r.rid
    stats = serve.latency_stats(done)
    assert stats["rejected"] == 1
