"""GPU parity of the preconditioned CG solver of mesh plans (tp_pcg_*)
against the oracle: the sparse direct solution of the coupled SIPG system,
the oracle's textbook PCG with the dense block-Jacobi preconditioner (same
recurrences, so the same iteration counts in FP64), and true residual rows
evaluated by the oracle on the GPU's solution."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import sipg
from paper_2609_04534_amd import tpfdm, workloads
from tests.gpu_util import from_blocked, to_blocked

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _rhs(ncell, n, seed):
    return np.random.default_rng(seed).uniform(-1, 1, ncell * n ** 3)


CASES = [(2, (5, 6, 7), (0.3, 0.2, 0.5)), (3, (4, 5, 6), (0.25, 0.5, 0.4)), (4, (3, 4, 5), (1.0, 0.5, 0.7)),
         (3, (1, 1, 70), (0.1, 0.1, 0.1)), (4, (2, 9, 1), (0.5, 0.5, 0.5)),
         # one cell per wave (n >= 5)
         (8, (2, 2, 3), (0.5, 0.5, 0.5)), (5, (3, 2, 3), (0.3, 0.4, 0.5)), (6, (2, 2, 2), (1.0, 0.7, 0.5)),
         (7, (1, 2, 3), (0.4, 0.4, 0.4))]


@pytest.mark.parametrize("n,cells,h", CASES)
@pytest.mark.parametrize("inner", [tpfdm.F64, tpfdm.F32])
def test_pcg_matches_oracle(n, cells, h, inner):
    torch = _torch()
    p = n - 1
    ncell = cells[0] * cells[1] * cells[2]
    b = _rhs(ncell, n, seed=ncell + n)
    rtol = 1e-10 if inner == tpfdm.F64 else 1e-8
    A = sipg.assemble(p, cells, h)
    xs = spl.spsolve(A.tocsc(), b)
    xo, ito, _ = sipg.pcg(A, b, lambda r: sipg.block_jacobi(p, cells, h, r), rtol, 2000)
    print(f"n={n} cells={cells} inner={tpfdm.DTYPE_NAMES[inner]} oracle_iters={ito}", flush=True)
    with tpfdm.Plan.mesh(n, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bb = to_blocked(plan, b, tpfdm.F64)
        bx = torch.full_like(bb, float("nan"))
        with tpfdm.PCG(plan) as solver:
            s = solver.solve(bb, bx, inner=inner, rtol=rtol, maxit=2000, check_every=8)
        x = from_blocked(plan, bx, tpfdm.F64)
    true_rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    print(f"  iters={s['iterations']} relres={s['relres']:.2e} true={true_rel:.2e} err={err:.2e}")
    assert s["converged"] and s["relres"] <= rtol
    assert true_rel <= 2 * rtol
    if inner == tpfdm.F64:
        # same recurrences in FP64: the same iteration count up to rounding at the threshold
        assert abs(s["iterations"] - ito) <= 1
        assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)
    else:
        assert abs(s["iterations"] - ito) <= max(3, ito // 10)


def test_block_jacobi_pcg_preconditioned_criterion_matches_oracle():
    torch = _torch()
    n, cells, h = 3, (4, 5, 6), (0.25, 0.5, 0.4)
    p = n - 1
    b = _rhs(120, n, 12)
    A = sipg.assemble(p, cells, h)
    _, ito, _ = sipg.pcg(A, b, lambda r: sipg.block_jacobi(p, cells, h, r), 1e-9, 2000, criterion="preconditioned")
    with tpfdm.Plan.mesh(n, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bb = to_blocked(plan, b, tpfdm.F64)
        bx = torch.empty_like(bb)
        with tpfdm.PCG(plan) as solver:
            solver.set_norm(tpfdm.PCG_PRECONDITIONED)
            s = solver.solve(bb, bx, rtol=1e-9, maxit=2000)
    assert s["converged"] and abs(s["iterations"] - ito) <= 1


def test_pcg_initial_guess_and_zero_rhs():
    torch = _torch()
    n, cells, h = 3, (4, 4, 4), (0.25, 0.25, 0.25)
    p = n - 1
    b = _rhs(64, n, 1)
    A = sipg.assemble(p, cells, h)
    xs = spl.spsolve(A.tocsc(), b)
    with tpfdm.Plan.mesh(n, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bb = to_blocked(plan, b, tpfdm.F64)
        with tpfdm.PCG(plan) as solver:
            # the exact solution as the initial guess: no iteration needed
            bx = to_blocked(plan, xs, tpfdm.F64)
            s = solver.solve(bb, bx, x_is_zero=False, rtol=1e-9)
            assert s["iterations"] == 0 and s["converged"]
            # a random initial guess converges to the same solution
            bx = to_blocked(plan, _rhs(64, n, 2), tpfdm.F64)
            s = solver.solve(bb, bx, x_is_zero=False, rtol=1e-11, maxit=3000)
            x = from_blocked(plan, bx, tpfdm.F64)
            assert s["converged"] and np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
            # b = 0 with x_is_zero: x = 0 written, no iteration
            bz = torch.zeros_like(bb)
            bx = torch.full_like(bb, float("nan"))
            s = solver.solve(bz, bx, x_is_zero=True)
            assert s["iterations"] == 0 and s["converged"]
            assert np.all(from_blocked(plan, bx, tpfdm.F64) == 0.0)


def test_pcg_iteration_limit_returns_the_iterate():
    """maxit reached: TP_ERR_NOT_CONVERGED, and x is the oracle PCG's iterate
    after the same number of steps."""
    torch = _torch()
    n, cells, h = 4, (3, 3, 3), (0.5, 0.5, 0.5)
    p = n - 1
    b = _rhs(27, n, 3)
    A = sipg.assemble(p, cells, h)
    xo, ito, _ = sipg.pcg(A, b, lambda r: sipg.block_jacobi(p, cells, h, r), 1e-14, 5)
    assert ito == 5
    with tpfdm.Plan.mesh(n, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bb = to_blocked(plan, b, tpfdm.F64)
        bx = torch.empty_like(bb)
        with tpfdm.PCG(plan) as solver:
            s = solver.solve(bb, bx, rtol=1e-14, maxit=5, check_every=3, raise_on_failure=False)
        x = from_blocked(plan, bx, tpfdm.F64)
    assert s["status"] == -5 and s["iterations"] == 5 and not s["converged"]
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)


def test_pcg_errors():
    torch = _torch()
    with tpfdm.Plan([tpfdm.GroupSpec(3, 64, np.ones((8, 3)))]) as plan:
        with pytest.raises(tpfdm.TpfdmError) as e:
            tpfdm.PCG(plan)
        assert e.value.status == -2
    with tpfdm.Plan.mesh(3, (2, 2, 2), (1, 1, 1)) as plan:
        buf = torch.zeros(plan.vector_elems, dtype=torch.float64, device="cuda")
        with tpfdm.PCG(plan) as solver:
            with pytest.raises(tpfdm.TpfdmError) as e:
                solver.solve(buf, torch.zeros_like(buf))
            assert e.value.status == -9          # no setup
            plan.setup_inverse(tpfdm.OP_CELL)
            with pytest.raises(tpfdm.TpfdmError) as e:
                solver.solve(buf, torch.zeros_like(buf), inner=tpfdm.F16)
            assert e.value.status == -2
            with pytest.raises(tpfdm.TpfdmError) as e:
                solver.solve(buf, torch.zeros_like(buf), rtol=0.0)
            assert e.value.status == -1


@pytest.mark.parametrize("p,m,inner", [(3, 48, tpfdm.F32), (2, 32, tpfdm.F64), (7, 16, tpfdm.F64)])
def test_pcg_serving_size_sampled_residual(p, m, inner):
    """The largest serving mesh: the solver's residual bound holds, and the
    oracle's true residual rows on sampled cells (corners, edges, interior)
    of the GPU solution are small against b's scale."""
    torch = _torch()
    mesh = workloads.unit_cube_mesh(p, m, seed=9)
    n, cells, h = mesh.n, mesh.cells, mesh.h
    print(f"p={p} m={m} inner={tpfdm.DTYPE_NAMES[inner]}", flush=True)
    with tpfdm.Plan.mesh(n, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bb = to_blocked(plan, mesh.u, tpfdm.F64)
        bx = torch.empty_like(bb)
        with tpfdm.PCG(plan) as solver:
            s = solver.solve(bb, bx, inner=inner, rtol=1e-8, maxit=5000)
        x = from_blocked(plan, bx, tpfdm.F64)
    print(f"  {s}")
    assert s["converged"] and s["relres"] <= 1e-8
    corners = [sipg.cell_index(cells, a, b_, c) for a in (0, m - 1) for b_ in (0, m - 1) for c in (0, m - 1)]
    rng = np.random.default_rng(1)
    sample = sorted(set(corners + rng.choice(m ** 3, 24, replace=False).tolist()))
    n3 = n ** 3
    Ax = sipg.cell_apply(p, cells, h, x, sample)
    rows = mesh.u.reshape(-1, n3)[sample] - Ax
    # each sampled row of the true residual is a piece of r with ||r|| <= ~1e-8 ||b||
    assert np.linalg.norm(rows) <= 1e-7 * np.linalg.norm(mesh.u)


@pytest.mark.parametrize("m", [24, 48])
def test_mg_pcg_degree_level_at_serving_size(m):
    """Degree 7 on the serving meshes whose coarsest geometric level is 3^3
    cells (24^3 and 48^3): MG-PCG through the degree-1 coarsest level
    converges in a multigrid-like iteration count, and the oracle's true
    residual rows on sampled cells of the GPU solution are small."""
    torch = _torch()
    p = 7
    mesh = workloads.unit_cube_mesh(p, m, seed=11)
    n, cells, h = mesh.n, mesh.cells, mesh.h
    print(f"p={p} m={m}", flush=True)
    with tpfdm.Plan.mesh(n, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        bb = to_blocked(plan, mesh.u, tpfdm.F64)
        bx = torch.empty_like(bb)
        with tpfdm.MG(plan) as V, tpfdm.PCG(plan) as solver:
            solver.set_multigrid(V)
            s = solver.solve(bb, bx, inner=tpfdm.F64, rtol=1e-8, maxit=200, check_every=4)
        x = from_blocked(plan, bx, tpfdm.F64)
    print(f"  {s}")
    assert s["converged"] and s["relres"] <= 1e-8 and s["iterations"] <= 24
    corners = [sipg.cell_index(cells, a, b_, c) for a in (0, m - 1) for b_ in (0, m - 1) for c in (0, m - 1)]
    rng = np.random.default_rng(2)
    sample = sorted(set(corners + rng.choice(m ** 3, 16, replace=False).tolist()))
    Ax = sipg.cell_apply(p, cells, h, x, sample)
    rows = mesh.u.reshape(-1, n ** 3)[sample] - Ax
    assert np.linalg.norm(rows) <= 1e-7 * np.linalg.norm(mesh.u)
