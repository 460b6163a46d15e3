"""GPU parity of the multigrid V-cycle (tp_mg_*) and of CG preconditioned by
it (tp_pcg_set_multigrid) against the oracle's hierarchy: the same levels,
Chebyshev-accelerated block-Jacobi smoothing, embedding transfers and dense
coarse solve in FP64, so the V-cycle agrees element by element up to
rounding and MG-PCG takes the same number of iterations."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import mg, sipg
from paper_2609_04534_amd import tpfdm
from tests.gpu_util import from_blocked, to_blocked

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _rhs(nd, seed):
    return np.random.default_rng(seed).uniform(-1, 1, nd)


_HIER = {}


def _hierarchy(p, m):
    if (p, m) not in _HIER:
        _HIER[(p, m)] = mg.Hierarchy(p, m)
    return _HIER[(p, m)]


def _cube_plan(p, m):
    plan = tpfdm.Plan.mesh(p + 1, (m, m, m), (1.0 / m,) * 3)
    plan.setup_inverse(tpfdm.OP_CELL)
    return plan


# (p, m): levels m, m/2, ... down to the odd part of m (1 cell, or 3^3 cells)
VCYCLE_CASES = [(1, 8), (2, 4), (2, 6), (3, 2), (3, 4), (3, 6), (1, 12)]


@pytest.mark.parametrize("p,m", VCYCLE_CASES)
def test_vcycle_matches_oracle(p, m):
    torch = _torch()
    H = _hierarchy(p, m)
    nd = m ** 3 * (p + 1) ** 3
    print(f"p={p} m={m} levels={H.ms}", flush=True)
    for seed in (1, 2):
        b = _rhs(nd, seed + 10 * m + p)
        xo = H.vcycle(b)
        with _cube_plan(p, m) as plan, tpfdm.MG(plan) as V:
            bb = to_blocked(plan, b, tpfdm.F64)
            bx = torch.full_like(bb, float("nan"))
            V.vcycle(bb, bx)
            x = from_blocked(plan, bx, tpfdm.F64)
        scale = np.abs(xo).max()
        err = np.abs(x - xo).max()
        print(f"  seed={seed} max|x|={scale:.3e} max err={err:.3e}")
        # FP64 on both sides, summation orders differ: a few hundred ulps of
        # the solution's scale through a handful of smoothing sweeps
        assert err <= 1e-11 * scale


# boxes with unequal counts and lengths: (p, cells, h)
BOX_CASES = [(2, (4, 8, 2), (0.25, 0.125, 0.4)), (3, (2, 4, 6), (0.5, 0.3, 0.2)), (1, (8, 4, 4), (0.1, 0.2, 0.3))]


@pytest.mark.parametrize("p,cells,h", BOX_CASES)
def test_vcycle_matches_oracle_on_boxes(p, cells, h):
    """Boxes: the levels halve all three counts while all are even, each
    level doubles its lengths; element by element against the oracle's box
    hierarchy, and MG-PCG with its iteration count."""
    torch = _torch()
    H = mg.Hierarchy(p, cells, h=h)
    nd = H.A[0].shape[0]
    b = _rhs(nd, sum(cells) + p)
    xo = H.vcycle(b)
    _, ito, _ = sipg.pcg(H.A[0], b, H.vcycle, 1e-10, 200)
    print(f"p={p} cells={cells} levels={H.cells} oracle_iters={ito}", flush=True)
    with tpfdm.Plan.mesh(p + 1, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        with tpfdm.MG(plan) as V, tpfdm.PCG(plan) as solver:
            bb = to_blocked(plan, b, tpfdm.F64)
            bx = torch.full_like(bb, float("nan"))
            V.vcycle(bb, bx)
            x = from_blocked(plan, bx, tpfdm.F64)
            solver.set_multigrid(V)
            s = solver.solve(bb, torch.empty_like(bb), rtol=1e-10, maxit=200, check_every=4)
    err = np.abs(x - xo).max() / np.abs(xo).max()
    print(f"  vcycle rel err={err:.2e} {s}")
    assert err <= 1e-11
    assert s["converged"] and abs(s["iterations"] - ito) <= 1


def test_vcycle_single_level_is_the_exact_solve():
    """m odd: the finest level is the coarsest, and the V-cycle is A^{-1} b."""
    torch = _torch()
    p, m = 2, 3
    A = sipg.assemble(p, (m,) * 3, (1.0 / m,) * 3)
    b = _rhs(A.shape[0], 5)
    xs = spl.spsolve(A.tocsc(), b)
    with _cube_plan(p, m) as plan, tpfdm.MG(plan) as V:
        bb = to_blocked(plan, b, tpfdm.F64)
        bx = torch.empty_like(bb)
        V.vcycle(bb, bx)
        x = from_blocked(plan, bx, tpfdm.F64)
    assert np.abs(x - xs).max() <= 1e-10 * np.abs(xs).max()


def test_vcycle_symmetric_on_a_box():
    """A box that the oracle's cube hierarchy does not cover (cells 4 x 8 x 2,
    unequal lengths): the V-cycle is a symmetric operator, (V a, c) = (a, V c),
    and positive, (V a, a) > 0."""
    torch = _torch()
    n, cells, h = 3, (4, 8, 2), (0.25, 0.125, 0.4)
    nd = 64 * n ** 3
    a, c = _rhs(nd, 7), _rhs(nd, 8)
    with tpfdm.Plan.mesh(n, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        with tpfdm.MG(plan) as V:
            out = []
            for v in (a, c):
                bv = to_blocked(plan, v, tpfdm.F64)
                bx = torch.empty_like(bv)
                V.vcycle(bv, bx)
                out.append(from_blocked(plan, bx, tpfdm.F64))
    Va, Vc = out
    assert abs(Va @ c - a @ Vc) <= 1e-11 * np.linalg.norm(Va) * np.linalg.norm(c)
    assert Va @ a > 0 and Vc @ c > 0


MGPCG_CASES = [(1, 8), (2, 4), (2, 6), (3, 4), (1, 12)]


@pytest.mark.parametrize("p,m", MGPCG_CASES)
@pytest.mark.parametrize("inner", [tpfdm.F64, tpfdm.F32])
def test_mg_pcg_matches_oracle(p, m, inner):
    torch = _torch()
    H = _hierarchy(p, m)
    nd = m ** 3 * (p + 1) ** 3
    b = _rhs(nd, 100 + m + p)
    rtol = 1e-10
    xo, ito, _ = sipg.pcg(H.A[0], b, H.vcycle, rtol, 200)
    print(f"p={p} m={m} inner={tpfdm.DTYPE_NAMES[inner]} oracle_iters={ito}", flush=True)
    with _cube_plan(p, m) as plan, tpfdm.MG(plan) as V, tpfdm.PCG(plan) as solver:
        solver.set_multigrid(V)
        bb = to_blocked(plan, b, tpfdm.F64)
        bx = torch.full_like(bb, float("nan"))
        s = solver.solve(bb, bx, inner=inner, rtol=rtol, maxit=200, check_every=4)
        x = from_blocked(plan, bx, tpfdm.F64)
    true_rel = np.linalg.norm(b - H.A[0] @ x) / np.linalg.norm(b)
    print(f"  {s} true={true_rel:.2e}")
    assert s["converged"] and s["relres"] <= rtol
    assert true_rel <= 2 * rtol
    if inner == tpfdm.F64:
        assert abs(s["iterations"] - ito) <= 1
        assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    else:
        # FP32 block inverse in the smoother: a slightly different
        # preconditioner, still a few iterations
        assert s["iterations"] <= ito + 3


@pytest.mark.parametrize("p,m,inner", [(3, 64, tpfdm.F32), (2, 96, tpfdm.F64)])
def test_mg_pcg_full_size_sampled_residual(p, m, inner):
    """The largest meshes the solver is timed on (seven and six levels):
    the iteration count stays in the range of the small cubes, the solver's
    residual bound holds, and the oracle's true residual rows on sampled
    cells (the eight corners and random ones) of the GPU solution are small
    against b's scale."""
    torch = _torch()
    from paper_2609_04534_amd import workloads
    mesh = workloads.unit_cube_mesh(p, m, seed=9)
    print(f"p={p} m={m} inner={tpfdm.DTYPE_NAMES[inner]}", flush=True)
    with _cube_plan(p, m) as plan, tpfdm.MG(plan) as V, tpfdm.PCG(plan) as solver:
        solver.set_multigrid(V)
        bb = to_blocked(plan, mesh.u, tpfdm.F64)
        bx = torch.empty_like(bb)
        s = solver.solve(bb, bx, inner=inner, rtol=1e-8, maxit=100, check_every=4)
        x = from_blocked(plan, bx, tpfdm.F64)
    print(f"  {s}")
    assert s["converged"] and s["relres"] <= 1e-8
    assert s["iterations"] <= 16
    cells = (m,) * 3
    corners = [sipg.cell_index(cells, a, b_, c) for a in (0, m - 1) for b_ in (0, m - 1) for c in (0, m - 1)]
    rng = np.random.default_rng(2)
    sample = sorted(set(corners + rng.choice(m ** 3, 24, replace=False).tolist()))
    n3 = (p + 1) ** 3
    Ax = sipg.cell_apply(p, cells, (1.0 / m,) * 3, x, sample)
    rows = mesh.u.reshape(-1, n3)[sample] - Ax
    assert np.linalg.norm(rows) <= 1e-7 * np.linalg.norm(mesh.u)


def test_mg_pcg_nonblocking_and_switching_back():
    """begin/poll with the V-cycle gives the blocking solve's result bitwise;
    resetting to block-Jacobi restores its own (larger) iteration count."""
    torch = _torch()
    p, m = 2, 4
    nd = m ** 3 * (p + 1) ** 3
    b = _rhs(nd, 3)
    H = _hierarchy(p, m)
    _, it_bj, _ = sipg.pcg(H.A[0], b, lambda r: sipg.block_jacobi(p, (m,) * 3, (1.0 / m,) * 3, r), 1e-9, 2000)
    with _cube_plan(p, m) as plan, tpfdm.MG(plan) as V, tpfdm.PCG(plan) as solver:
        bb = to_blocked(plan, b, tpfdm.F64)
        solver.set_multigrid(V)
        x1 = torch.empty_like(bb)
        s1 = solver.solve(bb, x1, rtol=1e-9, check_every=3)
        x2 = torch.empty_like(bb)
        solver.begin(bb, x2, rtol=1e-9, check_every=3)
        s2 = None
        while s2 is None:
            s2 = solver.poll()
        assert s1["iterations"] == s2["iterations"] and torch.equal(x1, x2)
        solver.set_multigrid(None)
        x3 = torch.empty_like(bb)
        s3 = solver.solve(bb, x3, rtol=1e-9, maxit=2000)
    assert abs(s3["iterations"] - it_bj) <= 1
    assert s1["iterations"] < s3["iterations"] // 4


@pytest.mark.parametrize("basis", [tpfdm.BASIS_LAGRANGE, tpfdm.BASIS_HERMITE])
def test_mg_pcg_preconditioned_criterion_matches_oracle(basis):
    """The stopping rule of Sec. 6.1 (<r, z>^{1/2} reduced by rtol): the
    oracle's iteration count in both bases."""
    torch = _torch()
    p, m = 3, 4
    bname = sipg.HERMITE if basis == tpfdm.BASIS_HERMITE else sipg.LAGRANGE
    b = _rhs(m ** 3 * 64, 77)
    Hh = mg.Hierarchy(p, m, bname=bname)
    xo, ito, relo = sipg.pcg(Hh.A[0], b, Hh.vcycle, 1e-10, 200, criterion="preconditioned")
    with tpfdm.Plan.mesh(p + 1, (m,) * 3, (1.0 / m,) * 3, basis=basis) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        with tpfdm.MG(plan) as V, tpfdm.PCG(plan) as solver:
            solver.set_multigrid(V)
            solver.set_norm(tpfdm.PCG_PRECONDITIONED)
            bb = to_blocked(plan, b, tpfdm.F64)
            bx = torch.empty_like(bb)
            s = solver.solve(bb, bx, rtol=1e-10, maxit=200, check_every=4)
            x = from_blocked(plan, bx, tpfdm.F64)
    print(f"basis={basis} oracle_iters={ito} {s}")
    assert s["converged"] and abs(s["iterations"] - ito) <= 1
    if s["iterations"] == ito:
        # the same iterate up to rounding: the oracle's residual and solution
        assert abs(s["relres"] - relo) <= 0.05 * relo
        assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)


def test_mg_errors():
    torch = _torch()
    # no cell inverse set up
    with tpfdm.Plan.mesh(3, (4, 4, 4), (0.25,) * 3) as plan:
        with pytest.raises(tpfdm.TpfdmError) as e:
            tpfdm.MG(plan)
        assert e.value.status == -9
    # coarsest level too large for the dense solve: 5^3 cells x 27
    with _cube_plan(2, 5) as plan:
        with pytest.raises(tpfdm.TpfdmError) as e:
            tpfdm.MG(plan)
        assert e.value.status == -2
    # n >= 5 in the Hermite-type basis
    with tpfdm.Plan.mesh(6, (2, 2, 2), (0.5,) * 3, basis=tpfdm.BASIS_HERMITE) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        with pytest.raises(tpfdm.TpfdmError) as e:
            tpfdm.MG(plan)
        assert e.value.status == -2
    # a multigrid of another plan
    with _cube_plan(2, 2) as p1, _cube_plan(2, 2) as p2, tpfdm.MG(p1) as V, tpfdm.PCG(p2) as solver:
        with pytest.raises(tpfdm.TpfdmError) as e:
            solver.set_multigrid(V)
        assert e.value.status == -1
        buf = torch.zeros(p1.vector_elems, dtype=torch.float64, device="cuda")
        with pytest.raises(tpfdm.TpfdmError):
            V.vcycle(buf, buf)
        with pytest.raises(tpfdm.TpfdmError) as e:
            solver.set_norm(2)
        assert e.value.status == -1
    # the plan's inverse set up for another operator afterwards: refused
    with _cube_plan(2, 2) as plan, tpfdm.MG(plan) as V:
        buf = torch.zeros(plan.vector_elems, dtype=torch.float64, device="cuda")
        plan.setup_inverse(tpfdm.OP_CELL, mode=tpfdm.FACTOR_GENERAL)
        with pytest.raises(tpfdm.TpfdmError) as e:
            V.vcycle(buf, torch.zeros_like(buf))
        assert e.value.status == -9


@pytest.mark.parametrize("multigrid", [False, True])
def test_nonfinite_rhs_is_reported(multigrid):
    """A NaN in b: the solve stops at once with TP_ERR_NONFINITE (the start
    reduction sees it), with the V-cycle as with block-Jacobi; a following
    finite solve on the same solver is unaffected."""
    torch = _torch()
    p, m = 2, 4
    b = _rhs(m ** 3 * 27, 5)
    with _cube_plan(p, m) as plan, tpfdm.MG(plan) as V, tpfdm.PCG(plan) as solver:
        if multigrid:
            solver.set_multigrid(V)
        bad = b.copy()
        bad[17] = np.nan
        bb = to_blocked(plan, bad, tpfdm.F64)
        bx = torch.empty_like(bb)
        s = solver.solve(bb, bx, rtol=1e-9, maxit=100, raise_on_failure=False)
        assert s["status"] == -6 and not s["converged"] and s["iterations"] == 0
        bb = to_blocked(plan, b, tpfdm.F64)
        s = solver.solve(bb, bx, rtol=1e-9, maxit=2000)
        assert s["converged"]


# ------------------------------------------------------------------ FP32 level storage
@pytest.mark.parametrize("p,m", [(1, 8), (2, 4), (3, 4), (3, 6), (4, 4), (6, 2), (7, 2)])
def test_vcycle_fp32_storage_matches_oracle(p, m):
    """Level vectors stored in FP32 (tp_mg_create_typed), the smoother's and
    the residual's operator rows computed in FP32, the transfers in FP64;
    the V-cycle agrees with the oracle's FP64 V-cycle to a few FP32
    roundings of the solution's scale per sweep (lane kernels for n <= 4,
    wave kernels for n >= 5)."""
    torch = _torch()
    H = _hierarchy(p, m)
    nd = m ** 3 * (p + 1) ** 3
    b = _rhs(nd, 40 + 10 * m + p)
    xo = H.vcycle(b)
    with _cube_plan(p, m) as plan, tpfdm.MG(plan, storage=tpfdm.F32) as V:
        bb = to_blocked(plan, b, tpfdm.F64)
        bx = torch.full_like(bb, float("nan"))
        V.vcycle(bb, bx)
        x = from_blocked(plan, bx, tpfdm.F64)
    err = np.abs(x - xo).max() / np.abs(xo).max()
    print(f"p={p} m={m} FP32-storage V-cycle rel err {err:.2e}")
    assert np.all(np.isfinite(x))
    assert err <= 2e-5


@pytest.mark.parametrize("p,m,inner", [(2, 8, tpfdm.F32), (3, 8, tpfdm.F32), (3, 4, tpfdm.F64),
                                       (4, 4, tpfdm.F32), (7, 2, tpfdm.F32), (7, 2, tpfdm.F64)])
def test_mg_pcg_fp32_storage_reaches_the_oracle_residual(p, m, inner):
    """MG-PCG with FP32 level storage (z in FP32; x, r, p and the dot
    products in FP64) reaches the same true residual as the FP64 solve,
    measured with the oracle's operator, within the FP64 solve's iteration
    count + 1."""
    torch = _torch()
    cells, h = (m,) * 3, (1.0 / m,) * 3
    A = sipg.assemble(p, cells, h)
    b = _rhs(A.shape[0], 60 + p + m)
    rtol = 1e-10
    res = {}
    with _cube_plan(p, m) as plan:
        bb = to_blocked(plan, b, tpfdm.F64)
        for storage in (tpfdm.F64, tpfdm.F32):
            with tpfdm.MG(plan, storage=storage) as V, tpfdm.PCG(plan) as solver:
                solver.set_multigrid(V)
                bx = torch.full_like(bb, float("nan"))
                s = solver.solve(bb, bx, inner=inner, rtol=rtol, maxit=100, check_every=4)
                x = from_blocked(plan, bx, tpfdm.F64)
            true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
            res[storage] = (s, true, x)
            print(f"p={p} m={m} storage={tpfdm.DTYPE_NAMES[storage]} {s} true relres {true:.2e}")
    s64, t64, x64 = res[tpfdm.F64]
    s32, t32, x32 = res[tpfdm.F32]
    assert s64["converged"] and s32["converged"]
    assert s32["iterations"] <= s64["iterations"] + 1
    assert t64 <= 2 * rtol and t32 <= 2 * rtol
    xs = spl.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x32 - xs) <= 1e-7 * np.linalg.norm(xs)


# ------------------------------------------------------------------ n >= 5 (one cell per wave)
@pytest.mark.parametrize("p,m", [(4, 4), (6, 2), (7, 2)])
def test_vcycle_wave_degrees_match_oracle(p, m):
    """The V-cycle for n >= 5 (wave kernels, layout B = 1) element by element
    against the oracle's hierarchy."""
    torch = _torch()
    H = _hierarchy(p, m)
    nd = m ** 3 * (p + 1) ** 3
    b = _rhs(nd, 70 + p + m)
    xo = H.vcycle(b)
    with _cube_plan(p, m) as plan, tpfdm.MG(plan) as V:
        bb = to_blocked(plan, b, tpfdm.F64)
        bx = torch.full_like(bb, float("nan"))
        V.vcycle(bb, bx)
        x = from_blocked(plan, bx, tpfdm.F64)
    err = np.abs(x - xo).max() / np.abs(xo).max()
    print(f"p={p} m={m} levels={H.ms} V-cycle rel err {err:.2e}")
    assert err <= 1e-11


@pytest.mark.parametrize("p,m,inner", [(4, 4, tpfdm.F64), (7, 2, tpfdm.F64), (7, 2, tpfdm.F32)])
def test_mg_pcg_wave_degrees_iteration_count(p, m, inner):
    """MG-PCG for n >= 5 takes the oracle's MG-PCG iteration count (+-1) and
    reaches its true residual."""
    torch = _torch()
    H = _hierarchy(p, m)
    b = _rhs(H.A[0].shape[0], 80 + p + m)
    rtol = 1e-10
    _, ito, _ = sipg.pcg(H.A[0], b, H.vcycle, rtol, 200)
    with _cube_plan(p, m) as plan, tpfdm.MG(plan) as V, tpfdm.PCG(plan) as solver:
        solver.set_multigrid(V)
        bb = to_blocked(plan, b, tpfdm.F64)
        bx = torch.full_like(bb, float("nan"))
        s = solver.solve(bb, bx, inner=inner, rtol=rtol, maxit=200, check_every=4)
        x = from_blocked(plan, bx, tpfdm.F64)
    true = np.linalg.norm(b - H.A[0] @ x) / np.linalg.norm(b)
    print(f"p={p} m={m} inner={tpfdm.DTYPE_NAMES[inner]} oracle_iters={ito} {s} true relres {true:.2e}")
    assert s["converged"] and abs(s["iterations"] - ito) <= 1
    assert true <= 2 * rtol


def test_mg_wave_rejects_what_it_does_not_cover():
    # coarsest level 343 cells: too many for the dense solve even at degree 1
    with _cube_plan(7, 7) as plan:
        with pytest.raises(tpfdm.TpfdmError) as e:
            tpfdm.MG(plan)
        assert e.value.status == -2
    with _cube_plan(7, 2) as plan:
        with pytest.raises(tpfdm.TpfdmError) as e:
            tpfdm.MG(plan, storage=tpfdm.F16)
        assert e.value.status == -2


# coarsest geometric level above 2048 unknowns: the degree-1 level on its
# cells is solved densely; (p, cells, h)
DEGREE_CASES = [(7, (3, 3, 1), (0.3, 0.3, 0.5)), (7, (3, 3, 3), (1.0 / 3,) * 3),
                (6, (6, 6, 2), (1.0 / 6, 1.0 / 6, 0.5)), (4, (6, 6, 6), (1.0 / 6,) * 3)]


@pytest.mark.parametrize("p,cells,h", DEGREE_CASES)
def test_vcycle_degree_level_matches_oracle(p, cells, h):
    """The V-cycle with the degree-coarsened coarsest level (Galerkin E^T A E
    probed on the GPU, the oracle forms it from its sparse matrices) element
    by element, and MG-PCG with the oracle's iteration count."""
    torch = _torch()
    H = mg.Hierarchy(p, cells, h=h, coarse_degree=1)
    nd = H.A[0].shape[0]
    b = _rhs(nd, 90 + p + sum(cells))
    xo = H.vcycle(b)
    _, ito, _ = sipg.pcg(H.A[0], b, H.vcycle, 1e-10, 200)
    print(f"p={p} cells={cells} levels={H.cells} degrees={H.degrees} oracle_iters={ito}", flush=True)
    with tpfdm.Plan.mesh(p + 1, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        with tpfdm.MG(plan) as V, tpfdm.PCG(plan) as solver:
            bb = to_blocked(plan, b, tpfdm.F64)
            bx = torch.full_like(bb, float("nan"))
            V.vcycle(bb, bx)
            x = from_blocked(plan, bx, tpfdm.F64)
            solver.set_multigrid(V)
            bs = torch.zeros_like(bb)
            s = solver.solve(bb, bs, rtol=1e-10, maxit=200, check_every=4)
            xs = from_blocked(plan, bs, tpfdm.F64)
    err = np.abs(x - xo).max() / np.abs(xo).max()
    true = np.linalg.norm(b - H.A[0] @ xs) / np.linalg.norm(b)
    print(f"  vcycle rel err={err:.2e} {s} true relres {true:.2e}")
    assert err <= 1e-11
    assert s["converged"] and abs(s["iterations"] - ito) <= 1
    assert true <= 2e-10


@pytest.mark.parametrize("p,cells,h", [DEGREE_CASES[1], DEGREE_CASES[2]])
def test_vcycle_degree_level_fp32_storage(p, cells, h):
    """FP32 level vectors on a hierarchy that ends on the degree-1 level (its
    right-hand side, correction and dense solve in FP64): the V-cycle within
    FP32 roundings of the oracle's, MG-PCG with an FP32 inner precision in
    the oracle's iteration count + 1 to its true residual."""
    torch = _torch()
    H = mg.Hierarchy(p, cells, h=h, coarse_degree=1)
    b = _rhs(H.A[0].shape[0], 95 + p + sum(cells))
    xo = H.vcycle(b)
    _, ito, _ = sipg.pcg(H.A[0], b, H.vcycle, 1e-10, 200)
    with tpfdm.Plan.mesh(p + 1, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        with tpfdm.MG(plan, storage=tpfdm.F32) as V, tpfdm.PCG(plan) as solver:
            bb = to_blocked(plan, b, tpfdm.F64)
            bx = torch.full_like(bb, float("nan"))
            V.vcycle(bb, bx)
            x = from_blocked(plan, bx, tpfdm.F64)
            solver.set_multigrid(V)
            bs = torch.zeros_like(bb)
            s = solver.solve(bb, bs, inner=tpfdm.F32, rtol=1e-10, maxit=200, check_every=4)
            xs = from_blocked(plan, bs, tpfdm.F64)
    err = np.abs(x - xo).max() / np.abs(xo).max()
    true = np.linalg.norm(b - H.A[0] @ xs) / np.linalg.norm(b)
    print(f"p={p} cells={cells} FP32 levels: vcycle rel err={err:.2e} oracle_iters={ito} {s} true relres {true:.2e}")
    assert np.all(np.isfinite(x)) and err <= 2e-5
    assert s["converged"] and s["iterations"] <= ito + 1
    assert true <= 2e-10


@pytest.mark.parametrize("p,cells,h", BOX_CASES + [(7, (2, 4, 2), (0.5, 0.25, 0.4)), (5, (4, 2, 2), (0.2, 0.4, 0.3))])
def test_vcycle_fp32_storage_on_boxes(p, cells, h):
    """FP32 level vectors on boxes with unequal counts and lengths (lane
    kernels for n <= 4, wave kernels for n >= 5): the V-cycle within FP32
    roundings of the oracle's FP64 one, MG-PCG with an FP32 inner precision
    within the oracle's iteration count + 1 to its true residual."""
    torch = _torch()
    H = mg.Hierarchy(p, cells, h=h)
    b = _rhs(H.A[0].shape[0], 3 * sum(cells) + p)
    xo = H.vcycle(b)
    _, ito, _ = sipg.pcg(H.A[0], b, H.vcycle, 1e-10, 200)
    with tpfdm.Plan.mesh(p + 1, cells, h) as plan:
        plan.setup_inverse(tpfdm.OP_CELL)
        with tpfdm.MG(plan, storage=tpfdm.F32) as V, tpfdm.PCG(plan) as solver:
            bb = to_blocked(plan, b, tpfdm.F64)
            bx = torch.full_like(bb, float("nan"))
            V.vcycle(bb, bx)
            x = from_blocked(plan, bx, tpfdm.F64)
            solver.set_multigrid(V)
            bs = torch.zeros_like(bb)
            s = solver.solve(bb, bs, inner=tpfdm.F32, rtol=1e-10, maxit=200, check_every=4)
            xs = from_blocked(plan, bs, tpfdm.F64)
    err = np.abs(x - xo).max() / np.abs(xo).max()
    true = np.linalg.norm(b - H.A[0] @ xs) / np.linalg.norm(b)
    print(f"p={p} cells={cells} FP32 levels: vcycle rel err={err:.2e} oracle_iters={ito} {s} true {true:.2e}")
    assert np.all(np.isfinite(x)) and err <= 2e-5
    assert s["converged"] and s["iterations"] <= ito + 1
    assert true <= 2e-10
