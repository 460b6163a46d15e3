"""GPU parity of mesh plans in the Hermite-type basis (n = 4, p = 3) against
the oracle assembled in that basis: the coupled operator and its parts
element by element, the change of basis, the cell-block inverse, PCG, the
multigrid V-cycle, agreement of the solution with the Lagrange plan's after
conversion, and sampled cells at the full benchmark size."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import dense, hermite, mg, sipg
from paper_2609_04534_amd import tpfdm
from tests.gpu_util import from_blocked, to_blocked

pytestmark = pytest.mark.gpu

H = sipg.HERMITE
TOL = {tpfdm.F64: 1e-12, tpfdm.F32: 2e-6}
P = 3
N = 4


def _torch():
    import torch
    return torch


def _u(ncell, seed):
    return np.random.default_rng(seed).uniform(-1, 1, ncell * N ** 3)


def _plan(cells, h, B=None, setup=True):
    plan = tpfdm.Plan.mesh(N, cells, h, layout_B=B, basis=tpfdm.BASIS_HERMITE)
    if setup:
        plan.setup_inverse(tpfdm.OP_CELL)
    return plan


# several 64-cell tiles with ragged tails, one-cell-thick meshes along each
# axis, layouts B = 1, 8, 128, a single cell
CASES = [
    ((3, 5, 13), (0.25, 0.5, 1.0), None),
    ((1, 1, 70), (0.3, 0.3, 0.3), None),
    ((70, 1, 1), (0.1, 0.4, 0.2), None),
    ((2, 33, 1), (1.0, 0.5, 2.0), None),
    ((4, 5, 6), (0.7, 1.3, 0.45), 1),
    ((3, 4, 5), (0.7, 1.3, 0.45), 8),
    ((6, 6, 8), (0.2, 0.3, 0.15), 128),
    ((1, 1, 1), (1.0, 1.0, 1.0), None),
]
OPS = [(tpfdm.OP_SIPG, sipg.FULL), (tpfdm.OP_SIPG_FACE, sipg.FACE), (tpfdm.OP_NEUMANN, sipg.VOLUME)]


@pytest.mark.parametrize("cells,h,B", CASES)
@pytest.mark.parametrize("dt", [tpfdm.F64, tpfdm.F32])
def test_operators_match_oracle(cells, h, B, dt):
    torch = _torch()
    ncell = cells[0] * cells[1] * cells[2]
    u = _u(ncell, ncell + 11)
    print(f"cells={cells} B={B} dt={tpfdm.DTYPE_NAMES[dt]}", flush=True)
    with _plan(cells, h, B, setup=False) as plan:
        bu = to_blocked(plan, u, dt)
        for op, part in OPS:
            A = sipg.assemble(P, cells, h, part, bname=H)
            ref = A @ u
            bv = torch.full_like(bu, float("nan"))
            plan.apply(bu, bv, op=op)
            got = from_blocked(plan, bv, dt)
            scale = np.max(np.abs(abs(A) @ np.abs(u)))
            err = float(np.max(np.abs(got - ref)) / scale)
            print(f"  op={op} err={err:.2e}")
            assert err <= TOL[dt]


@pytest.mark.parametrize("cells,h,B", [((3, 5, 13), (0.25, 0.5, 1.0), None), ((4, 5, 6), (0.7, 1.3, 0.45), 1)])
def test_change_basis_matches_oracle(cells, h, B):
    torch = _torch()
    ncell = cells[0] * cells[1] * cells[2]
    u = _u(ncell, 4)
    with _plan(cells, h, B, setup=False) as plan:
        bu = to_blocked(plan, u, tpfdm.F64)
        bv = torch.full_like(bu, float("nan"))
        plan.change_basis(bu, bv, to_nodal=True)
        nodal = from_blocked(plan, bv, tpfdm.F64)
        bw = torch.full_like(bu, float("nan"))
        plan.change_basis(bv, bw, to_nodal=False)
        back = from_blocked(plan, bw, tpfdm.F64)
        bh = torch.full_like(bu, float("nan"))
        plan.change_basis(bu, bh, to_nodal=False)
        herm = from_blocked(plan, bh, tpfdm.F64)
    assert np.abs(nodal - hermite.to_lagrange(P, u, ncell)).max() <= 1e-14 * 8
    assert np.abs(herm - hermite.to_hermite(P, u, ncell)).max() <= 1e-12 * np.abs(herm).max()
    # the round trip through T and T^-1 in three directions loses up to
    # about cond(T)^3 eps (cond(T) = 18.8 at p = 3): 1.5e-12
    kappa = np.linalg.cond(hermite.transform(P))
    assert np.abs(back - u).max() <= 4 * kappa ** 3 * np.finfo(float).eps


@pytest.mark.parametrize("dt", [tpfdm.F64, tpfdm.F32])
def test_cell_inverse_matches_oracle(dt):
    """apply_inverse with the cell blocks (the block-Jacobi preconditioner)
    against the oracle's dense solve of its Hermite cell block, refined with a
    long-double residual.  The block is badly scaled in this basis (2-norm
    condition number 1.9e8 on these lengths, 1.4e4 after symmetric diagonal
    scaling), so an unrefined LAPACK solve is itself off by 1.8e-12; the
    refined solve is exact to a few ulps."""
    torch = _torch()
    cells, h = (3, 5, 13), (0.25, 0.5, 1.0)
    ncell = 195
    r = _u(ncell, 8).reshape(ncell, -1)
    D = sipg.cell_block(P, h, bname=H)
    ref = np.array([dense.solve_block(D, rb) for rb in r])
    with _plan(cells, h) as plan:
        br = to_blocked(plan, r.reshape(-1), dt)
        bx = torch.full_like(br, float("nan"))
        plan.apply_inverse(br, bx)
        x = from_blocked(plan, bx, dt).reshape(ncell, -1)
    err = np.linalg.norm(x - ref, axis=1) / np.linalg.norm(ref, axis=1)
    print(f"dt={tpfdm.DTYPE_NAMES[dt]} max block rel err (2-norm)={err.max():.2e}")
    assert err.max() <= (1e-12 if dt == tpfdm.F64 else 5e-6)


@pytest.mark.parametrize("inner", [tpfdm.F64, tpfdm.F32])
def test_pcg_matches_oracle(inner):
    torch = _torch()
    cells, h = (4, 5, 6), (0.25, 0.5, 0.4)
    ncell = 120
    b = _u(ncell, 21)
    A = sipg.assemble(P, cells, h, bname=H)
    xs = spl.spsolve(A.tocsc(), b)
    rtol = 1e-10
    xo, ito, _ = sipg.pcg(A, b, lambda r: sipg.block_jacobi(P, cells, h, r, bname=H), rtol, 3000)
    with _plan(cells, h) as plan, tpfdm.PCG(plan) as solver:
        bb = to_blocked(plan, b, tpfdm.F64)
        bx = torch.full_like(bb, float("nan"))
        s = solver.solve(bb, bx, inner=inner, rtol=rtol, maxit=3000, check_every=8)
        x = from_blocked(plan, bx, tpfdm.F64)
    print(f"inner={tpfdm.DTYPE_NAMES[inner]} oracle_iters={ito} {s}")
    assert s["converged"] and np.linalg.norm(b - A @ x) <= 2 * rtol * np.linalg.norm(b)
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)
    if inner == tpfdm.F64:
        assert abs(s["iterations"] - ito) <= 1
    else:
        assert abs(s["iterations"] - ito) <= max(3, ito // 10)


@pytest.mark.parametrize("m", [4, 6])
def test_vcycle_and_mg_pcg_match_oracle(m):
    torch = _torch()
    Hh = mg.Hierarchy(P, m, bname=H)
    b = _u(m ** 3, 30 + m)
    xo = Hh.vcycle(b)
    _, ito, _ = sipg.pcg(Hh.A[0], b, Hh.vcycle, 1e-10, 200)
    with _plan((m,) * 3, (1.0 / m,) * 3) as plan, tpfdm.MG(plan) as V, tpfdm.PCG(plan) as solver:
        bb = to_blocked(plan, b, tpfdm.F64)
        bx = torch.full_like(bb, float("nan"))
        V.vcycle(bb, bx)
        x = from_blocked(plan, bx, tpfdm.F64)
        solver.set_multigrid(V)
        by = torch.full_like(bb, float("nan"))
        s = solver.solve(bb, by, rtol=1e-10, maxit=200, check_every=4)
    err = np.abs(x - xo).max() / np.abs(xo).max()
    print(f"m={m} vcycle rel err={err:.2e} oracle_iters={ito} {s}")
    assert err <= 1e-10
    assert s["converged"] and abs(s["iterations"] - ito) <= 1


@pytest.mark.parametrize("p", [3, 7])
def test_change_basis_of_loads(p):
    """Mode 2 (loads): b_H = T3^T b_L cell by cell, against the oracle."""
    torch = _torch()
    cells = (2, 3, 2)
    ncell = 12
    n = p + 1
    bL = np.random.default_rng(p + 50).uniform(-1, 1, ncell * n ** 3)
    T = hermite.transform(p)
    ref = (bL.reshape(ncell, -1) @ np.kron(np.kron(T, T), T)).reshape(-1)
    with tpfdm.Plan.mesh(n, cells, (0.5, 0.4, 0.6), basis=tpfdm.BASIS_HERMITE) as plan:
        bu = to_blocked(plan, bL, tpfdm.F64)
        bv = torch.full_like(bu, float("nan"))
        plan.change_basis(bu, bv, loads=True)
        got = from_blocked(plan, bv, tpfdm.F64)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_solution_agrees_with_the_lagrange_plan():
    """The same discrete problem in both bases: solve A_H x_H = T3^T b_L,
    convert x_H to nodal values, compare with the Lagrange plan's solution."""
    torch = _torch()
    cells, h = (4, 4, 6), (0.25, 0.25, 0.2)
    ncell = 96
    bL = _u(ncell, 40)
    T = hermite.transform(P)
    T3 = np.kron(np.kron(T, T), T)
    bH = (bL.reshape(ncell, -1) @ T3).reshape(-1)          # T3^T b per cell
    with tpfdm.Plan.mesh(N, cells, h) as pl:
        pl.setup_inverse(tpfdm.OP_CELL)
        b1 = to_blocked(pl, bL, tpfdm.F64)
        x1 = torch.empty_like(b1)
        with tpfdm.PCG(pl) as s1:
            s1.solve(b1, x1, rtol=1e-12, maxit=5000)
        xL = from_blocked(pl, x1, tpfdm.F64)
    with _plan(cells, h) as ph:
        b2 = to_blocked(ph, bH, tpfdm.F64)
        x2 = torch.empty_like(b2)
        with tpfdm.PCG(ph) as s2:
            s2.solve(b2, x2, rtol=1e-12, maxit=5000)
        xn = torch.empty_like(x2)
        ph.change_basis(x2, xn, to_nodal=True)
        xH_nodal = from_blocked(ph, xn, tpfdm.F64)
    assert np.linalg.norm(xH_nodal - xL) <= 1e-9 * np.linalg.norm(xL)


@pytest.mark.parametrize("m,dt", [(128, tpfdm.F64), (64, tpfdm.F32)])
def test_full_size_sampled_cells(m, dt):
    """The benchmark meshes: the operator on sampled cells (corners, edges,
    random) against the oracle's row blocks in this basis."""
    torch = _torch()
    cells, h = (m,) * 3, (1.0 / m,) * 3
    rng = np.random.default_rng(m)
    ncell = m ** 3
    print(f"m={m} dt={tpfdm.DTYPE_NAMES[dt]}", flush=True)
    u = rng.uniform(-1, 1, ncell * 64)
    corners = [sipg.cell_index(cells, a, b, c) for a in (0, m - 1) for b in (0, m - 1) for c in (0, m - 1)]
    edges = [sipg.cell_index(cells, 0, m // 2, m - 1), sipg.cell_index(cells, m - 1, 0, m // 3)]
    sample = sorted(set(corners + edges + rng.choice(ncell, 24, replace=False).tolist()))
    with _plan(cells, h, setup=False) as plan:
        bu = to_blocked(plan, u, dt)
        bv = torch.empty_like(bu)
        plan.apply(bu, bv, op=tpfdm.OP_SIPG)
        v = from_blocked(plan, bv, dt).reshape(ncell, 64)[sample]
        del bu, bv
    uq = u.astype(np.float32).astype(np.float64) if dt == tpfdm.F32 else u
    ref = sipg.cell_apply(P, cells, h, uq, sample, bname=H)
    scale = 0.0
    ub = uq.reshape(ncell, 64)
    for c in sample:
        for nb, blk in sipg.cell_row_blocks(P, cells, h, c, bname=H):
            scale = max(scale, float(np.max(np.abs(blk) @ np.abs(ub[nb]))))
    err = np.abs(v - ref).max() / scale
    print(f"  sampled err={err:.2e}")
    assert err <= TOL[dt]


# ---------------------------------------------------------------- n >= 5 (one cell per wave)
# Degrees 4..7: the wave kernels on sign-flipped tables (the basis is
# centrosymmetric up to the sign of the derivative-at-1 function).
WAVE_CASES = [(4, (3, 2, 4), (0.25, 0.5, 1.0)), (5, (2, 3, 2), (1.0, 0.5, 0.7)),
              (6, (3, 1, 2), (0.4, 0.4, 0.9)), (7, (2, 3, 2), (0.7, 1.3, 0.45)), (7, (1, 1, 5), (0.5, 0.5, 0.5))]


def _plan_p(p, cells, h, setup=True):
    plan = tpfdm.Plan.mesh(p + 1, cells, h, basis=tpfdm.BASIS_HERMITE)
    if setup:
        plan.setup_inverse(tpfdm.OP_CELL)
    return plan


@pytest.mark.parametrize("p,cells,h", WAVE_CASES)
@pytest.mark.parametrize("dt", [tpfdm.F64, tpfdm.F32])
def test_wave_operators_match_oracle(p, cells, h, dt):
    torch = _torch()
    ncell = cells[0] * cells[1] * cells[2]
    u = np.random.default_rng(ncell + p).uniform(-1, 1, ncell * (p + 1) ** 3)
    print(f"p={p} cells={cells} dt={tpfdm.DTYPE_NAMES[dt]}", flush=True)
    with _plan_p(p, cells, h, setup=False) as plan:
        bu = to_blocked(plan, u, dt)
        for op, part in OPS[:2]:
            A = sipg.assemble(p, cells, h, part, bname=H)
            bv = torch.full_like(bu, float("nan"))
            plan.apply(bu, bv, op=op)
            got = from_blocked(plan, bv, dt)
            err = float(np.max(np.abs(got - A @ u)) / np.max(np.abs(abs(A) @ np.abs(u))))
            print(f"  op={op} err={err:.2e}")
            assert err <= TOL[dt]


@pytest.mark.parametrize("p", [4, 7])
def test_wave_change_basis_matches_oracle(p):
    torch = _torch()
    cells = (2, 2, 3)
    ncell = 12
    u = np.random.default_rng(p).uniform(-1, 1, ncell * (p + 1) ** 3)
    with _plan_p(p, cells, (0.5, 0.5, 0.3), setup=False) as plan:
        bu = to_blocked(plan, u, tpfdm.F64)
        bv = torch.full_like(bu, float("nan"))
        plan.change_basis(bu, bv, to_nodal=True)
        nodal = from_blocked(plan, bv, tpfdm.F64)
        bw = torch.full_like(bu, float("nan"))
        plan.change_basis(bu, bw, to_nodal=False)
        herm = from_blocked(plan, bw, tpfdm.F64)
    ref_n = hermite.to_lagrange(p, u, ncell)
    ref_h = hermite.to_hermite(p, u, ncell)
    assert np.abs(nodal - ref_n).max() <= 1e-13 * np.abs(ref_n).max()
    assert np.abs(herm - ref_h).max() <= 1e-11 * np.abs(ref_h).max()


@pytest.mark.parametrize("p,cells,h", [(4, (2, 3, 2), (0.5, 0.4, 0.6)), (7, (2, 2, 2), (0.5, 0.5, 0.5))])
@pytest.mark.parametrize("inner", [tpfdm.F64, tpfdm.F32])
def test_wave_pcg_matches_oracle(p, cells, h, inner):
    """Block-Jacobi PCG in the Hermite-type basis with the wave kernels: the
    oracle's iteration count in FP64 (same recurrences), the true residual.
    The right-hand side is the load of a random nodal vector, b = T3^T b_L
    (a random vector taken directly as Hermite-basis data is a wildly
    oscillating load at high degree: its solution's coefficients reach 1e16
    at p = 7 and no FP64 residual is meaningful against it)."""
    torch = _torch()
    ncell = cells[0] * cells[1] * cells[2]
    bL = np.random.default_rng(7 * p).uniform(-1, 1, ncell * (p + 1) ** 3)
    T = hermite.transform(p)
    b = (bL.reshape(ncell, -1) @ np.kron(np.kron(T, T), T)).reshape(-1)
    A = sipg.assemble(p, cells, h, bname=H)
    rtol = 1e-10
    _, ito, _ = sipg.pcg(A, b, lambda r: sipg.block_jacobi(p, cells, h, r, bname=H), rtol, 5000)
    with _plan_p(p, cells, h) as plan, tpfdm.PCG(plan) as solver:
        bb = to_blocked(plan, b, tpfdm.F64)
        bx = torch.full_like(bb, float("nan"))
        s = solver.solve(bb, bx, inner=inner, rtol=rtol, maxit=5000, check_every=8)
        x = from_blocked(plan, bx, tpfdm.F64)
    print(f"p={p} inner={tpfdm.DTYPE_NAMES[inner]} oracle_iters={ito} {s}")
    assert s["converged"] and np.linalg.norm(b - A @ x) <= 2 * rtol * np.linalg.norm(b)
    if inner == tpfdm.F64:
        assert abs(s["iterations"] - ito) <= 1
    else:
        # the basis' mass matrix is ill-conditioned at high degree (about
        # 1.8e6 at p = 7), so an FP32 block inverse is a coarser
        # preconditioner here than in the Lagrange basis: measured 86 vs 85
        # iterations at p = 4 and 109 vs 96 at p = 7
        assert ito - 1 <= s["iterations"] <= int(1.25 * ito) + 3


def test_wave_block_calls_are_rejected():
    """n >= 5 in the Hermite-type basis serves the coupled operator, PCG and
    the change of basis; block calls and multigrid say so."""
    torch = _torch()
    with _plan_p(5, (2, 2, 2), (0.5, 0.5, 0.5)) as plan:
        buf = torch.zeros(plan.vector_elems, dtype=torch.float64, device="cuda")
        for call in (lambda: plan.apply(buf, torch.zeros_like(buf), tpfdm.OP_NEUMANN),
                     lambda: plan.apply_inverse(buf, torch.zeros_like(buf)),
                     lambda: plan.solve(buf, torch.zeros_like(buf)),
                     lambda: tpfdm.MG(plan)):
            with pytest.raises(tpfdm.TpfdmError) as e:
                call()
            assert e.value.status == -2


def test_wave_full_size_sampled_cells():
    """p = 7 on 64^3 cells (134 M DoF, the benchmark mesh of the wave
    kernels) in FP64: sampled cells (corners, edges, random) against the
    oracle's row blocks in this basis."""
    torch = _torch()
    p, m = 7, 64
    n3 = (p + 1) ** 3
    cells, h = (m,) * 3, (1.0 / m,) * 3
    ncell = m ** 3
    rng = np.random.default_rng(77)
    u = rng.uniform(-1, 1, ncell * n3)
    corners = [sipg.cell_index(cells, a, b, c) for a in (0, m - 1) for b in (0, m - 1) for c in (0, m - 1)]
    sample = sorted(set(corners + rng.choice(ncell, 12, replace=False).tolist()))
    print(f"p={p} m={m}", flush=True)
    with _plan_p(p, cells, h, setup=False) as plan:
        bu = to_blocked(plan, u, tpfdm.F64)
        bv = torch.empty_like(bu)
        plan.apply(bu, bv, op=tpfdm.OP_SIPG)
        v = from_blocked(plan, bv, tpfdm.F64).reshape(ncell, n3)[sample]
        del bu, bv
    ub = u.reshape(ncell, n3)
    ref = np.zeros((len(sample), n3))
    scale = 0.0
    for r, c in enumerate(sample):
        for nb, blk in sipg.cell_row_blocks(p, cells, h, c, bname=H):
            ref[r] += blk @ ub[nb]
            scale = max(scale, float(np.max(np.abs(blk) @ np.abs(ub[nb]))))
    err = np.abs(v - ref).max() / scale
    print(f"  sampled err={err:.2e}")
    assert err <= TOL[tpfdm.F64]
