"""Pins of the whole-batch oracle forms and of the sum-factorized CPU
reference against the plain per-block dense oracle (CPU only).

The per-block dense oracle (``dense.apply`` / ``dense.solve``) is pinned by
closed forms, brute-force quadrature and the paper's printed stencil in the
other oracle tests; the faster forms used for checks at full size must equal
it on random anisotropic blocks of every degree.
"""
import numpy as np
import pytest

from oracle import dense, sumfact


def _blocks(p, k, seed, lo=0.5, hi=4.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (k, 3)), rng.uniform(-1.0, 1.0, (k, (p + 1) ** 3))


def _rel(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("op", [dense.NEUMANN, dense.CELL])
def test_apply_batch_equals_per_block_dense(p, op):
    h, u = _blocks(p, 9, seed=p)
    assert _rel(dense.apply_batch(p, h, u, op), dense.apply(p, h, u, op)) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 7])
def test_solve_batch_equals_per_block_dense(p):
    h, r = _blocks(p, 5, seed=10 + p)
    x = dense.solve_batch(p, h, r, chunk=2)
    assert _rel(x, dense.solve(p, h, r)) < 1e-14
    # several right-hand sides per block share one factorization
    r2 = np.stack([r, 2.0 * r[::-1]], axis=2)
    x2 = dense.solve_batch(p, h, r2, chunk=3)
    assert _rel(x2[:, :, 0], x) < 1e-14
    assert _rel(x2[:, :, 1], dense.solve(p, h, 2.0 * r[::-1])) < 1e-14
    # and the residual of the batch form vanishes
    res = dense.residual_batch(p, h, x, r)
    assert float(np.max(np.abs(res))) < 1e-12 * float(np.max(np.abs(r)))


def test_apply_batch_absolute_bounds_the_product():
    p = 3
    h, u = _blocks(p, 7, seed=3)
    v = dense.apply_batch(p, h, u)
    w = dense.apply_batch(p, h, np.abs(u), absolute=True)
    assert np.all(np.abs(v) <= w * (1 + 1e-14))


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("op", [dense.NEUMANN, dense.CELL])
def test_sumfact_apply_equals_dense(p, op):
    h, u = _blocks(p, 11, seed=20 + p)
    assert _rel(sumfact.apply(p, h, u, op), dense.apply(p, h, u, op)) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7])
def test_sumfact_inverse_equals_dense_solve(p):
    h, r = _blocks(p, 11, seed=30 + p)
    kappa = max(dense.condition_number(p, hb) for hb in h[:3])
    assert _rel(sumfact.inverse(p, h, r), dense.solve(p, h, r)) < max(1e-13, 10 * kappa * 2.2e-16)


def test_sumfact_inverse_of_neumann_is_singular_mode():
    # the Neumann pair has a zero eigenvalue: the scaling divides by zero for
    # the constant mode, so the reference is only meaningful for the cell block
    S, lam = sumfact.eigenpairs(3, dense.NEUMANN)
    assert abs(lam[0]) < 1e-12


def test_sumfact_mutation_transposed_eigenvectors_is_caught():
    """A plausible slip (S instead of S^T in the first contraction) must fail
    the comparison with the dense solve."""
    p = 3
    h, r = _blocks(p, 4, seed=40)
    S, lam = sumfact.eigenpairs(p)
    n = p + 1
    rb = r.reshape(-1, n, n, n)
    sx, sy, sz = (1.0 / np.sqrt(h[:, d])[:, None, None, None] for d in range(3))
    y = np.einsum("kc,bijc->bijk", S, rb) * sz          # mutated: S applied, not S^T
    y = np.einsum("cj,bick->bijk", S, y) * sy
    y = np.einsum("ci,bcjk->bijk", S, y) * sx
    L = (lam[None, :, None, None] / h[:, 0, None, None, None] ** 2 + lam[None, None, :, None] / h[:, 1, None, None, None] ** 2
         + lam[None, None, None, :] / h[:, 2, None, None, None] ** 2)
    y = y / L
    x = np.einsum("ic,bcjk->bijk", S, y) * sx
    x = np.einsum("jc,bick->bijk", S, x) * sy
    x = np.einsum("kc,bijc->bijk", S, x) * sz
    assert _rel(x.reshape(len(h), -1), dense.solve(p, h, r)) > 1e-3
