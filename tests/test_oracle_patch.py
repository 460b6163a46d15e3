"""Pins of the vertex-patch oracle (oracle/patch.py): the patch block built
from its 1D factors equals the corresponding rows and columns of the
assembled mesh operator, and has the symmetries the kernels rely on."""
import numpy as np
import pytest

from oracle import dense, patch, sipg


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("op,part", [(dense.CELL, sipg.FULL), (dense.NEUMANN, sipg.VOLUME)])
def test_patch_block_is_the_restricted_mesh_operator(p, op, part):
    """For a patch away from the boundary, the eight cells' rows and columns
    of the assembled SIPG operator (and of its volume part) are the Kronecker
    sum of the 1D patch factors: two routes to the same matrix."""
    m, h = (4, 5, 4), (0.3, 0.2, 0.45)
    A = sipg.assemble(p, m, h, part).toarray()
    idx = patch.patch_dofs(p, m, (1, 2, 1))
    ref = A[np.ix_(idx, idx)]
    got = patch.patch_operator(p, h, op)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_patch_factors_symmetric_definite_and_reflection_invariant(p):
    Mp, Kp, Ap = patch.patch_factors(p)
    J = np.eye(2 * (p + 1))[::-1]
    for X in (Mp, Kp, Ap):
        assert np.allclose(X, X.T, atol=1e-13 * np.abs(X).max())
        assert np.allclose(J @ X @ J, X, atol=1e-12 * np.abs(X).max())
    assert np.linalg.eigvalsh(Mp).min() > 0 and np.linalg.eigvalsh(Ap).min() > 0
    # the broken stiffness annihilates constants on each cell
    assert np.abs(Kp @ np.ones(2 * (p + 1))).max() < 1e-11
