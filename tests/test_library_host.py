"""Host-side checks of libtpfdm that need no GPU: the library loads and
exports every symbol its header declares, its host reference data agree with
the oracle, and argument validation fails cleanly."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import basis
from paper_2609_04534_amd import tpfdm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "tpfdm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = tpfdm.load()
    declared = _header_functions()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(tpfdm.EXPORTS) == declared


def test_version_string():
    assert "gfx950" in tpfdm.version()


@pytest.mark.parametrize("n", range(2, 9))
@pytest.mark.parametrize("C", [1.0, 2.0, 3.5])
def test_reference_matrices_match_oracle(n, C):
    M, K, A = tpfdm.reference_matrices(n, C)
    Mo, Ko = basis.mass_stiffness(n - 1)
    Ao = basis.penalized_stiffness(n - 1, C)
    scale = np.abs(Ao).max()
    assert np.abs(M - Mo).max() < 1e-15
    assert np.abs(K - Ko).max() < 1e-14 * np.abs(Ko).max()
    assert np.abs(A - Ao).max() < 1e-14 * scale


@pytest.mark.parametrize("n", range(2, 9))
def test_reference_eigen_properties(n):
    import scipy.linalg as sl
    M, K, A = tpfdm.reference_matrices(n)
    S, lam = tpfdm.reference_eigen(n, 2.0, tpfdm.OP_CELL)
    assert np.all(np.diff(lam) > 0)
    assert np.abs(S.T @ M @ S - np.eye(n)).max() < 1e-13
    assert np.abs(S.T @ A @ S - np.diag(lam)).max() < 1e-13 * lam.max()
    lam_o = sl.eigh(basis.penalized_stiffness(n - 1), basis.mass_stiffness(n - 1)[0], eigvals_only=True)
    assert np.allclose(lam, lam_o, rtol=1e-12)
    # sign convention: largest-magnitude entry of every column is positive
    idx = np.argmax(np.abs(S), axis=0)
    assert np.all(S[idx, np.arange(n)] > 0)
    # Neumann: the constant is an eigenvector of eigenvalue 0
    Sn, lamn = tpfdm.reference_eigen(n, 2.0, tpfdm.OP_NEUMANN)
    assert abs(lamn[0]) < 1e-10 * lamn[-1]


def test_reference_argument_errors():
    lib = tpfdm.load()
    buf = np.zeros(100)
    assert lib.tp_reference_matrices(1, 2.0, buf.ctypes.data, None, None) == -2
    assert lib.tp_reference_matrices(9, 2.0, buf.ctypes.data, None, None) == -2
    assert lib.tp_reference_matrices(3, -1.0, buf.ctypes.data, None, None) == -1
    assert lib.tp_reference_eigen(3, 2.0, 7, buf.ctypes.data, buf.ctypes.data) == -1
    assert lib.tp_reference_eigen(3, 2.0, 1, None, buf.ctypes.data) == -1
    assert "null" in lib.tp_last_error().decode()


def _create(groups, opts=None):
    lib = tpfdm.load()
    arr = (tpfdm._Group * max(1, len(groups)))()
    keep = []
    for i, (n, B, nb, off) in enumerate(groups):
        h = np.ones((max(nb, 1), 3))
        keep.append(h)
        arr[i].n, arr[i].layout_B, arr[i].nblocks, arr[i].h, arr[i].offset = n, B, nb, h.ctypes.data, off
    out = ctypes.c_void_p()
    st = lib.tp_plan_create(arr, len(groups), opts, ctypes.byref(out))
    if st == 0:
        lib.tp_plan_destroy(out)
    return st


def test_plan_argument_validation_before_device():
    assert _create([(9, 64, 10, 0)]) == -2          # n out of range
    assert _create([(1, 64, 10, 0)]) == -2
    assert _create([(3, 48, 10, 0)]) == -1          # B not a power of two
    assert _create([(3, 2048, 10, 0)]) == -1        # B too large
    assert _create([(3, 64, -1, 0)]) == -1          # negative count
    assert _create([(3, 64, 10, -5)]) == -1         # negative offset
    # overlapping ranges: 64 * 27 elements from 0, second group starts inside
    assert _create([(3, 64, 10, 0), (4, 64, 10, 100)]) == -1
    opts = tpfdm._Opts()
    tpfdm.load().tp_plan_opts_default(ctypes.byref(opts))
    opts.penalty_C = float("nan")
    assert _create([(3, 64, 10, 0)], ctypes.byref(opts)) == -1
    opts.penalty_C = 2.0
    opts.reserved[3] = 1
    assert _create([(3, 64, 10, 0)], ctypes.byref(opts)) == -1
    opts.reserved[3] = 0
    opts.mapping = 3
    assert _create([(3, 64, 10, 0)], ctypes.byref(opts)) == -1


def test_null_plan_calls_fail_cleanly():
    lib = tpfdm.load()
    assert lib.tp_apply(None, 0, None, None, 0, None) == -1
    assert lib.tp_apply_inverse(None, None, None, 0, None) == -1
    assert lib.tp_setup_inverse(None, 1, 0, 0.0) == -1
    assert lib.tp_solve(None, None, None, 1, 1e-10, 10, None, None, None, None) == -1
    assert lib.tp_pack(None, None, None, 0, None) == -1
    assert lib.tp_plan_destroy(None) == 0
    assert lib.tp_plan_vector_elems(None) == -1


def test_no_device_gives_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _create([(3, 64, 10, 0)]) == -7
    assert "hip" in tpfdm.load().tp_last_error().decode().lower()


def _create_factor(n, nb, with_h=False, only_M=False, persistent=False):
    lib = tpfdm.load()
    arr = (tpfdm._Group * 1)()
    M = np.tile(np.eye(n), (nb, 3, 1, 1))
    h = np.ones((nb, 3))
    arr[0].n, arr[0].layout_B, arr[0].nblocks, arr[0].offset = n, 1, nb, 0
    arr[0].h = h.ctypes.data if with_h else None
    arr[0].M = M.ctypes.data
    arr[0].P = None if only_M else M.ctypes.data
    opts = tpfdm._Opts()
    lib.tp_plan_opts_default(ctypes.byref(opts))
    opts.persistent = 1 if persistent else 0
    out = ctypes.c_void_p()
    st = lib.tp_plan_create(arr, 1, ctypes.byref(opts), ctypes.byref(out))
    if st == 0:
        lib.tp_plan_destroy(out)
    return st


def test_factor_group_validation_before_device():
    assert _create_factor(3, 4, only_M=True) == -1       # M without P
    assert _create_factor(3, 4, with_h=True) == -1       # factors and h together
    assert _create_factor(3, 4, persistent=True) == -2   # persistent plans take no factor groups


def test_setup_inverse_rejects_unknown_mode():
    lib = tpfdm.load()
    assert lib.tp_setup_inverse(None, 1, 7, 0.0) == -1


def _create_mesh(n=3, B=64, cells=(2, 3, 4), h=(0.5, 1.0, 0.25), basis=0, persistent=0, mapping=0):
    lib = tpfdm.load()
    m = tpfdm._Mesh()
    m.n = n
    m.layout_B = B
    for d in range(3):
        m.cells[d] = cells[d]
        m.h[d] = h[d]
    m.basis = basis
    opts = tpfdm._Opts()
    lib.tp_plan_opts_default(ctypes.byref(opts))
    opts.persistent = persistent
    opts.mapping = mapping
    out = ctypes.c_void_p()
    return lib.tp_plan_create_mesh(ctypes.byref(m), ctypes.byref(opts), ctypes.byref(out))


def test_mesh_plan_validation_before_device():
    assert _create_mesh(cells=(0, 3, 4)) == -1
    assert _create_mesh(cells=(2, -1, 4)) == -1
    assert _create_mesh(h=(0.5, 0.0, 1.0)) == -1
    assert _create_mesh(h=(0.5, float("nan"), 1.0)) == -1
    assert _create_mesh(basis=2) == -1                        # no such basis
    assert _create_mesh(basis=-1) == -1
    assert _create_mesh(n=3, basis=tpfdm.BASIS_HERMITE) == -2   # Hermite-type basis: p >= 3
    assert _create_mesh(n=2, basis=tpfdm.BASIS_HERMITE) == -2
    assert _create_mesh(n=4, basis=tpfdm.BASIS_HERMITE, mapping=tpfdm.MAP_WAVE) == -2
    assert _create_mesh(cells=(2048, 2048, 1024)) == -1       # 2^32 cells
    assert _create_mesh(persistent=1) == -2
    lib = tpfdm.load()
    assert lib.tp_plan_create_mesh(None, None, None) == -1


def test_patch_blocks_validation_before_device():
    lib = tpfdm.load()
    opts = tpfdm._Opts()
    lib.tp_plan_opts_default(ctypes.byref(opts))
    assert opts.blocks == tpfdm.BLOCKS_CELLS
    opts.blocks = 2
    assert _create([(4, 64, 10, 0)], ctypes.byref(opts)) == -1          # no such block kind
    opts.blocks = tpfdm.BLOCKS_PATCHES
    for n in (2, 3, 5, 7):                                               # patches have n = 2 (p+1) >= 4
        assert _create([(n, 64, 10, 0)], ctypes.byref(opts)) == -2
    m = tpfdm._Mesh()
    m.n, m.layout_B = 4, 64
    for d in range(3):
        m.cells[d], m.h[d] = 2, 0.5
    out = ctypes.c_void_p()
    assert lib.tp_plan_create_mesh(ctypes.byref(m), ctypes.byref(opts), ctypes.byref(out)) == -2


@pytest.mark.parametrize("n,C", [(4, 2.0), (4, 3.5), (5, 2.0), (6, 2.0), (7, 2.0), (8, 2.0)])
def test_hermite_reference_tables_match_oracle(n, C):
    """The library's own Hermite-type tables (host code, no GPU) against the
    oracle's, two independent implementations of the basis of
    eq. (hermite_conditions)."""
    from oracle import hermite
    p = n - 1
    M, K, A, T = tpfdm.reference_basis(n, tpfdm.BASIS_HERMITE, penalty_C=C)
    Mo, Ko = hermite.mass_stiffness(p)
    Ao = hermite.penalized_stiffness(p, C)
    assert np.allclose(M, Mo, atol=1e-13 * np.abs(Mo).max())
    assert np.allclose(K, Ko, atol=1e-12 * np.abs(Ko).max())
    assert np.allclose(A, Ao, atol=1e-12 * np.abs(Ao).max())
    assert np.allclose(T, hermite.transform(p), atol=1e-13)
    # conjugated by the sign of the derivative-at-1 function the matrices are
    # centrosymmetric (what the even-odd kernels of n >= 5 rely on)
    d = np.ones(n)
    d[n - 2] = -1.0
    J = np.eye(n)[::-1]
    for X in (M, K, A):
        Xf = d[:, None] * X * d[None, :]
        assert np.allclose(J @ Xf @ J, Xf, atol=1e-12 * np.abs(X).max())


@pytest.mark.parametrize("n", [4, 6, 8])
def test_patch_reference_tables_match_oracle(n):
    from oracle import patch
    M, K, A, T = tpfdm.reference_basis(n, blocks=tpfdm.BLOCKS_PATCHES)
    Mo, Ko, Ao = patch.patch_factors(n // 2 - 1)
    assert np.allclose(M, Mo, atol=1e-14)
    assert np.allclose(K, Ko, atol=1e-12 * np.abs(Ko).max())
    assert np.allclose(A, Ao, atol=1e-12 * np.abs(Ao).max())
    assert np.array_equal(T, np.eye(n))


def test_reference_basis_errors():
    lib = tpfdm.load()
    assert lib.tp_reference_basis(3, tpfdm.BASIS_HERMITE, 0, 2.0, None, None, None, None) == -2
    assert lib.tp_reference_basis(6, tpfdm.BASIS_HERMITE, tpfdm.BLOCKS_PATCHES, 2.0, None, None, None, None) == -2
    assert lib.tp_reference_basis(5, 0, tpfdm.BLOCKS_PATCHES, 2.0, None, None, None, None) == -2
    assert lib.tp_reference_basis(4, 7, 0, 2.0, None, None, None, None) == -1
    assert lib.tp_reference_basis(4, 0, 3, 2.0, None, None, None, None) == -1
    assert lib.tp_reference_basis(4, 0, 0, -1.0, None, None, None, None) == -1
