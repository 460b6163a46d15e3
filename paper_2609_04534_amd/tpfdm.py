"""Thin ctypes binding of libtpfdm (include/tpfdm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the shared library.  Torch tensors supply device memory and
streams.  There is no fallback: when the library is missing or fails to load
every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpfdm.so")

TP_OK = 0
STATUS = {
    0: "TP_OK", -1: "TP_ERR_ARG", -2: "TP_ERR_UNSUPPORTED", -3: "TP_ERR_NOT_SPD",
    -4: "TP_ERR_SINGULAR", -5: "TP_ERR_NOT_CONVERGED", -6: "TP_ERR_NONFINITE",
    -7: "TP_ERR_HIP", -8: "TP_ERR_OOM", -9: "TP_ERR_STATE", 1: "TP_PENDING",
}
TP_PENDING = 1
F64, F32, F16, BF16 = 0, 1, 2, 3
DTYPE_NAMES = {F64: "f64", F32: "f32", F16: "f16", BF16: "bf16"}
OP_NEUMANN, OP_CELL, OP_SIPG, OP_SIPG_FACE = 0, 1, 2, 3
FACTOR_SCALED, FACTOR_GENERAL = 0, 1
MAP_AUTO, MAP_LANE, MAP_WAVE = 0, 1, 2
BASIS_LAGRANGE, BASIS_HERMITE = 0, 1
BLOCKS_CELLS, BLOCKS_PATCHES = 0, 1
PCG_RESIDUAL, PCG_PRECONDITIONED = 0, 1

# The public symbol set declared in include/tpfdm.h.
EXPORTS = (
    "tp_plan_opts_default", "tp_plan_create", "tp_plan_destroy", "tp_plan_vector_elems",
    "tp_plan_ndof", "tp_plan_nblocks", "tp_apply", "tp_setup_inverse", "tp_apply_inverse",
    "tp_solve", "tp_pack", "tp_unpack", "tp_reference_matrices", "tp_reference_eigen",
    "tp_last_error", "tp_version", "tp_solve_summary_fetch", "tp_graph_create", "tp_graph_launch",
    "tp_graph_destroy", "tp_plan_autotune", "tp_plan_group_kernel", "tp_plan_create_mesh",
    "tp_pcg_create", "tp_pcg_solve", "tp_pcg_destroy", "tp_pcg_begin", "tp_pcg_poll",
    "tp_mg_create", "tp_mg_vcycle", "tp_mg_destroy", "tp_pcg_set_multigrid", "tp_change_basis",
    "tp_pcg_set_norm", "tp_reference_basis", "tp_solve_static", "tp_mg_create_typed",
)
KIND_NAMES = {0: "lane", 1: "wave", 2: "mfma", 3: "general"}
GRAPH_APPLY, GRAPH_INVERSE, GRAPH_SOLVE = 0, 1, 2


class TpfdmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class _Group(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("layout_B", ctypes.c_int32), ("nblocks", ctypes.c_int64),
                ("h", ctypes.c_void_p), ("offset", ctypes.c_int64), ("M", ctypes.c_void_p),
                ("P", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("penalty_C", ctypes.c_double), ("persistent", ctypes.c_int32),
                ("mapping", ctypes.c_int32), ("blocks", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class _Mesh(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("layout_B", ctypes.c_int32), ("cells", ctypes.c_int32 * 3),
                ("basis", ctypes.c_int32), ("h", ctypes.c_double * 3)]


class _PcgSummary(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("relres", ctypes.c_double)]


class _Summary(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("n_failed", ctypes.c_int32),
                ("max_relres", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libtpfdm.so (built in-tree by paper_2609_04534_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libtpfdm.so not found at {path}; run `python -m paper_2609_04534_amd.build`")
    # torch's ROCm libraries are loaded first, so that the library's HIP
    # runtime finds the HSA runtime the tensors it is handed come from
    # (loaded the other way round, the library saw no device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "tp_plan_opts_default": (None, [ctypes.POINTER(_Opts)]),
        "tp_plan_create": (i32, [ctypes.POINTER(_Group), i32, ctypes.POINTER(_Opts), ctypes.POINTER(vp)]),
        "tp_plan_destroy": (i32, [vp]),
        "tp_plan_vector_elems": (i64, [vp]),
        "tp_plan_ndof": (i64, [vp]),
        "tp_plan_nblocks": (i64, [vp]),
        "tp_apply": (i32, [vp, i32, vp, vp, i32, vp]),
        "tp_setup_inverse": (i32, [vp, i32, i32, dbl]),
        "tp_apply_inverse": (i32, [vp, vp, vp, i32, vp]),
        "tp_solve": (i32, [vp, vp, vp, i32, dbl, i32, vp, vp, ctypes.POINTER(_Summary), vp]),
        "tp_solve_static": (i32, [vp, vp, vp, i32, dbl, i32, vp, vp, ctypes.POINTER(_Summary), vp]),
        "tp_pack": (i32, [vp, vp, vp, i32, vp]),
        "tp_unpack": (i32, [vp, vp, vp, i32, vp]),
        "tp_reference_matrices": (i32, [i32, dbl, vp, vp, vp]),
        "tp_reference_eigen": (i32, [i32, dbl, i32, vp, vp]),
        "tp_last_error": (ctypes.c_char_p, []),
        "tp_solve_summary_fetch": (i32, [vp, ctypes.POINTER(_Summary), vp]),
        "tp_graph_create": (i32, [vp, i32, i32, i32, vp, vp, dbl, i32, vp, vp, ctypes.POINTER(vp)]),
        "tp_graph_launch": (i32, [vp, vp]),
        "tp_graph_destroy": (i32, [vp]),
        "tp_version": (ctypes.c_char_p, []),
        "tp_plan_autotune": (i32, [vp, i32, i32, vp]),
        "tp_plan_group_kernel": (i32, [vp, i32, i32, i32]),
        "tp_plan_create_mesh": (i32, [ctypes.POINTER(_Mesh), ctypes.POINTER(_Opts), ctypes.POINTER(vp)]),
        "tp_pcg_create": (i32, [vp, ctypes.POINTER(vp)]),
        "tp_pcg_solve": (i32, [vp, vp, vp, i32, i32, dbl, i32, i32, ctypes.POINTER(_PcgSummary), vp]),
        "tp_pcg_destroy": (i32, [vp]),
        "tp_pcg_begin": (i32, [vp, vp, vp, i32, i32, dbl, i32, i32, vp]),
        "tp_pcg_poll": (i32, [vp, ctypes.POINTER(_PcgSummary)]),
        "tp_mg_create": (i32, [vp, ctypes.POINTER(vp)]),
        "tp_mg_create_typed": (i32, [vp, i32, ctypes.POINTER(vp)]),
        "tp_mg_vcycle": (i32, [vp, vp, vp, vp]),
        "tp_mg_destroy": (i32, [vp]),
        "tp_pcg_set_multigrid": (i32, [vp, vp]),
        "tp_change_basis": (i32, [vp, i32, vp, vp, vp]),
        "tp_pcg_set_norm": (i32, [vp, i32]),
        "tp_reference_basis": (i32, [i32, i32, i32, dbl, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != TP_OK:
        msg = load().tp_last_error().decode(errors="replace")
        raise TpfdmError(status, msg)


def version() -> str:
    return load().tp_version().decode()


def reference_matrices(n: int, penalty_C: float = 2.0):
    """(M_hat, K_hat, A_hat) of the n-point GLL basis, computed by the library's host code."""
    M = np.zeros((n, n))
    K = np.zeros((n, n))
    A = np.zeros((n, n))
    _check(load().tp_reference_matrices(n, penalty_C, M.ctypes.data, K.ctypes.data, A.ctypes.data))
    return M, K, A


def reference_basis(n: int, basis: int = BASIS_LAGRANGE, blocks: int = BLOCKS_CELLS, penalty_C: float = 2.0):
    """(M_hat, K_hat, A_hat, T) a plan with this basis and block kind uses
    (tp_reference_basis), computed by the library's host code."""
    out = [np.zeros((n, n)) for _ in range(4)]
    _check(load().tp_reference_basis(n, basis, blocks, penalty_C, *(a.ctypes.data for a in out)))
    return tuple(out)


def reference_eigen(n: int, penalty_C: float = 2.0, op: int = OP_CELL):
    """(S_hat, lam_hat) with P_hat S = M_hat S diag(lam), S^T M_hat S = I."""
    S = np.zeros((n, n))
    lam = np.zeros(n)
    _check(load().tp_reference_eigen(n, penalty_C, op, S.ctypes.data, lam.ctypes.data))
    return S, lam


def torch_dtype_code(t) -> int:
    import torch
    m = {torch.float64: F64, torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


@dataclass
class GroupSpec:
    """One group: n points per direction, interleave width B, and either edge
    lengths h (nblocks, 3) or per-block factors M, P (nblocks, 3, n, n)."""
    n: int
    layout_B: int
    h: object            # numpy (host) or torch tensor (host or device), float64 [nblocks, 3]; None with M, P
    offset: int = -1     # element offset; -1 = place after the previous group
    M: object = None     # factor group: float64 [nblocks, 3, n, n] mass factors
    P: object = None     # factor group: float64 [nblocks, 3, n, n] operator factors

    @property
    def nblocks(self) -> int:
        return int((self.h if self.h is not None else self.M).shape[0])

    def elems(self) -> int:
        t = (self.nblocks + self.layout_B - 1) // self.layout_B
        return t * self.n ** 3 * self.layout_B


def default_layout_B(n: int) -> int:
    """Interleave width used by default: 64 (one wave of lanes) for the
    lane-per-block kernels (n <= 4), 1 (block-contiguous) otherwise."""
    return 64 if n <= 4 else 1


class Plan:
    """Owning wrapper of a tp_plan."""

    def __init__(self, groups, penalty_C: float = 2.0, persistent: bool = False, mapping: int = MAP_AUTO,
                 blocks: int = BLOCKS_CELLS):
        lib = load()
        self._keep = []
        arr = (_Group * max(1, len(groups)))()
        off = 0
        self.groups = []
        def host_or_device(a):
            if a is None:
                return None
            if isinstance(a, np.ndarray):
                a = np.ascontiguousarray(a, dtype=np.float64)
                self._keep.append(a)
                return a.ctypes.data
            import torch  # torch tensor, host or device
            a = a.to(torch.float64).contiguous()
            self._keep.append(a)
            return a.data_ptr()

        for i, g in enumerate(groups):
            o = off if g.offset < 0 else g.offset
            arr[i].n = g.n
            arr[i].layout_B = g.layout_B
            arr[i].nblocks = g.nblocks
            arr[i].h = host_or_device(g.h)
            arr[i].offset = o
            arr[i].M = host_or_device(g.M)
            arr[i].P = host_or_device(g.P)
            off = o + g.elems()
            self.groups.append(GroupSpec(g.n, g.layout_B, g.h, o, g.M, g.P))
        opts = _Opts()
        lib.tp_plan_opts_default(ctypes.byref(opts))
        opts.penalty_C = penalty_C
        opts.persistent = 1 if persistent else 0
        opts.mapping = mapping
        opts.blocks = blocks
        handle = ctypes.c_void_p()
        _check(lib.tp_plan_create(arr, len(groups), ctypes.byref(opts), ctypes.byref(handle)))
        self._h = handle
        self._keep = []

    @classmethod
    def mesh(cls, n: int, cells, h, layout_B: int | None = None, penalty_C: float = 2.0,
             mapping: int = MAP_AUTO, basis: int = BASIS_LAGRANGE) -> "Plan":
        """Plan over a uniform box mesh of cells[0] x cells[1] x cells[2] cells
        of edge lengths h (tp_plan_create_mesh): one group of blocks in mesh
        order, with the coupled operators OP_SIPG and OP_SIPG_FACE; basis is
        BASIS_LAGRANGE (nodal) or BASIS_HERMITE (n = 4)."""
        lib = load()
        B = default_layout_B(n) if layout_B is None else layout_B
        m = _Mesh()
        m.n = n
        m.layout_B = B
        for d in range(3):
            m.cells[d] = int(cells[d])
            m.h[d] = float(h[d])
        m.basis = basis
        opts = _Opts()
        lib.tp_plan_opts_default(ctypes.byref(opts))
        opts.penalty_C = penalty_C
        opts.mapping = mapping
        handle = ctypes.c_void_p()
        _check(lib.tp_plan_create_mesh(ctypes.byref(m), ctypes.byref(opts), ctypes.byref(handle)))
        self = cls.__new__(cls)
        self._h = handle
        self._keep = []
        ncell = int(cells[0]) * int(cells[1]) * int(cells[2])
        self.groups = [GroupSpec(n, B, np.broadcast_to(np.asarray(h, dtype=np.float64), (ncell, 3)), 0)]
        self.cells = tuple(int(c) for c in cells)
        return self

    # ---------------------------------------------------------------- sizes
    @property
    def handle(self):
        if self._h is None:
            raise TpfdmError(-9, "plan destroyed")
        return self._h

    @property
    def vector_elems(self) -> int:
        return int(load().tp_plan_vector_elems(self.handle))

    @property
    def ndof(self) -> int:
        return int(load().tp_plan_ndof(self.handle))

    @property
    def nblocks(self) -> int:
        return int(load().tp_plan_nblocks(self.handle))

    # ---------------------------------------------------------------- ops
    def apply(self, u, v, op: int = OP_NEUMANN, stream=None):
        _check(load().tp_apply(self.handle, op, _ptr(u), _ptr(v), torch_dtype_code(u), _stream(stream)))

    def setup_inverse(self, op: int = OP_CELL, singular_tol: float = 0.0, mode: int | None = None):
        """Fast-diagonalization setup; mode defaults to GENERAL when the plan has
        factor groups, SCALED otherwise."""
        if mode is None:
            mode = FACTOR_GENERAL if any(g.M is not None for g in self.groups) else FACTOR_SCALED
        _check(load().tp_setup_inverse(self.handle, op, mode, singular_tol))

    def apply_inverse(self, r, x, stream=None):
        _check(load().tp_apply_inverse(self.handle, _ptr(r), _ptr(x), torch_dtype_code(r), _stream(stream)))

    def solve(self, b, x, inner: int = F32, rtol: float = 1e-10, maxit: int = 50, iters=None, relres=None,
              summary: bool = True, stream=None, raise_on_failure: bool = True, static: bool = False):
        """Returns the summary dict (or None when summary=False).  static=True
        calls tp_solve_static (no allocation; the library's static workspace)."""
        s = _Summary()
        fn = load().tp_solve_static if static else load().tp_solve
        st = fn(self.handle, _ptr(b), _ptr(x), inner, rtol, maxit, _ptr(iters), _ptr(relres),
                ctypes.byref(s) if summary else None, _stream(stream))
        if st != TP_OK and (raise_on_failure or st not in (-5, -6)):
            _check(st)
        if not summary:
            return None
        return {"status": STATUS[st], "max_iters": s.max_iters, "n_failed": s.n_failed,
                "max_relres": s.max_relres}

    def solve_summary(self, stream=None, raise_on_failure: bool = False):
        """Summary of the most recent solve (also one replayed from a graph)."""
        s = _Summary()
        st = load().tp_solve_summary_fetch(self.handle, ctypes.byref(s), _stream(stream))
        if st != TP_OK and (raise_on_failure or st not in (-5, -6)):
            _check(st)
        return {"status": STATUS[st], "max_iters": s.max_iters, "n_failed": s.n_failed,
                "max_relres": s.max_relres}

    def graph(self, what: int, inp, out, op: int = OP_NEUMANN, dtype: int | None = None, rtol: float = 1e-10,
              maxit: int = 50, iters=None, relres=None):
        """Capture one call into a replayable HIP graph (see tp_graph_create)."""
        if dtype is None:
            dtype = torch_dtype_code(inp) if what != GRAPH_SOLVE else F32
        h = ctypes.c_void_p()
        _check(load().tp_graph_create(self.handle, what, op, dtype, _ptr(inp), _ptr(out), rtol, maxit,
                                      _ptr(iters), _ptr(relres), ctypes.byref(h)))
        return Graph(h, self)

    def autotune(self, dtype: int = F64, reps: int = 10):
        """Time the kernel variants per group (tp_plan_autotune) and keep the
        fastest; returns [(apply_us, inverse_us, solve_us)] per group.  For a
        persistent plan the first entry holds the tuned single launch's times
        (solve: inner precision = dtype) and the others are -1."""
        us = (ctypes.c_double * (3 * max(1, len(self.groups))))()
        _check(load().tp_plan_autotune(self.handle, dtype, reps, us))
        return [tuple(us[3 * i:3 * i + 3]) for i in range(len(self.groups))]

    def kernel(self, group: int, call: int, dtype: int = F64, grid: bool = False) -> str:
        """Kernel family a call would use for a group: lane / wave / mfma / general
        (with grid=True, wave kernels also report their grid: full / half / tile)."""
        code = load().tp_plan_group_kernel(self.handle, group, call, dtype)
        name = KIND_NAMES.get(code & 15 if code >= 0 else code, "none")
        if grid and name == "wave" and call != 2:
            name += "/" + {1: "full", 2: "half", 0: "tile"}.get(code >> 4, "?")
        return name

    def launch_config(self, group: int, call: int, dtype: int = F64) -> dict:
        """A persistent plan's single-launch choice for a group
        (tp_plan_group_kernel): its tile body (lane / wave), tiles per
        workgroup, the position of its segment in the launch and, for the
        solve (call 2), the grid (full / half / item)."""
        code = load().tp_plan_group_kernel(self.handle, group, call, dtype)
        if code < 0:
            raise TpfdmError(-1, "no launch configuration (not a persistent plan, or invalid argument)")
        out = {"body": KIND_NAMES[code & 15], "tiles_per_workgroup": 1 << ((code >> 8) & 15),
               "position": (code >> 12) & 0xFFFF}
        if call == 2:
            out["grid"] = {1: "full", 2: "half", 0: "item"}.get((code >> 4) & 15, "?")
        return out

    def change_basis(self, u, v, to_nodal: bool = True, stream=None, loads: bool = False):
        """v = (T (x) T (x) T) u (to_nodal), its inverse (not to_nodal), or
        with loads=True the transpose T^T (x) T^T (x) T^T (a nodally assembled
        load vector to this basis), cell by cell (tp_change_basis), blocked
        FP64 device vectors."""
        mode = 2 if loads else (1 if to_nodal else 0)
        _check(load().tp_change_basis(self.handle, mode, _ptr(u), _ptr(v), _stream(stream)))

    def pack(self, canonical, blocked, stream=None):
        _check(load().tp_pack(self.handle, _ptr(canonical), _ptr(blocked), torch_dtype_code(canonical),
                              _stream(stream)))

    def unpack(self, blocked, canonical, stream=None):
        _check(load().tp_unpack(self.handle, _ptr(blocked), _ptr(canonical), torch_dtype_code(blocked),
                                _stream(stream)))

    def destroy(self):
        if self._h is not None:
            load().tp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


class PCG:
    """Preconditioned CG for the coupled SIPG system of a mesh plan (tp_pcg_*)."""

    def __init__(self, plan: "Plan"):
        h = ctypes.c_void_p()
        _check(load().tp_pcg_create(plan.handle, ctypes.byref(h)))
        self._h = h
        self.plan = plan
        self.mg = None

    def set_norm(self, norm: int):
        """Stopping test of later solves: PCG_RESIDUAL (||r|| <= rtol ||b||) or
        PCG_PRECONDITIONED (<r, z>^{1/2} reduced by rtol)."""
        _check(load().tp_pcg_set_norm(self._h, norm))

    def set_multigrid(self, mg: "MG | None"):
        """Precondition later solves with one V-cycle of mg (None: block-Jacobi)."""
        _check(load().tp_pcg_set_multigrid(self._h, mg.handle if mg is not None else None))
        self.mg = mg

    def solve(self, b, x, x_is_zero: bool = True, inner: int = F64, rtol: float = 1e-8, maxit: int = 1000,
              check_every: int = 16, stream=None, raise_on_failure: bool = True) -> dict:
        """Solve A x = b; returns {iterations, converged, relres, status}."""
        summ = _PcgSummary()
        st = load().tp_pcg_solve(self._h, _ptr(b), _ptr(x), 1 if x_is_zero else 0, inner, rtol, maxit,
                                 check_every, ctypes.byref(summ), _stream(stream))
        out = {"iterations": summ.iterations, "converged": bool(summ.converged), "relres": summ.relres,
               "status": st}
        if st != TP_OK and raise_on_failure:
            _check(st)
        return out

    def begin(self, b, x, x_is_zero: bool = True, inner: int = F64, rtol: float = 1e-8, maxit: int = 1000,
              check_every: int = 16, stream=None):
        """Enqueue a solve without waiting (tp_pcg_begin); drive it with poll()."""
        _check(load().tp_pcg_begin(self._h, _ptr(b), _ptr(x), 1 if x_is_zero else 0, inner, rtol, maxit,
                                   check_every, _stream(stream)))

    def poll(self, raise_on_failure: bool = True):
        """None while the solve runs (tp_pcg_poll), else the summary dict."""
        summ = _PcgSummary()
        st = load().tp_pcg_poll(self._h, ctypes.byref(summ))
        if st == TP_PENDING:
            return None
        out = {"iterations": summ.iterations, "converged": bool(summ.converged), "relres": summ.relres,
               "status": st}
        if st != TP_OK and raise_on_failure:
            _check(st)
        return out

    def destroy(self):
        if self._h is not None:
            load().tp_pcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


class MG:
    """Multigrid V-cycle for the coupled SIPG system of a mesh plan (tp_mg_*)."""

    def __init__(self, plan: "Plan", storage: int = F64):
        """storage: element type of the level vectors (F64, or F32 via
        tp_mg_create_typed)."""
        h = ctypes.c_void_p()
        if storage == F64:
            _check(load().tp_mg_create(plan.handle, ctypes.byref(h)))
        else:
            _check(load().tp_mg_create_typed(plan.handle, storage, ctypes.byref(h)))
        self._h = h
        self.plan = plan
        self.storage = storage

    @property
    def handle(self):
        return self._h

    def vcycle(self, b, x, stream=None):
        """x = V(b), blocked FP64 device vectors of the plan."""
        _check(load().tp_mg_vcycle(self._h, _ptr(b), _ptr(x), _stream(stream)))

    def destroy(self):
        if self._h is not None:
            load().tp_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


class Graph:
    """A captured call; launch() replays it on a stream."""

    def __init__(self, handle, plan):
        self._h = handle
        self._plan = plan   # keeps the plan alive while the graph exists

    def launch(self, stream=None):
        _check(load().tp_graph_launch(self._h, _stream(stream)))

    def destroy(self):
        if self._h is not None:
            load().tp_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def groups_for_workload(workload, layout_B=None):
    """GroupSpecs for a workloads.Workload (one group per degree, packed one
    after another)."""
    specs = []
    for g in workload.groups:
        B = layout_B(g.n) if callable(layout_B) else (layout_B or default_layout_B(g.n))
        specs.append(GroupSpec(n=g.n, layout_B=B, h=g.h))
    return specs
