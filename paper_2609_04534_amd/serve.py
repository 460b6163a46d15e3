"""Continuous-batching server for preconditioned-CG Poisson solves on box
meshes (the coupled SIPG system of mesh plans, solved by tp_pcg_*).

Requests arrive over time, each a mesh (degree p, m^3 unit-cube cells) and a
right-hand side already resident in device memory.  The server keeps every
admitted solve in flight on its own HIP stream and drives all of them from
one host loop with the non-blocking tp_pcg_begin / tp_pcg_poll calls, so the
kernels of different solves overlap on the GPU.  A request is admitted (in
arrival order) as soon as a solver slot for its mesh class is free or the
device-memory budget has room for a new one; finished solves return their
slot to a per-class free pool, and idle slots of other classes are released
when a new class needs the memory.  With multigrid on, the solves whose
coarsest level fits the dense coarse solve (uses_multigrid; every class of
the mix) are preconditioned by one V-cycle per iteration (tp_mg_*), the
others by block-Jacobi.  Marshalling and scheduling only: every step of a solve runs
in the library's kernels.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import tpfdm


@dataclass
class Request:
    rid: int
    p: int
    m: int
    arrival: float              # seconds from the start of the run
    b: object                   # device tensor, canonical order (ncells * n^3 FP64 values)
    x: object = None            # device tensor of the result (canonical), filled on completion
    start: float = -1.0         # admission time
    done: float = -1.0          # completion time
    summary: dict = field(default_factory=dict)
    rejected: bool = False      # its slot alone exceeds the memory budget: never run


class _Slot:
    """A solver and its blocked b, x buffers for one mesh class, on its own
    stream; with multigrid, the slot's own V-cycle object (its level vectors
    are scratch that concurrent solves must not share)."""

    def __init__(self, plan, p, m, multigrid, storage=tpfdm.F64):
        import torch
        self.plan = plan
        self.cls = (p, m)
        self.stream = torch.cuda.Stream()
        self.solver = tpfdm.PCG(plan)
        self.mg = None
        if multigrid:
            self.mg = tpfdm.MG(plan, storage)
            self.solver.set_multigrid(self.mg)
        E = plan.vector_elems
        self.b = torch.empty(E, dtype=torch.float64, device="cuda")
        self.x = torch.empty(E, dtype=torch.float64, device="cuda")
        self.req = None

    def destroy(self):
        self.solver.destroy()
        if self.mg is not None:
            self.mg.destroy()
        self.b = self.x = None


def uses_multigrid(p: int, m: int) -> bool:
    """The V-cycle covers a mesh when its coarsest level (the odd part of m
    cells per side) has at most 2048 unknowns for the dense solve, at degree
    p or, for p >= 4, on the degree-1 level the library adds on the same
    cells: every m of the mix for p = 2, 3 and 7."""
    odd = m
    while odd % 2 == 0:
        odd //= 2
    return odd ** 3 * (p + 1) ** 3 <= 2048 or (p >= 4 and odd ** 3 * 8 <= 2048)


def mg_storage(p: int, inner: int) -> int:
    """Element type of a slot's multigrid level vectors: FP32 when the solve's
    inner precision is below FP64, FP64 otherwise (every degree)."""
    return tpfdm.F32 if inner != tpfdm.F64 else tpfdm.F64


def mg_bytes(p: int, m: int, storage: int = tpfdm.F64) -> int:
    """Device memory of a V-cycle object on an m^3 cube: a residual vector on
    every level plus right-hand side and correction below the finest (the
    shared coarse inverse is not counted), in the level storage type."""
    n3 = (p + 1) ** 3
    B = tpfdm.default_layout_B(p + 1)
    es = 4 if storage == tpfdm.F32 else 8
    total, ml, first = 0, m, True
    while True:
        E = (ml ** 3 + B - 1) // B * B * n3
        total += (1 if first else 3) * E * es
        first = False
        if ml % 2:
            break
        ml //= 2
    return total


def slot_bytes(plan, p: int = None, m: int = None, multigrid: bool = False, storage: int = tpfdm.F64) -> int:
    """Device memory of one slot: the solver's five vectors and partials plus
    b and x, and the V-cycle's levels (of the given storage type) when it
    has one."""
    return _slot_bytes(plan.vector_elems, plan.nblocks, p, m, multigrid, storage)


def class_slot_bytes(p: int, m: int, multigrid: bool = False, storage: int = tpfdm.F64) -> int:
    """slot_bytes of the mesh class (p, m) in the default layout, computed
    without creating its plan."""
    n = p + 1
    B = tpfdm.default_layout_B(n)
    ncell = m ** 3
    return _slot_bytes((ncell + B - 1) // B * B * n ** 3, ncell, p, m, multigrid, storage)


def _slot_bytes(E, nblocks, p, m, multigrid, storage=tpfdm.F64):
    nwg = (nblocks + 63) // 64
    out = 7 * E * 8 + 3 * nwg * 8 + 256
    if multigrid:
        out += mg_bytes(p, m, storage)
    return out


class Server:
    def __init__(self, hbm_budget: int, inner: int = tpfdm.F32, rtol: float = 1e-8, maxit: int = 20000,
                 check_every: int = 8, max_inflight: int = 16, multigrid: bool = False):
        self.budget = int(hbm_budget)
        self.multigrid = multigrid      # one V-cycle as the preconditioner where it applies
        self.max_inflight = max_inflight
        self.inner = inner
        self.rtol = rtol
        self.maxit = maxit
        self.check_every = check_every
        self.plans = {}         # (p, m) -> plan with the cell-block inverse set up
        self.free = {}          # (p, m) -> [idle slots]
        self.used = 0           # bytes of live slots (busy and idle)
        self.busy = []
        self.max_concurrent = 0
        self.rejected = 0       # requests whose slot alone exceeds the budget

    def _plan(self, p, m):
        key = (p, m)
        if key not in self.plans:
            plan = tpfdm.Plan.mesh(p + 1, (m, m, m), (1.0 / m,) * 3)
            plan.setup_inverse(tpfdm.OP_CELL)
            self.plans[key] = plan
        return self.plans[key]

    def _slot_for(self, p, m):
        """An idle slot of the class, or a new one when the budget allows
        (releasing idle slots of other classes first); None when full."""
        key = (p, m)
        if self.free.get(key):
            return self.free[key].pop()
        mgc = self._mg(p, m)
        st = mg_storage(p, self.inner)
        need = slot_bytes(self._plan(p, m), p, m, mgc, st)
        for k in list(self.free):
            while self.used + need > self.budget and self.free[k]:
                s = self.free[k].pop()
                self.used -= slot_bytes(s.plan, *s.cls, s.mg is not None,
                                        s.mg.storage if s.mg is not None else tpfdm.F64)
                s.destroy()
        if self.used + need > self.budget:
            return None
        self.used += need
        return _Slot(self._plan(p, m), p, m, mgc, st)

    def _mg(self, p, m):
        return self.multigrid and uses_multigrid(p, m)

    def _class_bytes(self, p, m):
        return class_slot_bytes(p, m, self._mg(p, m), mg_storage(p, self.inner))

    def _admit(self, req, now):
        """True when the request leaves the queue: admitted, or rejected
        because its slot alone needs more than the whole budget (it could
        never run, and first-in-first-out admission would stall behind it)."""
        if self._class_bytes(req.p, req.m) > self.budget:
            req.rejected = True
            req.start = req.done = now
            req.summary = {"status": "rejected", "converged": False, "iterations": 0,
                           "reason": f"slot of {self._class_bytes(req.p, req.m)} bytes exceeds "
                                     f"the budget of {self.budget} bytes"}
            self.rejected += 1
            return True
        if len(self.busy) >= self.max_inflight:
            return False
        s = self._slot_for(req.p, req.m)
        if s is None:
            return False
        import torch
        with torch.cuda.stream(s.stream):
            s.plan.pack(req.b, s.b, stream=s.stream)
        s.solver.begin(s.b, s.x, x_is_zero=True, inner=self.inner, rtol=self.rtol, maxit=self.maxit,
                       check_every=4 if s.mg is not None else self.check_every, stream=s.stream)
        s.req = req
        req.start = now
        self.busy.append(s)
        self.max_concurrent = max(self.max_concurrent, len(self.busy))
        return True

    def _complete(self, s, summ):
        import torch
        req = s.req
        out = torch.empty(s.plan.ndof, dtype=torch.float64, device="cuda")
        s.plan.unpack(s.x, out, stream=s.stream)
        s.stream.synchronize()
        req.x = out
        req.done = time.perf_counter() - self.t0
        req.summary = summ
        s.req = None
        self.free.setdefault(s.cls, []).append(s)

    def run(self, requests):
        """Serve the requests (sorted by arrival) in real time; returns them
        with admission and completion times filled."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        i = 0
        waiting = []
        while i < len(reqs) or waiting or self.busy:
            now = time.perf_counter() - self.t0
            while i < len(reqs) and reqs[i].arrival <= now:
                waiting.append(reqs[i])
                i += 1
            while waiting and self._admit(waiting[0], now):
                waiting.pop(0)
            progressed = False
            for s in list(self.busy):
                summ = s.solver.poll(raise_on_failure=False)
                if summ is not None:
                    self.busy.remove(s)
                    self._complete(s, summ)
                    progressed = True
            if not progressed and not waiting and i < len(reqs) and not self.busy:
                time.sleep(max(0.0, min(1e-3, reqs[i].arrival - now)))
        return reqs

    def close(self):
        for lst in self.free.values():
            for s in lst:
                s.destroy()
        self.free = {}
        for plan in self.plans.values():
            plan.destroy()
        self.plans = {}


def poisson_requests(rate: float, count: int, mix, seed: int):
    """count requests with exponential inter-arrival times of mean 1/rate and
    (p, m) drawn uniformly from mix; right-hand sides ~ U[-1, 1] (seeded),
    placed in device memory before the run."""
    import torch
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    out = []
    for k in range(count):
        p, m = mix[int(rng.integers(len(mix)))]
        nd = m ** 3 * (p + 1) ** 3
        b = torch.from_numpy(rng.uniform(-1.0, 1.0, nd)).cuda()
        out.append(Request(k, p, m, float(t[k]), b))
    return out


def latency_stats(reqs):
    """Latency percentiles and throughput of the served (not rejected) requests."""
    served = [r for r in reqs if not r.rejected]
    lat = np.array([r.done - r.arrival for r in served]) * 1e3
    span = max(r.done for r in served) - min(r.arrival for r in served)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "solves_per_s": len(served) / span,
            "queue_p50_ms": float(np.percentile([(r.start - r.arrival) * 1e3 for r in served], 50)),
            "rejected": len(reqs) - len(served)}
