"""Benchmark of the batched tensor-product hot path on one MI355X.

One step = one pass of the hot path over one batch: the volume operator
v = A u (apply, Neumann factor K) followed by the fast-diagonalization
inverse x = D^{-1} v of the SIPG cell block, both in the workload's precision,
on inputs already resident in HBM.  Throughput = DoF / step time (the paper's
N_dof / t normalisation, Sec. 6.1).  Input/output buffer sets are rotated so
the working set exceeds the 256 MB last-level cache and the rate is an HBM
rate.

Prints ONE JSON line.  Besides the contract fields it carries:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                average launch time (HIP events), against 8 TB/s
  cpu_baseline  the FP64 dense oracle timed on a bounded sample on the host
  ops           per-operation rates (apply, apply_inverse, solve)
  solve_latency per-call wall time percentiles of the block-local solve

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_workload(name):
    from paper_2609_04534_amd import workloads
    table = {
        "p3_64cube_affine": (workloads.affine_p3, "f64"),
        "p2_8cube_h1/8": (workloads.small_p2, "f64"),
        "p2_128cube": (workloads.large_p2, "f64"),
        "p7_32cube_aniso": (workloads.mixed_precision_p7, "f32"),
        "uneven_p237_20000": (workloads.uneven_degrees, "f32"),
    }
    fn, dt = table[name]
    return fn(with_rhs=True), dt


def algorithmic_bytes(wl, esize):
    """2 n^3 s + 24 bytes per block: vector in, vector out, three FP64 lengths."""
    return sum(g.nblocks * (2 * g.n ** 3 * esize + 24) for g in wl.groups)


def flops(wl, which):
    per = {"apply": lambda n: 14 * n ** 4 + 2 * n ** 3, "inverse": lambda n: 12 * n ** 4 + n ** 3}[which]
    return sum(g.nblocks * per(g.n) for g in wl.groups)


def time_launches(fn, stream, reps, sets, warm=3):
    """Average milliseconds per call of fn(k) over reps calls, HIP events on
    stream, after warm untimed calls (the first launch of a kernel loads its
    code object, milliseconds that are no part of the kernel's time)."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    for i in range(warm):
        fn(i % sets)
    torch.cuda.synchronize()
    start.record(stream)
    for i in range(reps):
        fn(i % sets)
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps


def _host_cpu():
    """CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, int(os.cpu_count() or 0), int(avail or 0)


_CPU_WL = None   # the workload the CPU-baseline worker processes read (inherited at fork)


def _one_thread():
    """Each worker process runs its BLAS single-threaded (one per core)."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _dense_chunk(seed, chunk=64):
    """One random chunk per group: dense apply, then the dense refined solve."""
    from oracle import dense
    rng = np.random.default_rng(seed)
    dof = nblk = 0
    for g in _CPU_WL.groups:
        idx = rng.integers(0, g.nblocks, size=max(1, min(chunk, g.nblocks)))
        v = dense.apply_batch(g.p, g.h[idx], g.u[idx], dense.NEUMANN)
        dense.solve_batch(g.p, g.h[idx], v, dense.CELL, chunk=chunk)
        dof += len(idx) * g.n ** 3
        nblk += len(idx)
    return dof, nblk


def _sumfact_part(args):
    from oracle import dense, sumfact
    gi, lo, hi = args
    g = _CPU_WL.groups[gi]
    v = sumfact.apply(g.p, g.h[lo:hi], g.u[lo:hi], dense.NEUMANN)
    sumfact.inverse(g.p, g.h[lo:hi], v, dense.CELL)
    return hi - lo


def cpu_baseline(wl, budget_s=12.0):
    """Time the FP64 dense oracle on the host on a bounded random sample of
    the workload's blocks: the step's apply (dense Kronecker products,
    oracle.dense.apply_batch) and the cell-block inverse (dense LAPACK solves
    with long-double refinement, oracle.dense.solve_batch), in chunks of 64
    blocks spread over one worker process per available host core.  Reports
    DoF/s of the apply + inverse step, the cores actually busy (the workers'
    CPU time / wall time) and the host CPU.  The sum-factorized CPU reference
    (oracle.sumfact) is timed on the whole workload beside it, split the same
    way.  Must run before the process initialises the GPU: the workers are
    forked from it."""
    import multiprocessing as mp
    import resource
    global _CPU_WL
    _CPU_WL = wl
    model, ncpu, avail = _host_cpu()
    workers = max(1, avail)
    ctx = mp.get_context("fork")

    def child_cpu():
        r = resource.getrusage(resource.RUSAGE_CHILDREN)
        return r.ru_utime + r.ru_stime

    c0 = child_cpu()
    t0 = time.perf_counter()
    dof = nblk = 0
    with ctx.Pool(workers, initializer=_one_thread) as pool:
        seed = 0
        while time.perf_counter() - t0 < budget_s:
            for d, b in pool.map(_dense_chunk, range(seed, seed + workers)):
                dof += d
                nblk += b
            seed += workers
        wall = time.perf_counter() - t0
        pool.close()
        pool.join()
    cpu = child_cpu() - c0
    out = {"value": dof / wall / 1e9, "unit": "GDoF/s", "cores": max(1, int(round(cpu / wall))),
           "kind": "oracle",
           "sample": f"{nblk} random blocks of {wl.name} (dense Kronecker apply, then dense LAPACK solve of the "
                     f"cell block with long-double refinement; FP64; {workers} worker processes), "
                     f"{wall:.1f} s wall",
           "host_cpu": model, "nproc": ncpu, "cores_available": avail}
    parts = []
    for gi, g in enumerate(wl.groups):
        step = max(1, -(-g.nblocks // (4 * workers)))
        parts += [(gi, lo, min(g.nblocks, lo + step)) for lo in range(0, g.nblocks, step)]
    c0 = child_cpu()
    t0 = time.perf_counter()
    with ctx.Pool(workers, initializer=_one_thread) as pool:
        pool.map(_sumfact_part, parts)
        wall = time.perf_counter() - t0
        pool.close()
        pool.join()
    cpu = child_cpu() - c0
    out["sumfact"] = {"value": wl.ndof / wall / 1e9, "unit": "GDoF/s", "cores": max(1, int(round(cpu / wall))),
                      "sample": f"whole {wl.name} (numpy contractions, FP64; {workers} worker processes), "
                                f"{wall:.1f} s wall"}
    _CPU_WL = None
    return out


def cpu_sumfact_all(workers=None):
    """The sum-factorized CPU reference (oracle.sumfact: apply, then the
    cell-block inverse, FP64) on each whole benchmark workload, split over
    one forked worker process per available core (BLAS single-threaded in
    each).  Like cpu_baseline, it runs before the process touches the GPU."""
    import multiprocessing as mp
    global _CPU_WL
    _, _, avail = _host_cpu()
    workers = workers or max(1, avail)
    ctx = mp.get_context("fork")
    out = {}
    for name in ("p2_128cube", "p3_64cube_affine", "p7_32cube_aniso", "uneven_p237_20000"):
        wl = build_workload(name)[0]
        _CPU_WL = wl
        parts = []
        for gi, g in enumerate(wl.groups):
            step = max(1, -(-g.nblocks // (4 * workers)))
            parts += [(gi, lo, min(g.nblocks, lo + step)) for lo in range(0, g.nblocks, step)]
        t0 = time.perf_counter()
        with ctx.Pool(workers, initializer=_one_thread) as pool:
            pool.map(_sumfact_part, parts)
            wall = time.perf_counter() - t0
            pool.close()
            pool.join()
        out[name] = {"value": wl.ndof / wall / 1e9, "unit": "GDoF/s", "ndof": wl.ndof, "wall_s": round(wall, 2),
                     "workers": workers}
        _CPU_WL = None
        del wl
    return out


def measure_ops(name, dtname, stream, reps=100):
    """apply and apply_inverse of a workload in one storage precision with
    buffer sets rotated past the last-level cache (HIP events on stream;
    as for the headline kernels, 10 untimed and 100 timed launches each:
    sustained back-to-back launches run slower than short bursts on this
    GPU, so short loops would flatter the rate)."""
    import torch
    from paper_2609_04534_amd import tpfdm
    codes = {"f64": (tpfdm.F64, torch.float64, 8), "f32": (tpfdm.F32, torch.float32, 4),
             "f16": (tpfdm.F16, torch.float16, 2), "bf16": (tpfdm.BF16, torch.bfloat16, 2)}
    code, tdt, es = codes[dtname]
    wl, _ = build_workload(name)
    plan = tpfdm.Plan(tpfdm.groups_for_workload(wl))
    plan.setup_inverse(tpfdm.OP_CELL)
    E, ndof = plan.vector_elems, plan.ndof
    cu = torch.from_numpy(np.concatenate([g.u.reshape(-1) for g in wl.groups])).cuda().to(tdt)
    vec_bytes = E * es
    R = int(min(16, max(2, -(-1.0e9 // (3 * vec_bytes)))))
    U = [torch.empty(E, dtype=tdt, device="cuda") for _ in range(R)]
    for u in U:
        plan.pack(cu, u)
    V = [torch.empty_like(U[0]) for _ in range(R)]
    X = [torch.empty_like(U[0]) for _ in range(R)]
    for k in range(3):
        plan.apply(U[k % R], V[k % R], tpfdm.OP_NEUMANN, stream=stream)
        plan.apply_inverse(V[k % R], X[k % R], stream=stream)
    for k in range(10):
        plan.apply(U[k % R], V[k % R], tpfdm.OP_NEUMANN, stream=stream)
    ms_a = time_launches(lambda k: plan.apply(U[k], V[k], tpfdm.OP_NEUMANN, stream=stream), stream, reps, R)
    for k in range(10):
        plan.apply_inverse(V[k % R], X[k % R], stream=stream)
    ms_i = time_launches(lambda k: plan.apply_inverse(V[k], X[k], stream=stream), stream, reps, R)
    ms_s = time_launches(lambda k: (plan.apply(U[k], V[k], tpfdm.OP_NEUMANN, stream=stream),
                                    plan.apply_inverse(V[k], X[k], stream=stream)), stream, reps, R)
    ab = algorithmic_bytes(wl, es)
    kern = [[plan.kernel(i, 0, code, grid=True), plan.kernel(i, 1, code, grid=True)] for i in range(len(wl.groups))]
    out = {"workload": name, "dtype": dtname, "ndof": ndof, "kernels": kern,
           "step_GDoF/s": ndof / ms_s / 1e6, "ms_per_step": ms_s}
    for key, ms, which in (("apply", ms_a, "apply"), ("apply_inverse", ms_i, "inverse")):
        out[key] = {"ms": ms, "GDoF/s": ndof / ms / 1e6, "GB/s": ab / ms / 1e6,
                    "hbm_frac": ab / ms / 1e6 / HBM_PEAK_GBS, "TFLOP/s": flops(wl, which) / ms / 1e9}
    plan.destroy()
    del U, V, X, cu
    torch.cuda.empty_cache()
    return out


def true_relres(plan, b, x):
    """||b - A x||_2 / ||b||_2 with the library's coupled operator in FP64."""
    import torch
    from paper_2609_04534_amd import tpfdm
    ax = torch.empty_like(x)
    plan.apply(x, ax, tpfdm.OP_SIPG)
    torch.cuda.synchronize()
    return float(torch.linalg.vector_norm(b - ax) / torch.linalg.vector_norm(b))


# Mixed-precision MG-PCG: (degree, cells per side) and the stopping rules:
# the paper's (Sec. 6.1: <r, z>^{1/2} reduced by 1e-10) and the serving
# tolerance (||r||_2 <= 1e-8 ||b||_2)
MIXED_MESHES = [(3, 128), (3, 64), (2, 96)]
MIXED_RULES = [("precnorm", 1e-10), ("residual", 1e-8)]
# (name, multigrid level storage, inner block-inverse precision)
MIXED_CONFIGS = [("fp64", "f64", "f64"), ("fp64_storage_fp32_inner", "f64", "f32"),
                 ("fp32_storage", "f32", "f32")]


def run_mixed_mg(stream, meshes=MIXED_MESHES, reps=4, emit=True):
    """MG-PCG with FP64 level vectors vs FP32 level vectors (z in FP32, x, r,
    p and every dot product in FP64): median solve time, iterations and the
    true final residual of each; one JSON line per mesh, rule and config."""
    import torch
    from paper_2609_04534_amd import tpfdm, workloads
    dt = {"f64": tpfdm.F64, "f32": tpfdm.F32}
    recs = []
    for p, m in meshes:
        mesh = workloads.unit_cube_mesh(p, m, seed=11)
        plan = tpfdm.Plan.mesh(mesh.n, mesh.cells, mesh.h)
        plan.setup_inverse(tpfdm.OP_CELL)
        b = torch.empty(plan.vector_elems, dtype=torch.float64, device="cuda")
        plan.pack(torch.from_numpy(mesh.u).cuda(), b)
        x = torch.empty_like(b)
        for rule, rtol in MIXED_RULES:
            for cname, storage, inner in MIXED_CONFIGS:
                V = tpfdm.MG(plan, storage=dt[storage])
                solver = tpfdm.PCG(plan)
                solver.set_multigrid(V)
                solver.set_norm(tpfdm.PCG_PRECONDITIONED if rule == "precnorm" else tpfdm.PCG_RESIDUAL)
                lat, s = [], None
                for i in range(reps + 1):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    s = solver.solve(b, x, inner=dt[inner], rtol=rtol, maxit=100, check_every=4, stream=stream)
                    t1 = time.perf_counter()
                    if i >= 1:
                        lat.append(t1 - t0)
                t = float(np.median(lat))
                rec = {"workload": f"mg_pcg_p{p}_{m}cube", "rule": rule, "rtol": rtol, "config": cname,
                       "level_storage": storage, "inner": inner, "ndof": mesh.ndof,
                       "iterations": s["iterations"], "converged": bool(s["converged"]),
                       "relres_recursive": s["relres"], "relres_true": true_relres(plan, b, x),
                       "solve_ms": t * 1e3, "solve_MDoF/s": mesh.ndof / t / 1e6}
                recs.append(rec)
                if emit:
                    print(json.dumps(rec), flush=True)
                solver.destroy()
                V.destroy()
        plan.destroy()
        del b, x
        torch.cuda.empty_cache()
    return recs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="p3_64cube_affine")
    ap.add_argument("--rotate", type=int, default=4)
    ap.add_argument("--solve-calls", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--suite", action="store_true",
                    help="time apply / apply_inverse / solve for every workload and precision "
                         "(one JSON line per case) instead of the headline step")
    ap.add_argument("--serve", action="store_true",
                    help="serve Poisson arrival streams of PCG solves at several rates (JSON lines)")
    ap.add_argument("--pcg", action="store_true",
                    help="time preconditioned-CG solves of the SIPG system on the serving mesh sizes (JSON lines)")
    ap.add_argument("--pcg-mesh", default=None, metavar="P,M[,BASIS]",
                    help="with --pcg: only the unit cube of degree P with M cells per side "
                         "(BASIS lagrange or hermite)")
    ap.add_argument("--patches", action="store_true",
                    help="time the operator and the exact solve on vertex-patch blocks (JSON lines)")
    ap.add_argument("--mg-paper", action="store_true",
                    help="time the paper's solver configuration (MG-PCG, p = 3, <r, z>^{1/2} reduced by 1e-10) "
                         "on 32^3 .. 128^3 cubes in both bases (JSON lines)")
    ap.add_argument("--sipg", action="store_true",
                    help="time only the coupled SIPG operator on the unit-cube meshes (JSON lines)")
    ap.add_argument("--dtype", default=None, choices=["f64", "f32", "f16", "bf16"],
                    help="storage precision of the step (default: the workload's)")
    ap.add_argument("--mixed", action="store_true",
                    help="MG-PCG with FP64 vs FP32 multigrid level storage at the paper's and the serving "
                         "stopping rules (JSON lines)")
    ap.add_argument("--uneven", action="store_true",
                    help="only the batched uneven-degree modes (per-group, single launch, tuned, graphs; JSON lines)")
    ap.add_argument("--counters", action="store_true",
                    help="no timing: launch a plain device copy of one vector, apply and "
                         "apply_inverse 3 times each and one FP64- and one FP32-inner solve "
                         "(for hardware-counter runs), then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the blocks are independent and each GPU would run the "
              f"same kernels on its share; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    headline = not (args.suite or args.mg_paper or args.patches or args.pcg or args.serve or args.sipg
                    or args.uneven or args.mixed or args.counters)
    cpu_base = None
    if headline and not args.no_cpu_baseline:
        # before anything initialises the GPU: the baseline forks its workers
        _log("cpu baseline")
        cpu_base = cpu_baseline(build_workload(args.workload)[0])
        cpu_base["sumfact_by_workload"] = cpu_sumfact_all()

    import torch
    from paper_2609_04534_amd import tpfdm
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    tpfdm.load()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    if args.suite:
        run_suite(args, stream)
        return
    if args.uneven:
        run_uneven(args, stream)
        return
    if args.mixed:
        run_mixed_mg(stream)
        return
    if args.mg_paper:
        run_mg_paper(args, stream)
        return
    if args.patches:
        run_patches(args, stream)
        return
    if args.pcg:
        run_pcg(args, stream)
        return
    if args.serve:
        run_serve(args)
        return
    if args.sipg:
        if args.counters:
            sipg_counters()
            return
        run_sipg(args, stream)
        return

    _log(f"workload {args.workload}")
    wl, dtname = build_workload(args.workload)
    if args.dtype:
        dtname = args.dtype
    dt = {"f64": tpfdm.F64, "f32": tpfdm.F32, "f16": tpfdm.F16, "bf16": tpfdm.BF16}[dtname]
    tdt = {tpfdm.F64: torch.float64, tpfdm.F32: torch.float32, tpfdm.F16: torch.float16,
           tpfdm.BF16: torch.bfloat16}[dt]
    esize = {tpfdm.F64: 8, tpfdm.F32: 4, tpfdm.F16: 2, tpfdm.BF16: 2}[dt]
    plan = tpfdm.Plan(tpfdm.groups_for_workload(wl))
    plan.setup_inverse(tpfdm.OP_CELL)
    ndof = plan.ndof
    E = plan.vector_elems
    canon_u = torch.from_numpy(np.concatenate([g.u.reshape(-1) for g in wl.groups])).cuda()
    canon_b = torch.from_numpy(np.concatenate([g.b.reshape(-1) for g in wl.groups])).cuda()
    R = max(1, args.rotate)
    U, V, X = [], [], []
    for _ in range(R):
        bu = torch.empty(E, dtype=tdt, device="cuda")
        plan.pack(canon_u.to(tdt), bu)
        U.append(bu)
        V.append(torch.empty(E, dtype=tdt, device="cuda"))
        X.append(torch.empty(E, dtype=tdt, device="cuda"))
    torch.cuda.synchronize()
    _log(f"ndof={ndof} vector_elems={E} sets={R}")

    if args.counters:
        # calibration: a plain elementwise kernel over exactly one vector
        # (vector_elems * esize bytes read and written; torch's copy_ would
        # go to a DMA engine, which the shader counters do not see), then
        # the two kernels of the step
        for k in range(3):
            torch.mul(U[k % R], 1.0, out=V[k % R])
        for k in range(3):
            plan.apply(U[k % R], V[k % R], tpfdm.OP_NEUMANN, stream=stream)
        for k in range(3):
            plan.apply_inverse(V[k % R], X[k % R], stream=stream)
        bb = torch.empty(E, dtype=torch.float64, device="cuda")
        plan.pack(canon_b, bb)
        for inner in (tpfdm.F64, tpfdm.F32):
            xs = torch.zeros_like(bb)
            plan.solve(bb, xs, inner=inner, rtol=1e-10, maxit=50, summary=False, stream=stream)
        torch.cuda.synchronize()
        print(json.dumps({"counters_run": args.workload, "copy_bytes": E * esize,
                          "algorithmic_bytes_per_launch": algorithmic_bytes(wl, esize)}), flush=True)
        plan.destroy()
        return

    def step(k):
        plan.apply(U[k], V[k], tpfdm.OP_NEUMANN, stream=stream)
        plan.apply_inverse(V[k], X[k], stream=stream)

    for i in range(args.warmup):
        step(i % R)
    torch.cuda.synchronize()
    _log("warmup done")
    ms_step = time_launches(step, stream, args.steps, R, warm=0)
    _log(f"step {ms_step:.4f} ms")
    # each kernel alone: 10 untimed launches, then at least 100 timed ones
    reps = max(args.steps, 100)
    for k in range(10):
        plan.apply(U[k % R], V[k % R], tpfdm.OP_NEUMANN, stream=stream)
    ms_apply = time_launches(lambda k: plan.apply(U[k], V[k], tpfdm.OP_NEUMANN, stream=stream), stream, reps, R)
    for k in range(10):
        plan.apply_inverse(V[k % R], X[k % R], stream=stream)
    ms_inv = time_launches(lambda k: plan.apply_inverse(V[k], X[k], stream=stream), stream, reps, R)
    _log(f"apply {ms_apply:.4f} ms, inverse {ms_inv:.4f} ms")

    # solve: FP64 residual, rtol 1e-10, per-call latency (launch + sync) for
    # every inner precision (time to the same final residual)
    bb = torch.empty(E, dtype=torch.float64, device="cuda")
    plan.pack(canon_b, bb)
    xs = torch.zeros(E, dtype=torch.float64, device="cuda")
    by_inner = {}
    for inner in (tpfdm.F64, tpfdm.F32, tpfdm.F16, tpfdm.BF16):
        lat = []
        summ = None
        for i in range(args.solve_calls + 3):
            xs.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            summ = plan.solve(bb, xs, inner=inner, rtol=1e-10, maxit=50, stream=stream)
            t1 = time.perf_counter()
            if i >= 3:
                lat.append((t1 - t0) * 1e3)
        lat = np.array(lat)
        by_inner[tpfdm.DTYPE_NAMES[inner]] = {
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "GDoF/s_p50": ndof / np.percentile(lat, 50) / 1e6, "max_iters": summ["max_iters"],
            "max_relres": summ["max_relres"]}
        _log(f"solve inner={tpfdm.DTYPE_NAMES[inner]} p50 {np.percentile(lat, 50):.3f} ms "
             f"p99 {np.percentile(lat, 99):.3f} ms {summ}")

    bytes_launch = algorithmic_bytes(wl, esize)
    dom_name, dom_ms = ("tp_apply_inverse", ms_inv) if ms_inv >= ms_apply else ("tp_apply", ms_apply)
    achieved = bytes_launch / (dom_ms * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            tj = json.load(open(tfile))
            ent = tj.get(args.workload, {}).get(dom_name)
            if ent and ent.get("kernel_hash") == kernel_hash():
                traffic = ent["bytes_per_launch"]
        except Exception:
            traffic = None

    out = {
        "metric": "GDoF/s apply+FDM-inverse at p=2/3/7, FP64 vs mixed; solve p50/p99 latency",
        "value": ndof / (ms_step * 1e-3) / 1e9,
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtname,
        "data": "synthetic (seeded uniform[-1,1] vectors, seeded cell lengths)",
        "config": {"workload": args.workload, "nblocks": wl.nblocks, "ndof": ndof,
                   "degrees": sorted({g.p for g in wl.groups}),
                   "layout_B": {str(g.n): tpfdm.default_layout_B(g.n) for g in wl.groups},
                   "buffer_sets": R, "step": "apply(Neumann) then apply_inverse(cell block)"},
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_launch, "avg_launch_ms": dom_ms},
        "ops": {
            "apply": {"ms": ms_apply, "GDoF/s": ndof / ms_apply / 1e6,
                      "GB/s": bytes_launch / ms_apply / 1e6, "TFLOP/s": flops(wl, "apply") / ms_apply / 1e9},
            "apply_inverse": {"ms": ms_inv, "GDoF/s": ndof / ms_inv / 1e6,
                              "GB/s": bytes_launch / ms_inv / 1e6,
                              "TFLOP/s": flops(wl, "inverse") / ms_inv / 1e9},
        },
        "solve_latency": {"rtol": 1e-10, "calls": int(args.solve_calls), "residual": "f64",
                          "by_inner": by_inner,
                          "fastest_inner": min(by_inner, key=lambda k: by_inner[k]["p50_ms"])},
    }
    plan.destroy()
    del U, V, X, bb, xs
    torch.cuda.empty_cache()
    # the metric's other degrees and precisions, same step, same measurement
    extra = {}
    for name, dtn in EXTRA_OPS:
        _log(f"ops {name} {dtn}")
        r = measure_ops(name, dtn, stream, reps=max(args.steps, 100))
        extra[f"{name}/{dtn}"] = r
    out["ops_other_workloads"] = extra
    # mixed precision at equal final residual: MG-PCG with FP32 level storage
    # against FP64 on the paper's configuration (p = 3, 128^3 cells)
    _log("mixed-precision MG-PCG")
    recs = run_mixed_mg(stream, meshes=[(3, 128)], reps=3, emit=False)
    out["mixed_precision_mg_pcg"] = [
        {k: r[k] for k in ("rule", "rtol", "config", "iterations", "relres_true", "solve_ms")} for r in recs]
    out["cpu_baseline"] = cpu_base
    print(json.dumps(out), flush=True)


# the headline line also carries these (workload, storage precision) cases
EXTRA_OPS = [("p2_128cube", "f64"), ("p7_32cube_aniso", "f64"), ("p7_32cube_aniso", "f32"),
             ("p7_32cube_aniso", "f16"), ("p7_32cube_aniso", "bf16")]

SUITE = [
    ("p2_8cube_h1/8", ["f64", "f32"]),
    ("p2_128cube", ["f64", "f32"]),
    ("p3_64cube_affine", ["f64", "f32", "f16", "bf16"]),
    ("p7_32cube_aniso", ["f64", "f32", "f16", "bf16"]),
    ("uneven_p237_20000", ["f64", "f32"]),
]


def run_suite(args, stream):
    """Per workload and storage precision: apply and apply_inverse rates with
    rotated buffers, and solve latency with FP64 and FP32 inner solves."""
    import torch
    from paper_2609_04534_amd import tpfdm
    codes = {"f64": (tpfdm.F64, torch.float64, 8), "f32": (tpfdm.F32, torch.float32, 4),
             "f16": (tpfdm.F16, torch.float16, 2), "bf16": (tpfdm.BF16, torch.bfloat16, 2)}
    for name, dts in SUITE:
        wl, _ = build_workload(name)
        plan = tpfdm.Plan(tpfdm.groups_for_workload(wl))
        plan.setup_inverse(tpfdm.OP_CELL)
        E, ndof = plan.vector_elems, plan.ndof
        cu = torch.from_numpy(np.concatenate([g.u.reshape(-1) for g in wl.groups])).cuda()
        cb = torch.from_numpy(np.concatenate([g.b.reshape(-1) for g in wl.groups])).cuda()
        for dtn in dts:
            code, tdt, es = codes[dtn]
            vec_bytes = E * es
            # rotate enough buffer sets that one pass touches >= 1 GB (4x the
            # last-level cache); tiny cases stay cache resident and say so
            R = int(min(16, max(1, -(-1.0e9 // (3 * vec_bytes)))))
            if 3 * R * vec_bytes < 0.75e9:
                R = 1
            U = [torch.empty(E, dtype=tdt, device="cuda") for _ in range(R)]
            for u in U:
                plan.pack(cu.to(tdt), u)
            V = [torch.empty_like(U[0]) for _ in range(R)]
            X = [torch.empty_like(U[0]) for _ in range(R)]
            for k in range(3):
                plan.apply(U[k % R], V[k % R], tpfdm.OP_NEUMANN, stream=stream)
                plan.apply_inverse(V[k % R], X[k % R], stream=stream)
            reps = max(args.steps, 100)
            ms_a = time_launches(lambda k: plan.apply(U[k], V[k], tpfdm.OP_NEUMANN, stream=stream), stream, reps, R)
            ms_i = time_launches(lambda k: plan.apply_inverse(V[k], X[k], stream=stream), stream, reps, R)
            # a plain device copy of the same vector: the bandwidth reachable at this size
            ms_c = time_launches(lambda k: X[k].copy_(U[k]), stream, reps, R)
            # the same after per-group autotuning of the kernel choice
            plan.autotune(code, reps=5)
            ms_at = time_launches(lambda k: plan.apply(U[k], V[k], tpfdm.OP_NEUMANN, stream=stream), stream, reps, R)
            ms_it = time_launches(lambda k: plan.apply_inverse(V[k], X[k], stream=stream), stream, reps, R)
            tuned = {"apply_ms": ms_at, "inverse_ms": ms_it,
                     "kernels": [(plan.kernel(i, 0, code, grid=True), plan.kernel(i, 1, code, grid=True))
                                 for i in range(len(wl.groups))]}
            ab = algorithmic_bytes(wl, es)
            rec = {"workload": name, "dtype": dtn, "ndof": ndof, "buffer_sets": R, "tuned": tuned,
                   "cache_resident": 3 * R * vec_bytes < 0.75e9,
                   "copy_ms": ms_c, "copy_GB/s": 2 * vec_bytes / ms_c / 1e6,
                   "apply_ms": ms_a, "apply_GDoF/s": ndof / ms_a / 1e6, "apply_GB/s": ab / ms_a / 1e6,
                   "apply_TFLOP/s": flops(wl, "apply") / ms_a / 1e9,
                   "inverse_ms": ms_i, "inverse_GDoF/s": ndof / ms_i / 1e6, "inverse_GB/s": ab / ms_i / 1e6,
                   "inverse_TFLOP/s": flops(wl, "inverse") / ms_i / 1e9}
            del U, V, X
            print(json.dumps(rec), flush=True)
        bb = torch.empty(E, dtype=torch.float64, device="cuda")
        plan.pack(cb, bb)
        xs = torch.zeros_like(bb)
        for inner in (tpfdm.F64, tpfdm.F32):
            lat = []
            summ = None
            for i in range(max(10, args.solve_calls // 4) + 2):
                xs.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                summ = plan.solve(bb, xs, inner=inner, rtol=1e-10, maxit=50, stream=stream)
                t1 = time.perf_counter()
                if i >= 2:
                    lat.append((t1 - t0) * 1e3)
            print(json.dumps({"workload": name, "solve_inner": tpfdm.DTYPE_NAMES[inner],
                              "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                              "max_iters": summ["max_iters"], "max_relres": summ["max_relres"]}), flush=True)
        plan.destroy()
        del bb, xs, cu, cb
        torch.cuda.empty_cache()
    run_uneven(args, stream)
    run_sipg(args, stream)


# Coupled SIPG operator on uniformly refined unit cubes (the meshes of the
# paper's face-kernel and operator measurements, Sec. 6.3 and 6.5).
# (degree, cells per side, dtypes, basis): the Lagrange basis, and the
# Hermite-type basis (face terms on the layers next to each face) at degrees
# 3 and 7
SIPG_SUITE = [(3, 128, ("f64", "f32"), "lagrange"), (3, 128, ("f64", "f32"), "hermite"),
              (3, 64, ("f64",), "lagrange"), (3, 64, ("f64",), "hermite"), (2, 128, ("f64",), "lagrange"),
              (7, 64, ("f64", "f32"), "lagrange"), (7, 64, ("f64", "f32"), "hermite")]


def run_sipg(args, stream):
    """Coupled operator v = A u (and its face part A^face u) on mesh plans:
    HBM-resident inputs, algorithmic bytes = one vector read + one written."""
    import torch
    from paper_2609_04534_amd import tpfdm, workloads
    codes = {"f64": (tpfdm.F64, torch.float64, 8), "f32": (tpfdm.F32, torch.float32, 4)}
    for p, m, dts, basis in SIPG_SUITE:
        mesh = workloads.unit_cube_mesh(p, m, seed=5)
        plan = tpfdm.Plan.mesh(mesh.n, mesh.cells, mesh.h,
                               basis=tpfdm.BASIS_HERMITE if basis == "hermite" else tpfdm.BASIS_LAGRANGE)
        cu = torch.from_numpy(mesh.u).cuda()
        for dtn in dts:
            code, tdt, es = codes[dtn]
            E = plan.vector_elems
            vec_bytes = E * es
            R = int(min(8, max(1, -(-1.0e9 // (2 * vec_bytes)))))
            U = [torch.empty(E, dtype=tdt, device="cuda") for _ in range(R)]
            for u in U:
                plan.pack(cu.to(tdt), u)
            V = [torch.empty_like(U[0]) for _ in range(R)]
            for k in range(3):
                plan.apply(U[k % R], V[k % R], tpfdm.OP_SIPG, stream=stream)
            reps = max(args.steps, 20)
            ms = time_launches(lambda k: plan.apply(U[k], V[k], tpfdm.OP_SIPG, stream=stream), stream, reps, R)
            ms_f = time_launches(lambda k: plan.apply(U[k], V[k], tpfdm.OP_SIPG_FACE, stream=stream), stream,
                                 reps, R)
            # the volume part alone is a block call (not served by plans in the
            # Hermite-type basis with n >= 5)
            ms_v = (None if basis == "hermite" and p >= 4 else
                    time_launches(lambda k: plan.apply(U[k], V[k], tpfdm.OP_NEUMANN, stream=stream), stream, reps, R))
            ms_c = time_launches(lambda k: V[k].copy_(U[k]), stream, reps, R)
            nd = mesh.ndof
            print(json.dumps({"workload": mesh.name, "basis": basis, "dtype": dtn, "ndof": nd, "buffer_sets": R,
                              "sipg_ms": ms, "sipg_GDoF/s": nd / ms / 1e6, "sipg_GB/s": 2 * nd * es / ms / 1e6,
                              "face_ms": ms_f, "face_GDoF/s": nd / ms_f / 1e6,
                              "volume_ms": ms_v, "volume_GDoF/s": nd / ms_v / 1e6 if ms_v else None,
                              "copy_ms": ms_c, "copy_GB/s": 2 * vec_bytes / ms_c / 1e6}), flush=True)
            del U, V
        plan.destroy()
        del cu
        torch.cuda.empty_cache()


# Serving meshes: unit cubes with m cells per side (the request mix of the
# serving configuration), rtol 1e-8, FP64 outer iteration.
PCG_SUITE = [(p, m) for p in (2, 3) for m in (8, 16, 24, 32, 48)] + [(7, m) for m in (8, 16, 24)]
# Larger meshes timed with the multigrid preconditioner only (block-Jacobi
# needs over a thousand iterations there).
PCG_MG_ONLY = [(3, 64), (2, 96), (7, 32), (7, 48)]
# Degree-3 meshes in the Hermite-type basis (two-layer face access), MG only.
PCG_HERMITE = [(3, 24), (3, 48), (3, 64)]


def run_pcg(args, stream):
    """Per mesh, preconditioner (block-Jacobi; one multigrid V-cycle where
    the serving loop uses one) and its precision: wall latency of whole
    solves (launch to host summary), p50 / p99 over repeated solves,
    iterations."""
    import torch
    from paper_2609_04534_amd import serve, tpfdm, workloads
    suite = [(p, m, "lagrange") for p, m in PCG_SUITE + PCG_MG_ONLY] + [(p, m, "hermite") for p, m in PCG_HERMITE]
    if args.pcg_mesh:
        f = args.pcg_mesh.split(",")
        suite = [(int(f[0]), int(f[1]), f[2] if len(f) > 2 else "lagrange")]
    for p, m, basis in suite:
        mesh = workloads.unit_cube_mesh(p, m, seed=7)
        plan = tpfdm.Plan.mesh(mesh.n, mesh.cells, mesh.h,
                               basis=tpfdm.BASIS_HERMITE if basis == "hermite" else tpfdm.BASIS_LAGRANGE)
        plan.setup_inverse(tpfdm.OP_CELL)
        b = torch.empty(plan.vector_elems, dtype=torch.float64, device="cuda")
        plan.pack(torch.from_numpy(mesh.u).cuda(), b)
        x = torch.empty_like(b)
        solver = tpfdm.PCG(plan)
        mg = tpfdm.MG(plan) if serve.uses_multigrid(p, m) and basis == "lagrange" or p <= 3 else None
        # the FP32-inner solves keep the level vectors in FP32
        mg32 = tpfdm.MG(plan, storage=serve.mg_storage(p, tpfdm.F32)) if mg is not None else None
        preconds = (("mg",) if (p, m) in PCG_MG_ONLY or basis == "hermite"
                    else ("block_jacobi", "mg") if mg else ("block_jacobi",))
        for precond in preconds:
            for inner in (tpfdm.F64, tpfdm.F32):
                V = (mg32 or mg) if inner == tpfdm.F32 else mg
                solver.set_multigrid(V if precond == "mg" else None)
                reps = 30 if m <= 24 or (precond == "mg" and m <= 48) else 10
                lat, s = [], None
                for i in range(reps + 2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    s = solver.solve(b, x, inner=inner, rtol=1e-8, maxit=10000,
                                     check_every=4 if precond == "mg" else 16, stream=stream)
                    t1 = time.perf_counter()
                    if i >= 2:
                        lat.append((t1 - t0) * 1e3)
                p50 = float(np.percentile(lat, 50))
                print(json.dumps({"workload": f"pcg_p{p}_{m}cube", "basis": basis, "precond": precond,
                                  "inner": tpfdm.DTYPE_NAMES[inner], "ndof": mesh.ndof,
                                  "level_storage": (tpfdm.DTYPE_NAMES[V.storage] if precond == "mg" else None),
                                  "iterations": s["iterations"], "relres": s["relres"],
                                  "p50_ms": p50, "p99_ms": float(np.percentile(lat, 99)),
                                  "ms_per_iteration": p50 / max(1, s["iterations"]),
                                  "solves_per_s": 1e3 / p50}), flush=True)
        solver.destroy()
        for V in (mg, mg32):
            if V is not None:
                V.destroy()
        plan.destroy()
        del b, x
        torch.cuda.empty_cache()


# Vertex patches of a uniformly refined unit cube: one block per interior
# vertex, the 2 x 2 x 2 cells around it (n = 2(p+1)); (degree, cells per side,
# dtypes).
PATCH_SUITE = [(3, 64, ("f64", "f32", "f16")), (1, 128, ("f64", "f32"))]


def run_patches(args, stream):
    """Patch operator (TP_OP_CELL on patch blocks) and the exact patch solve
    (apply_inverse): rates with HBM-resident buffers, one vector read and one
    written per call (algorithmic bytes)."""
    import torch
    from paper_2609_04534_amd import tpfdm
    codes = {"f64": (tpfdm.F64, torch.float64, 8), "f32": (tpfdm.F32, torch.float32, 4),
             "f16": (tpfdm.F16, torch.float16, 2)}
    for p, m, dts in PATCH_SUITE:
        n = 2 * (p + 1)
        nb = (m - 1) ** 3
        h = np.full((nb, 3), 1.0 / m)
        plan = tpfdm.Plan([tpfdm.GroupSpec(n, tpfdm.default_layout_B(n), h)], blocks=tpfdm.BLOCKS_PATCHES)
        plan.setup_inverse(tpfdm.OP_CELL)
        E, nd = plan.vector_elems, plan.ndof
        u = torch.from_numpy(np.random.default_rng(9).uniform(-1, 1, nd)).cuda()
        for dtn in dts:
            code, tdt, es = codes[dtn]
            R = int(min(8, max(1, -(-1.0e9 // (2 * E * es)))))
            U = [torch.empty(E, dtype=tdt, device="cuda") for _ in range(R)]
            for x in U:
                plan.pack(u.to(tdt), x)
            V = [torch.empty_like(U[0]) for _ in range(R)]
            for k in range(3):
                plan.apply(U[k % R], V[k % R], tpfdm.OP_CELL, stream=stream)
                plan.apply_inverse(U[k % R], V[k % R], stream=stream)
            reps = max(args.steps, 20)
            ms_a = time_launches(lambda k: plan.apply(U[k], V[k], tpfdm.OP_CELL, stream=stream), stream, reps, R)
            ms_i = time_launches(lambda k: plan.apply_inverse(U[k], V[k], stream=stream), stream, reps, R)
            ms_c = time_launches(lambda k: V[k].copy_(U[k]), stream, reps, R)
            print(json.dumps({"workload": f"patches_p{p}_{m}cube", "n": n, "patches": nb, "dtype": dtn,
                              "ndof": nd, "apply_ms": ms_a, "apply_GDoF/s": nd / ms_a / 1e6,
                              "apply_GB/s": 2 * nd * es / ms_a / 1e6, "inverse_ms": ms_i,
                              "inverse_GDoF/s": nd / ms_i / 1e6, "inverse_GB/s": 2 * nd * es / ms_i / 1e6,
                              "copy_GB/s": 2 * E * es / ms_c / 1e6}), flush=True)
            del U, V
        plan.destroy()
        del u
        torch.cuda.empty_cache()


# The paper's solver configuration on globally refined unit cubes (p = 3,
# 2^k cells per side down to a one-cell coarsest level): CG with one V-cycle,
# stopped when <r, z>^{1/2} has decreased by 1e-10; solve throughput is
# DoF / wall time of a whole solve.
MG_PAPER = [(3, 32), (3, 64), (3, 128)]


def run_mg_paper(args, stream):
    import torch
    from paper_2609_04534_amd import tpfdm, workloads
    for p, m in MG_PAPER:
        for basis in ("lagrange", "hermite"):
            mesh = workloads.unit_cube_mesh(p, m, seed=11)
            plan = tpfdm.Plan.mesh(mesh.n, mesh.cells, mesh.h,
                                   basis=tpfdm.BASIS_HERMITE if basis == "hermite" else tpfdm.BASIS_LAGRANGE)
            plan.setup_inverse(tpfdm.OP_CELL)
            b = torch.empty(plan.vector_elems, dtype=torch.float64, device="cuda")
            plan.pack(torch.from_numpy(mesh.u).cuda(), b)
            x = torch.empty_like(b)
            solver = tpfdm.PCG(plan)
            solver.set_norm(tpfdm.PCG_PRECONDITIONED)
            # the paper's configuration (FP64 throughout), then the mixed form:
            # FP32 level vectors and inner precision, FP64 CG
            for storage, inner in ((tpfdm.F64, tpfdm.F64), (tpfdm.F32, tpfdm.F32)):
                mg = tpfdm.MG(plan, storage=storage)
                solver.set_multigrid(mg)
                reps = 10 if m <= 64 else 4
                lat, s = [], None
                for i in range(reps + 1):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    s = solver.solve(b, x, inner=inner, rtol=1e-10, maxit=100, check_every=4, stream=stream)
                    t1 = time.perf_counter()
                    if i >= 1:
                        lat.append(t1 - t0)
                t = float(np.median(lat))
                print(json.dumps({"workload": f"mg_pcg_p{p}_{m}cube_precnorm_1e-10", "basis": basis,
                                  "level_storage": tpfdm.DTYPE_NAMES[storage], "inner": tpfdm.DTYPE_NAMES[inner],
                                  "ndof": mesh.ndof, "iterations": s["iterations"], "relres": s["relres"],
                                  "solve_ms": t * 1e3, "solve_MDoF/s": mesh.ndof / t / 1e6,
                                  "ms_per_iteration": t * 1e3 / max(1, s["iterations"])}), flush=True)
                solver.set_multigrid(None)
                mg.destroy()
            solver.destroy()
            plan.destroy()
            del b, x
            torch.cuda.empty_cache()


# Serving: arrival rates (requests/s), each with a bounded number of
# requests drawn from the mesh mix (unit cubes with m cells per side,
# degrees 2, 3 and 7; FP64 outer iteration, FP32 preconditioner, rtol 1e-8).
# Degree 7 is drawn at m = 8 and 16 only: with block-Jacobi alone a degree-7
# solve at m = 32 or 48 runs for seconds, longer than a bounded run allows.
SERVE_RATES = [50, 200, 500, 2000]
SERVE_MIX = [(p, m) for p in (2, 3, 7) for m in (8, 16, 24, 32, 48)]


def run_serve(args):
    """The 15-class serving mix at every rate with the V-cycle preconditioner
    (every class), then with block-Jacobi throughout at the two lower rates
    (its degree-7 solves on 48^3 cells take seconds each)."""
    import torch
    from paper_2609_04534_amd import serve, tpfdm
    for multigrid in (True, False):
        srv = serve.Server(hbm_budget=24 << 30, inner=tpfdm.F32, rtol=1e-8, multigrid=multigrid)
        # warm start: plans, solver slots and their iteration graphs exist
        # before the measured runs (one request of every class)
        warm = [serve.poisson_requests(rate=1e6, count=1, mix=[c], seed=i)[0] for i, c in enumerate(SERVE_MIX)]
        srv.run(warm)
        _log(f"serve warm-up done (multigrid={multigrid})")
        del warm
        for rate in (SERVE_RATES if multigrid else SERVE_RATES[:2]):
            count = int(min(120, max(20, rate * 1.0)))
            reqs = serve.poisson_requests(rate=float(rate), count=count, mix=SERVE_MIX, seed=rate)
            srv.max_concurrent = 0
            done = srv.run(reqs)
            st = serve.latency_stats(done)
            st.update({"workload": "serve_pcg_mix", "precond": "mg" if multigrid else "block_jacobi",
                       "rate_per_s": rate, "requests": count, "max_concurrent": srv.max_concurrent,
                       "all_converged": all(r.summary.get("converged") for r in done)})
            print(json.dumps(st), flush=True)
            del reqs, done
        srv.close()
        torch.cuda.empty_cache()


def sipg_counters():
    """Hardware-counter run of the coupled operator on the p=3 128^3 mesh in
    FP64: one plain device copy of a vector (the calibration), then three
    applies of A and three of A^face, in the Lagrange basis and then in the
    Hermite-type basis (two-layer face access)."""
    import torch
    from paper_2609_04534_amd import tpfdm, workloads
    mesh = workloads.unit_cube_mesh(3, 128, seed=5)
    for basis in (tpfdm.BASIS_LAGRANGE, tpfdm.BASIS_HERMITE):
        with tpfdm.Plan.mesh(mesh.n, mesh.cells, mesh.h, basis=basis) as plan:
            u = torch.empty(plan.vector_elems, dtype=torch.float64, device="cuda")
            plan.pack(torch.from_numpy(mesh.u).cuda(), u)
            v = torch.empty_like(u)
            v.copy_(u)
            for _ in range(3):
                plan.apply(u, v, tpfdm.OP_SIPG)
            for _ in range(3):
                plan.apply(u, v, tpfdm.OP_SIPG_FACE)
            torch.cuda.synchronize()
            del u, v
    _log("sipg counters run done")


def run_uneven(args, stream):
    """Batched uneven degrees: per-group launches (eager, or replayed from a HIP
    graph whose groups are parallel branches) vs one persistent launch (eager
    or from a graph), for apply, apply_inverse and the FP32-inner /
    FP64-refined solve, with cache-resident inputs."""
    import torch
    from paper_2609_04534_amd import tpfdm
    wl, _ = build_workload("uneven_p237_20000")
    cu = torch.from_numpy(np.concatenate([g.u.reshape(-1) for g in wl.groups])).cuda()
    cb = torch.from_numpy(np.concatenate([g.b.reshape(-1) for g in wl.groups])).cuda()
    reps = max(args.steps, 50)
    for mode in ("per_group", "per_group_tuned", "per_group_graph", "persistent", "persistent_graph",
                 "persistent_tuned", "persistent_tuned_graph"):
        plan = tpfdm.Plan(tpfdm.groups_for_workload(wl), persistent=mode.startswith("persistent"))
        plan.setup_inverse(tpfdm.OP_CELL)
        config = None
        if "_tuned" in mode:
            plan.autotune(tpfdm.F32, reps=50)
        if mode.startswith("persistent"):
            config = {f"p{g.p}": [plan.launch_config(i, c, tpfdm.F32) for c in (0, 1, 2)]
                      for i, g in enumerate(wl.groups)}
        E = plan.vector_elems
        u = torch.empty(E, dtype=torch.float32, device="cuda")
        plan.pack(cu.float(), u)
        v, x = torch.empty_like(u), torch.empty_like(u)
        b = torch.empty(E, dtype=torch.float64, device="cuda")
        plan.pack(cb, b)
        xs = torch.zeros_like(b)
        if mode.endswith("_graph"):
            ga = plan.graph(tpfdm.GRAPH_APPLY, u, v, op=tpfdm.OP_NEUMANN)
            gi = plan.graph(tpfdm.GRAPH_INVERSE, u, x)
            gs = plan.graph(tpfdm.GRAPH_SOLVE, b, xs, dtype=tpfdm.F32, rtol=1e-10, maxit=50)
            fa = lambda k: ga.launch(stream)
            fi = lambda k: gi.launch(stream)
            fs = lambda: gs.launch(stream)
        else:
            fa = lambda k: plan.apply(u, v, tpfdm.OP_NEUMANN, stream=stream)
            fi = lambda k: plan.apply_inverse(u, x, stream=stream)
            fs = lambda: plan.solve(b, xs, inner=tpfdm.F32, rtol=1e-10, maxit=50, summary=False, stream=stream)
        for _ in range(3):
            fa(0), fi(0)
        ms_a = time_launches(fa, stream, reps, 1)
        ms_i = time_launches(fi, stream, reps, 1)
        lat = []
        for i in range(max(20, args.solve_calls // 2) + 3):
            xs.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fs()
            torch.cuda.synchronize()
            if i >= 3:
                lat.append((time.perf_counter() - t0) * 1e3)
        summ = plan.solve_summary()
        print(json.dumps({"workload": wl.name, "mode": mode, "dtype": "f32", "ndof": plan.ndof,
                          "apply_ms": ms_a, "apply_GDoF/s": plan.ndof / ms_a / 1e6,
                          "inverse_ms": ms_i, "inverse_GDoF/s": plan.ndof / ms_i / 1e6,
                          "solve_p50_ms": float(np.percentile(lat, 50)),
                          "solve_p99_ms": float(np.percentile(lat, 99)),
                          "solve_max_iters": summ["max_iters"], "solve_max_relres": summ["max_relres"],
                          "launch_config": config}),
              flush=True)
        if mode.endswith("_graph"):
            ga.destroy(), gi.destroy(), gs.destroy()
        plan.destroy()


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "lane.h", "device.h"):
        h.update(open(os.path.join(ROOT, "paper_2609_04534_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
