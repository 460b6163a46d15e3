"""Helpers for the GPU parity tests: move seeded host arrays through the
library's pack -> op -> unpack path and back to numpy.  Marshalling only."""
from __future__ import annotations

import numpy as np

from paper_2609_04534_amd import tpfdm

TORCH_DT = {}


def torch_dtype(code):
    import torch
    return {tpfdm.F64: torch.float64, tpfdm.F32: torch.float32, tpfdm.F16: torch.float16,
            tpfdm.BF16: torch.bfloat16}[code]


def canon(arrs):
    return np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in arrs])


def split(flat, groups):
    out, o = [], 0
    for g in groups:
        k = g.nblocks * g.n ** 3
        out.append(flat[o:o + k].reshape(g.nblocks, g.n ** 3))
        o += k
    return out


def to_blocked(plan, flat, dt, fill=None):
    import torch
    cu = torch.from_numpy(np.ascontiguousarray(flat)).to("cuda").to(torch_dtype(dt))
    bu = torch.zeros(max(plan.vector_elems, 1), dtype=torch_dtype(dt), device="cuda")
    plan.pack(cu, bu)
    return bu


def from_blocked(plan, bv, dt):
    import torch
    cv = torch.empty(max(plan.ndof, 1), dtype=torch_dtype(dt), device="cuda")
    plan.unpack(bv, cv)
    torch.cuda.synchronize()
    return cv[:plan.ndof].double().cpu().numpy()


def gpu_apply(plan, flat_u, dt=tpfdm.F64, op=tpfdm.OP_NEUMANN, sentinel=True):
    import torch
    bu = to_blocked(plan, flat_u, dt)
    bv = torch.full_like(bu, float("nan")) if sentinel else torch.empty_like(bu)
    plan.apply(bu, bv, op)
    return from_blocked(plan, bv, dt), bv


def gpu_inverse(plan, flat_r, dt=tpfdm.F64):
    import torch
    br = to_blocked(plan, flat_r, dt)
    bx = torch.full_like(br, float("nan"))
    plan.apply_inverse(br, bx)
    return from_blocked(plan, bx, dt), bx


def rel_err_blocks(got, ref):
    """max over blocks of ||got_b - ref_b||_2 / ||ref_b||_2 (rows are blocks)."""
    num = np.linalg.norm(got - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    den = np.where(den == 0, 1.0, den)
    return float(np.max(num / den)) if len(num) else 0.0
