"""Helpers for the GPU tests: move seeded instances onto the device (marshalling only)."""
import numpy as np

import instances as I


def to_problem(inst, real_dtype=None, with_zero_h=False):
    import torch
    import paper_2312_05837_amd as P

    if inst.integer:
        dt = torch.int32
    else:
        dt = real_dtype or torch.float64
    has_h = with_zero_h or bool(np.any(inst.h != 0))
    h = torch.tensor(inst.h, dtype=dt, device="cuda") if has_h else None
    if inst.is_dense:
        return P.dense_problem(torch.tensor(inst.J, dtype=dt, device="cuda"), h)
    return P.csr_problem(torch.tensor(inst.row_ptr, dtype=torch.int32, device="cuda"),
                         torch.tensor(inst.col, dtype=torch.int32, device="cuda"),
                         torch.tensor(inst.val, dtype=dt, device="cuda"), h)


def as_float32_instance(inst):
    """Same instance with values rounded to float32 (what an F32 problem holds), kept as float64."""
    out = I.Instance(inst.n, inst.name + "/f32", inst.h.astype(np.float32).astype(np.float64),
                     None if inst.J is None else inst.J.astype(np.float32).astype(np.float64),
                     inst.row_ptr, inst.col,
                     None if inst.val is None else inst.val.astype(np.float32).astype(np.float64),
                     False, dict(inst.meta))
    return out


def energy_bound(inst):
    """gamma_{n+1} (sum|J| + sum|h|): summation error bound of an FP64 energy in any order."""
    u = 2.0 ** -53
    k = inst.n + 1
    gamma = k * u / (1 - k * u)
    s = (np.abs(inst.val).sum() if not inst.is_dense else np.abs(inst.J).sum()) + np.abs(inst.h).sum()
    return gamma * s


def iterate_error(sin_gpu, sin_ref):
    """Per-replica norm-wise relative error max_i |a - b| / max_i |b| (rows = replicas)."""
    den = np.maximum(np.abs(sin_ref).max(axis=1), 1e-300)
    return np.abs(sin_gpu - sin_ref).max(axis=1) / den
