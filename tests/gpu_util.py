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


def int8_represented(inst, digits):
    """The couplings the INT8 matrix-core forms compute with: J = 2^e Jq, Jq = rint(J / 2^e), e the
    smallest exponent in [-126, 127] with max|J| <= 2^e qmax and max_i sum_j |J_ij| + 2^e 257 n <=
    2^e (2^31 - 1) (qmax = 8355711 for three INT8 digits, 32639 for two), as the library documents
    the form; returns (instance with those couplings, e)."""
    qmax = {3: 8355711.0, 2: 32639.0}[digits]
    J = inst.J
    big = float(np.abs(J).max())
    rsum = float(np.abs(J).sum(axis=1).max())
    lim = 2.0 ** 31 - 1

    def fits(e):
        return big <= np.ldexp(qmax, e) and rsum + np.ldexp(257.0 * inst.n, e) <= np.ldexp(lim, e)

    e = -126
    while e < 127 and not fits(e):
        e += 1
    Jq = np.rint(np.ldexp(J, -e))
    assert np.abs(Jq).max() <= qmax
    rep = I.Instance(inst.n, f"{inst.name}/i8x{digits}", inst.h.copy(), np.ldexp(Jq, e), integer=inst.integer)
    return rep, e


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


def _subset(got, sel):
    out = dict(got)
    for k in ("theta", "m", "v", "s_best", "e_best", "best_step"):
        out[k] = got[k][sel]
    out["energy_trace"] = got["energy_trace"][:, sel]
    out["loss_trace"] = got["loss_trace"][:, sel]
    out["thetas"] = [t[sel] for t in got["thetas"]]
    return out


def compare_trajectories(inst, got, U, steps, opt, lr, chunks, TOL=1e-5, check_loss=True, max_excluded=None,
                         check_energy=True, loss="vertex"):
    """Oracle vs GPU iterates at every chunk boundary; exact energies for integer instances.

    A replica is compared up to the first step where its vertex may legitimately
    differ from the oracle's: a spin whose oracle |sin theta| is below TOL.  Vertex
    differences are seen every step through the energy trace (exact for integer
    instances, else beyond the energy tolerance) and at chunk boundaries through
    the signs of sin theta; each must sit at such a near-zero, else the test fails.
    """
    import oracle
    R = U.shape[0]
    if R > 128:  # the oracle checks the first and last 64 replicas (trajectories are independent)
        sel = np.r_[0:64, R - 64:R]
        got = _subset(got, sel)
        U = U[sel]
        R = U.shape[0]
    ref = oracle.ds_run(inst, U, steps, opt=opt, lr=lr, mu=0.5, record=True, record_sin=True, loss=loss)
    # vertex of step t is sgn(sin theta_{t-1}); theta_0 = asin U
    min_prev = np.empty((steps, R))
    min_prev[0] = np.abs(U).min(axis=1)
    min_prev[1:] = np.abs(ref.sin_trace[:-1]).min(axis=2)
    scale = np.abs(ref.energy_trace).max() + 1.0
    e_tol = max(1e-4, TOL) * scale
    excl_from = np.full(R, steps + 1)  # first step a replica is no longer compared
    if inst.integer or check_energy:
        ref_e = ref.energy_trace.astype(np.float64)
        if inst.integer:
            differ = got["energy_trace"] != ref_e
        else:
            differ = np.abs(got["energy_trace"] - ref_e) > e_tol
        for r in np.nonzero(differ.any(axis=0))[0]:
            t_m = int(np.argmax(differ[:, r])) + 1
            assert min_prev[t_m - 1, r] < TOL, f"replica {r}: vertex differs away from a discontinuity at step {t_m}"
            excl_from[r] = t_m
    per = steps // chunks
    worst = 0.0
    for c, th in enumerate(got["thetas"]):
        t = (c + 1) * per
        live = excl_from > t
        s_ref = ref.sin_trace[t - 1]
        s_gpu = np.sin(th)
        flip = (np.sign(s_ref) != np.sign(s_gpu)) & (s_ref != 0)
        legit = flip & (np.abs(s_ref) < TOL)
        assert not np.any(flip & ~legit & live[:, None]), f"vertex differs away from a discontinuity at step {t}"
        excl_from[legit.any(axis=1) & live] = t + 1
        live = excl_from > t
        err = iterate_error(s_gpu, s_ref)
        err[~live] = 0
        worst = max(worst, err.max())
    assert worst <= TOL, worst
    excluded = excl_from <= steps
    keep = ~excluded
    assert excluded.sum() <= (max(1, R // 16) if max_excluded is None else max_excluded), excluded.sum()
    # per-step traces up to each replica's exclusion step
    rows = np.arange(steps)[:, None] + 1 < excl_from[None, :]
    if inst.integer:
        assert np.array_equal(np.where(rows, got["energy_trace"], 0), np.where(rows, ref.energy_trace, 0))
        assert np.array_equal(got["e_best"][keep], ref.e_best[keep].astype(np.float64))
        assert np.array_equal(got["best_step"][keep], ref.best_step[keep])
        assert np.array_equal(got["s_best"][keep], ref.s_best[keep])
    elif check_energy:
        assert np.abs(np.where(rows, got["energy_trace"] - ref.energy_trace, 0)).max() <= e_tol
    if check_loss:
        scale_l = np.abs(ref.loss_trace).max() + 1.0
        assert np.abs(np.where(rows, got["loss_trace"] - ref.loss_trace, 0)).max() <= 1e-4 * scale_l
    return worst, int(excluded.sum())
