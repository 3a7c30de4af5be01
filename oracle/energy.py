"""Ising energy and exhaustive ground state (oracle; test infrastructure only).

Paper, Sec. II: E(s) = s^T J s + h^T s for s in {-1, +1}^d, with J real
symmetric, J_ii = 0 and J_ij = J-hat_ij / 2.  The double sum counts every pair
twice, so an edge of weight J_ij contributes 2 J_ij s_i s_j.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _matrix(inst):
    """J of an instance as a dense array or a scipy CSR matrix (values as stored)."""
    if inst.is_dense:
        return inst.J
    return sp.csr_matrix((inst.val, inst.col, inst.row_ptr), shape=(inst.n, inst.n))


def local_fields(inst, S):
    """Y = J S for spin columns S (n, R)."""
    return np.asarray(_matrix(inst) @ S)


def energies(inst, S):
    """E(s_r) for every column s_r of S (n, R).

    Integer instances: exact int64.  Real instances: float64.
    """
    S = np.asarray(S)
    if S.ndim == 1:
        S = S[:, None]
    if inst.integer:
        S = S.astype(np.int64)
        Y = local_fields(inst, S).astype(np.int64)
        return (S * Y).sum(axis=0) + inst.h.astype(np.int64) @ S
    S = S.astype(np.float64)
    Y = local_fields(inst, S)
    return (S * Y).sum(axis=0) + inst.h.astype(np.float64) @ S


def energy(inst, s):
    """E(s) of one spin vector."""
    return energies(inst, np.asarray(s).reshape(-1, 1))[0]


def cut_value(inst, s):
    """Weight of the cut {i : s_i = +1} | {i : s_i = -1}.

    With E = 2 sum_{i<j} J_ij s_i s_j (h = 0) and W = sum_{i<j} J_ij, the cut
    weight is (2W - E) / 4; here it is counted edge by edge instead.
    """
    rp, col, val = inst.csr()
    rows = np.repeat(np.arange(inst.n), np.diff(rp))
    upper = rows < col
    s = np.asarray(s)
    cut = s[rows[upper]] != s[col[upper]]
    return val[upper][cut].sum()


def brute_force_min(inst, chunk_bits: int = 16):
    """Exhaustive minimum of E over all 2^n spin vectors (n <= 22).

    Returns (E_min, one minimiser, number of minimisers).  The configuration
    with integer code k has s_i = +1 where bit i of k is 0.
    """
    n = inst.n
    if n > 22:
        raise ValueError("brute force limited to n <= 22")
    J = inst.dense()
    integer = inst.integer
    dt = np.int64 if integer else np.float64
    J = J.astype(dt)
    h = inst.h.astype(dt)
    best = None
    best_s = None
    count = 0
    total = 1 << n
    step = 1 << min(n, chunk_bits)
    bits = np.arange(n, dtype=np.int64)
    for start in range(0, total, step):
        codes = np.arange(start, min(total, start + step), dtype=np.int64)
        S = (1 - 2 * ((codes[:, None] >> bits[None, :]) & 1)).astype(dt)  # (chunk, n)
        E = ((S @ J) * S).sum(axis=1) + S @ h
        m = E.min()
        if best is None or m < best:
            best = m
            best_s = S[int(np.argmin(E))].astype(np.int8)
            count = int((E == m).sum())
        elif m == best:
            count += int((E == m).sum())
    return best, best_s, count
