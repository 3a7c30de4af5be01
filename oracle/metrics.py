"""Evaluation metrics of Sec. IV (oracle; test infrastructure only)."""
from __future__ import annotations

import numpy as np


def pruning_rate(n: int, n_G: int) -> float:
    """eta = 1 - d_G / d (pruning-rate equation)."""
    return 1.0 - n_G / n


def chi_hat(inst, e_hat: float) -> float:
    """Estimated Hamiltonian ratio: 1/2 - E / (2 (sqrt(d) ||J||_F + ||h||_1)).

    J is the full symmetric matrix of the E = s^T J s + h^T s convention and d
    the spin count of the original problem.
    """
    if inst.is_dense:
        fro = np.sqrt((inst.J.astype(np.float64) ** 2).sum())
    else:
        fro = np.sqrt((inst.val.astype(np.float64) ** 2).sum())
    scale = np.sqrt(inst.n) * fro + np.abs(inst.h.astype(np.float64)).sum()
    return 0.5 - float(e_hat) / (2.0 * scale)


def tts_hat(t_run: float, chi: float, d: int) -> float:
    """Estimated time-to-solution T log(1 - 0.99) / log(1 - e^chi / d).

    Defined only when e^chi < d (the estimated success probability is below 1).
    """
    p = np.exp(chi) / d
    if not (0.0 < p < 1.0):
        raise ValueError("estimated success probability outside (0, 1)")
    return t_run * np.log(1.0 - 0.99) / np.log(1.0 - p)


def speed(chi: float, t_run: float) -> float:
    """Solution speed v = chi / T."""
    return chi / t_run
