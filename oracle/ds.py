"""Domain selection (Sec. III-B) -- oracle, test infrastructure only.

The primal problem min_s E(s) is rewritten as max_s ||(J - mu I) s + h||_1
(the L1-norm form of the augmented Lagrangian), whose feasible set splits into
2^d domains C_i.  The local optimum of domain C_i is the vertex
s~* = sgn(X_{i} 1) (local-optimum equation), and the discrete flip pattern
X_{i} is relaxed to sin(theta), theta = diag(theta_1..theta_d).  The loss is

    L(theta) = 1^T sin(theta) ((J - mu I) s~* + h)        (loss-function equation)

Reading taken for s~* (the paper names it the local optimum of the current
domain): under the relaxation it is the vertex of the current angles,
s~* = sgn(sin theta), with sgn(0) := +1.  It is piecewise constant in theta, so
the almost-everywhere gradient is exact:

    dL/dtheta = cos(theta) * ((J - mu I) s~* + h).

One step for every replica r (columns of the (n, R) arrays), step index t >= 1:
  1. x = sin theta, s = sgn(x)
  2. y = J s
  3. E_t = s^T (y + h)                        (energy of the current vertex)
  4. L_t = x^T (y - mu s + h)                 (loss)
  5. if E_t < E_best: E_best = E_t, s_best = s, best_step = t  (ties keep the earlier)
  6. g = cos(theta) * (y - mu s + h)
  7. GD: theta -= lr g.   ADAM (Kingma and Ba; the paper's optimiser, Sec. IV-B):
     m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
     theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
  8. theta <- theta - 2 pi rint(theta / 2 pi): sin, cos, m and v do not depend
     on the representative, so this only keeps theta small.

Second reading (relaxed vertex, loss="relaxed"): s~* := sin(theta) itself, the
relaxed flip pattern.  The loss is then smooth,

    L(theta) = x^T (J - mu I) x + h^T x,   x = sin(theta),
    dL/dtheta = cos(theta) * (2 (J - mu I) x + h)          (J symmetric),

and steps 2, 4 and 6 become z = J x, L_t = x^T (z - mu x + h),
g = cos(theta) * (2 z - 2 mu x + h); the energy of the vertex s = sgn(x) is
still tracked with y = J s (steps 3 and 5).

Convergence test (Sec. IV-B, optional): with Delta L the spread (maximum minus
minimum) of the last w = 5 losses, the paper stops when Delta L / (L_now - L_init)
<= 0.005.  The loss decreases, so that denominator is <= 0 and the inequality as
printed holds at once; the reading taken is Delta L <= tol |L_now - L_init| with
L_init = L_1, checked from step t = w on.  A replica that meets it at step t stops
after that step: its angles, moments and best vertex are final and later steps
neither update nor score it.

Initial angles (the paper says only "randomly initialized"): theta_0 = asin(U)
with U uniform on [-1, 1), so that sin theta_0 is uniform; the draws U are an
input (instances.uniform_draws).  Defaults for ADAM are Kingma and Ba's
(b1 = 0.9, b2 = 0.999, eps = 1e-8); the paper states only lr = 6.0.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclass
class DSResult:
    theta: np.ndarray        # (R, n) final angles theta_T
    m: np.ndarray            # (R, n) ADAM first moment (zeros for GD)
    v: np.ndarray            # (R, n) ADAM second moment
    e_best: np.ndarray       # (R,) best vertex energy seen (int64 for integer instances)
    s_best: np.ndarray       # (R, n) int8 vertex of e_best
    best_step: np.ndarray    # (R,) step index (1-based) of e_best
    energy_trace: Optional[np.ndarray] = None   # (T, R) E_t
    loss_trace: Optional[np.ndarray] = None     # (T, R) L_t
    sin_trace: Optional[np.ndarray] = None      # (T, R, n) sin(theta_t) after step t
    spin_trace: Optional[np.ndarray] = None     # (T, R, n) s used in step t
    conv_step: Optional[np.ndarray] = None      # (R,) step at which the convergence test held (0: never)


def _matrix(inst):
    if inst.is_dense:
        return inst.J
    return sp.csr_matrix((inst.val, inst.col, inst.row_ptr), shape=(inst.n, inst.n))


def wrap_angle(theta):
    """theta - 2 pi rint(theta / 2 pi) (rint: round half to even)."""
    return theta - 2.0 * np.pi * np.rint(theta / (2.0 * np.pi))


def _sgn1(x):
    return np.where(x >= 0, 1, -1)


def ds_loss(inst, theta, s_tilde, mu):
    """L(theta) = 1^T sin(theta) ((J - mu I) s~ + h) for columns of theta (n, R), s~ given."""
    Jm = _matrix(inst)
    y = np.asarray(Jm @ s_tilde.astype(np.float64))
    return (np.sin(theta) * (y - mu * s_tilde + inst.h.astype(np.float64)[:, None])).sum(axis=0)


def ds_grad(inst, theta, mu):
    """dL/dtheta at theta (n, R) with s~ = sgn(sin theta) held fixed."""
    s = _sgn1(np.sin(theta)).astype(np.float64)
    y = np.asarray(_matrix(inst) @ s)
    return np.cos(theta) * (y - mu * s + inst.h.astype(np.float64)[:, None])


def ds_loss_relaxed(inst, theta, mu):
    """Relaxed-vertex loss x^T (J - mu I) x + h^T x, x = sin(theta), for columns of theta (n, R)."""
    x = np.sin(theta)
    z = np.asarray(_matrix(inst) @ x)
    return (x * (z - mu * x + inst.h.astype(np.float64)[:, None])).sum(axis=0)


def ds_grad_relaxed(inst, theta, mu):
    """cos(theta) * (2 (J - mu I) sin(theta) + h) at theta (n, R)."""
    x = np.sin(theta)
    z = np.asarray(_matrix(inst) @ x)
    return np.cos(theta) * (2.0 * z - 2.0 * mu * x + inst.h.astype(np.float64)[:, None])


def converged(losses, window: int, tol: float) -> bool:
    """Convergence test on the losses L_1..L_t of one replica (t = len(losses))."""
    t = len(losses)
    if tol <= 0 or t < window:
        return False
    last = losses[t - window:]
    return max(last) - min(last) <= tol * abs(losses[-1] - losses[0])


def convergence_step(loss_trace, window: int = 5, tol: float = 0.005) -> int:
    """First step t (1-based) at which the test holds on loss_trace[:t], 0 if none."""
    for t in range(1, len(loss_trace) + 1):
        if converged(list(loss_trace[:t]), window, tol):
            return t
    return 0


def ds_run(inst, U, steps: int, opt: str = "adam", lr: float = 6.0, mu: float = 0.5,
           beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
           record: bool = False, record_sin: bool = False, loss: str = "vertex",
           conv_tol: float = 0.0, conv_window: int = 5, dtype=np.float64) -> DSResult:
    """Run ``steps`` domain-selection steps for R replicas.

    U: (R, n) uniform draws on [-1, 1) (theta_0 = asin U).
    loss: "vertex" (s~* = sgn sin theta) or "relaxed" (s~* = sin theta).
    conv_tol > 0: each replica stops after the step at which the convergence test holds.
    dtype: the floating-point type every formula of the step is evaluated in.  The
    oracle is float64 (the default); np.float32 evaluates the same formulas, in the
    same order, with float32 inputs and results -- a model of what any FP32
    implementation rounds, used only to measure how much the method itself
    amplifies FP32 rounding at a given step size (it bounds the iterate horizon over
    which an FP32 implementation can match the float64 oracle).
    """
    if loss not in ("vertex", "relaxed"):
        raise ValueError(loss)
    n = inst.n
    U = np.asarray(U, dtype=np.float64)
    R = U.shape[0]
    assert U.shape == (R, n)
    Jm = _matrix(inst)
    Jr = Jm if dtype == np.float64 else Jm.astype(dtype)   # couplings in the arithmetic type
    integer = inst.integer
    h = inst.h.astype(dtype)[:, None]
    h_int = inst.h.astype(np.int64)[:, None] if integer else None

    theta = np.arcsin(U).T.astype(dtype)   # (n, R)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    e_best = np.full(R, np.iinfo(np.int64).max if integer else np.inf,
                     dtype=np.int64 if integer else np.float64)
    s_best = np.zeros((n, R), dtype=np.int8)
    best_step = np.zeros(R, dtype=np.int64)
    et = np.zeros((steps, R), dtype=e_best.dtype) if record else None
    lt = np.zeros((steps, R)) if record else None
    st = np.zeros((steps, R, n)) if record_sin else None
    sp_t = np.zeros((steps, R, n), dtype=np.int8) if record_sin else None
    active = np.ones(R, dtype=bool)
    conv_step = np.zeros(R, dtype=np.int64)
    hist = [[] for _ in range(R)]

    for t in range(1, steps + 1):
        x = np.sin(theta)
        c = np.cos(theta)
        s = _sgn1(x)
        sf = s.astype(dtype)
        if integer:
            yi = np.asarray(Jm @ s.astype(np.int64)).astype(np.int64)
            E = (s * (yi + h_int)).sum(axis=0)
            y = yi.astype(dtype)
        else:
            y = np.asarray(Jr @ sf)
            E = (sf * (y + h)).sum(axis=0)
        if loss == "vertex":
            tt = y - mu * sf + h
            L = (x * tt).sum(axis=0)
            g = c * tt
        else:
            z = np.asarray(Jr @ x)
            L = (x * (z - mu * x + h)).sum(axis=0)
            g = c * (2.0 * z - 2.0 * mu * x + h)
        better = (E < e_best) & active
        e_best = np.where(better, E, e_best)
        s_best[:, better] = s[:, better]
        best_step[better] = t
        if opt == "gd":
            theta_n = theta - lr * g
            m_n, v_n = m, v
        elif opt == "adam":
            m_n = beta1 * m + (1.0 - beta1) * g
            v_n = beta2 * v + (1.0 - beta2) * g * g
            mhat = m_n / (1.0 - beta1 ** t)
            vhat = v_n / (1.0 - beta2 ** t)
            theta_n = theta - lr * mhat / (np.sqrt(vhat) + eps)
        else:
            raise ValueError(opt)
        theta_n = wrap_angle(theta_n)
        # replicas that stopped keep their state
        theta = np.where(active[None, :], theta_n, theta)
        m = np.where(active[None, :], m_n, m)
        v = np.where(active[None, :], v_n, v)
        if conv_tol > 0:
            for r in np.nonzero(active)[0]:
                hist[r].append(L[r])
                if converged(hist[r], conv_window, conv_tol):
                    active[r] = False
                    conv_step[r] = t
        if record:
            et[t - 1] = E
            lt[t - 1] = L
        if record_sin:
            st[t - 1] = np.sin(theta).T
            sp_t[t - 1] = s.T
    return DSResult(theta.T.copy(), m.T.copy(), v.T.copy(), e_best, s_best.T.copy(), best_step,
                    et, lt, st, sp_t, conv_step)
