"""Problem front-ends: QUBO, MaxCut and NAE-3SAT as Ising instances -- oracle,
test infrastructure only.

The paper states its primal problem as the ground state of E(s) = s^T J s + h^T s
over s in {-1, +1}^d (Sec. II) and benchmarks MaxCut, SK-QUBO and NAE-3SAT
instances in that form (Sec. IV-D, Table 3).  The conversions are the plain
definitions, written out:

* QUBO: f(x) = x^T Q x + c^T x with x in {0, 1}^d and x = (1 + s) / 2.  With
  Q symmetrised, f(x) = E(s) + offset for J_ij = Q_ij / 4 (i != j), J_ii = 0,
  h_i = (sum_j Q_ij + c_i) / 2 and offset = (sum_ij Q_ij + sum_i Q_ii) / 4
  + sum_i c_i / 2 (the diagonal uses x_i^2 = x_i, i.e. s_i^2 = 1).
* MaxCut with edge weights w: J = W (the table's energies satisfy
  E = 2 (m - 2 cut) for unit weights), h = 0, so E(s) = 2 W_tot - 4 cut(s)
  with W_tot the total edge weight.
* NAE-3SAT: a clause of three literals sigma_k = sign_k s_{v_k} is satisfied
  unless all three are equal, and sigma_1 sigma_2 + sigma_2 sigma_3 +
  sigma_1 sigma_3 is 3 for a violated clause and -1 otherwise.  J_ab collects
  sign_a sign_b over every literal pair (a, b) of every clause (integers, as in
  the table), so E(s) = 2 sum_clauses (pair sum) - K, where K = 2 sum of
  sign_a sign_b over pairs that repeat one variable (constant terms), and the
  number of violated clauses is U(s) = (E(s) + base) / 8 with base = K + 2M.
"""
from __future__ import annotations

import numpy as np

import instances as I


def qubo_value(Q, c, x):
    """f(x) = x^T Q x + c^T x (x in {0, 1}^d), as given."""
    x = np.asarray(x, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    v = x @ Q @ x
    if c is not None:
        v += np.asarray(c, dtype=np.float64) @ x
    return v


def qubo_to_ising(Q, c=None):
    """(J (dense, zero diagonal), h, offset) with f(x) = E(s) + offset, x = (1 + s) / 2."""
    Q = np.asarray(Q, dtype=np.float64)
    Qs = (Q + Q.T) / 2.0
    n = Qs.shape[0]
    cc = np.zeros(n) if c is None else np.asarray(c, dtype=np.float64)
    J = Qs / 4.0
    np.fill_diagonal(J, 0.0)
    h = (Qs.sum(axis=1) + cc) / 2.0
    offset = (Qs.sum() + np.trace(Qs)) / 4.0 + cc.sum() / 2.0
    return J, h, offset


def qubo_instance(Q, c=None, name="qubo"):
    J, h, off = qubo_to_ising(Q, c)
    return I.Instance(J.shape[0], name, h, J, integer=False), off


def maxcut_instance(n, edges, w=None, name="maxcut"):
    """Ising instance of MaxCut (J = W, h = 0) and the total edge weight."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    ww = np.ones(len(e), dtype=np.int64) if w is None else np.asarray(w)
    integer = np.issubdtype(ww.dtype, np.integer)
    W = np.zeros((n, n), dtype=np.int64 if integer else np.float64)
    for (a, b), x in zip(e, ww):
        if a == b:
            raise ValueError("self-loop")
        W[a, b] += x
        W[b, a] += x
    iu, ju = np.nonzero(np.triu(W, 1))
    inst = I._from_upper_edges(n, iu, ju, W[iu, ju], np.zeros(n), name, integer)
    return inst, float(ww.sum())


def cut_of(n, edges, w, s):
    """Weight of edges whose endpoints have different spins, counted edge by edge."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    ww = np.ones(len(e)) if w is None else np.asarray(w, dtype=np.float64)
    s = np.asarray(s)
    return float(ww[s[e[:, 0]] != s[e[:, 1]]].sum())


def nae3sat_instance(n, clauses, name="nae3sat"):
    """Ising instance of NAE-3SAT (integer J) and base, U(s) = (E(s) + base) / 8.

    clauses: (M, 3) signed literals, +-(v + 1) for variable v (true = spin +1)."""
    cl = np.asarray(clauses, dtype=np.int64).reshape(-1, 3)
    J = np.zeros((n, n), dtype=np.int64)
    K = 0
    for lits in cl:
        v = np.abs(lits) - 1
        sg = np.sign(lits)
        for p, q in ((0, 1), (1, 2), (0, 2)):
            if v[p] == v[q]:
                K += 2 * sg[p] * sg[q]
            else:
                J[v[p], v[q]] += sg[p] * sg[q]
                J[v[q], v[p]] += sg[p] * sg[q]
    iu, ju = np.nonzero(np.triu(J, 1))
    inst = I._from_upper_edges(n, iu, ju, J[iu, ju], np.zeros(n), name, True)
    return inst, int(K + 2 * len(cl))


def nae_violated(clauses, s):
    """Clauses whose three literal values are all equal, counted clause by clause."""
    cl = np.asarray(clauses, dtype=np.int64).reshape(-1, 3)
    s = np.asarray(s)
    vals = np.sign(cl) * s[np.abs(cl) - 1]
    return int(np.sum((vals[:, 0] == vals[:, 1]) & (vals[:, 1] == vals[:, 2])))
