"""Pruning (Algorithm 1, Sec. III-A) and retrieval (Fig. 1c) -- oracle, test infrastructure only.

Reading of Algorithm 1 taken here ("D then S, in rounds"), which reproduces all
four terms of h_G and all three terms of C_{D,S} in the reduced problem:

Each round, on the set A of still-active spins:
  1. a_i = sum_{j in A} |J_ij|; D = {i in A : |h_i| > 2 a_i}  (strict, the
     determined-spin rule); s_i = -sgn(h_i) for i in D.
  2. C += sum_{i in D} h_i s_i + sum_{i,j in D} J_ij s_i s_j (ordered pairs);
     for j in A \\ D: h_j += 2 sum_{i in D} J_ji s_i;  A <- A \\ D.
  3. deg_k = #{j in A : J_kj != 0}.  K = {k : deg_k = 1 and 2|J_k,n(k)| >= |h_k|}
     (the semi-determined-spin rule, non-strict) with n(k) the unique active
     neighbour.  If k and n(k) are both in K and are each other's neighbour
     they would fix each other, so only the larger index of the pair is taken:
     S = K minus those smaller partners.
  4. For k in S, with i = n(k) and sigma = sgn(J_ki): record (k, i, sigma);
     h_i -= sum over those k of sigma h_k; C -= 2 |J_ki|;  A <- A \\ S.
  5. Stop when D and S are both empty.  G = A (ascending original index),
     J_G = J[G, G], h_G = h[G].

Because D is folded into h before S is chosen, the h_k used in step 4 already
carries the D terms; this is the fourth term of h_G in the paper.

Retrieval: s[G] = s_G, then rounds in reverse: s_k = -sigma s_i for S records
(n(k) survives its round, so it is already resolved) and the recorded value for
D records.

Rounding convention for real couplings (a reading; the paper is silent).  The
decisions of the algorithm (determined test, semi-determined test) compare a
field with the row sums a_i, so a_i is formed in one fixed order that any
implementation can follow and reproduce bit for bit: the stored entries of row
i (all n columns for a dense matrix, the stored nonzeros in ascending column
order for CSR) are numbered p = 0, 1, ...; partial sum l (0 <= l < 64) adds
the terms of p = l, l + 64, l + 128, ... in ascending p (0 for entries that do
not take part); then the 64 partials are combined pairwise by index xor 32, 16,
8, 4, 2, 1.  Everything else is the plain definition, summed one term after
another in ascending index: the fold of the determined spins into h_j (the
terms 2 J_ji s_i for i in D, added to h_j once summed), the fold of the
semi-determined spins into h_i (the terms sgn(J_ik) h_k for k in S with
n(k) = i, subtracted once summed) and the D-D couplings of C.  Another
summation order changes h_G and C only by rounding, bounded by
gamma_k * (sum of the magnitudes of the terms that make them up); those
magnitudes are returned as ``h_mass`` and ``C_mass`` so that a comparison can
state that bound.  Integer couplings are summed exactly in int64, where order
is irrelevant.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


LANES = 64


@dataclass
class PruneResult:
    n: int
    G: np.ndarray                 # surviving original indices, ascending
    h_G: np.ndarray               # reduced field
    C: object                     # constant of the reduced problem
    reduced: object               # instances.Instance on G (indices 0..|G|-1)
    kind: np.ndarray              # per spin: 0 = G, 1 = determined, 2 = semi-determined
    round_of: np.ndarray          # per spin: round index (0-based) it was pruned in, -1 for G
    fixed: np.ndarray             # per spin: s_i for determined spins, 0 otherwise
    partner: np.ndarray           # per spin: n(k) for semi-determined spins, -1 otherwise
    sigma: np.ndarray             # per spin: sgn(J_k,n(k)) for semi-determined spins, 0 otherwise
    rounds: int                   # rounds executed (the last one removes nothing)
    per_round: list = field(default_factory=list)  # (|D|, |S|) per round
    # rounding-bound helpers (real couplings): per spin, the sum of the magnitudes of the
    # terms whose sum is h_G (initial |h| plus every folded term, recursively); for C, the same
    h_mass: Optional[np.ndarray] = None
    C_mass: float = 0.0

    @property
    def eta(self) -> float:
        return 1.0 - self.G.shape[0] / self.n


def _entries(inst):
    """All stored entries as (row, col, val, pos): dense rows list every column."""
    n = inst.n
    if inst.is_dense:
        rows = np.repeat(np.arange(n), n)
        cols = np.tile(np.arange(n), n)
        vals = inst.J.reshape(-1)
        pos = cols.copy()
    else:
        counts = np.diff(inst.row_ptr)
        rows = np.repeat(np.arange(n), counts)
        cols = inst.col.astype(np.int64)
        vals = inst.val
        pos = np.arange(cols.shape[0]) - inst.row_ptr[rows]
    return rows, cols, vals, pos


def fixed_order_rowsum(n, rows, pos, terms, integer):
    """Per-row sums of per-entry terms in the fixed 64-partial order described above."""
    if integer:
        return _exact_int_rowsum(n, rows, terms)
    acc = np.zeros((n, LANES), dtype=np.float64)
    chunk = pos // LANES
    lane = pos % LANES
    terms = terms.astype(np.float64)
    for k in range(int(chunk.max()) + 1 if chunk.size else 0):
        sel = chunk == k
        acc[rows[sel], lane[sel]] = acc[rows[sel], lane[sel]] + terms[sel]
    idx = np.arange(LANES)
    for d in (32, 16, 8, 4, 2, 1):
        acc = acc + acc[:, idx ^ d]
    return acc[:, 0]


def ascending_rowsum(n, rows, pos, terms, integer):
    """Per-row sums of per-entry terms, each row's terms added one after another in
    ascending stored position (numpy's accumulate is that sequential recurrence)."""
    if integer:
        return _exact_int_rowsum(n, rows, terms)
    width = int(pos.max()) + 1 if pos.size else 1
    mat = np.zeros((n, width), dtype=np.float64)
    mat[rows, pos] = terms
    return np.add.accumulate(mat, axis=1)[:, -1]


def _ascending_sum(x, integer):
    """Sum of a 1-D array, one term after another in index order."""
    if integer:
        return np.asarray(x, dtype=np.int64).sum()
    x = np.asarray(x, dtype=np.float64)
    return np.add.accumulate(x)[-1] if x.size else 0.0


def fixed_order_abs_rowsum(n, rows, cols, vals, pos, active, integer):
    """a_i = sum_{j active} |J_ij| in the fixed 64-partial order described above."""
    return fixed_order_rowsum(n, rows, pos, np.abs(vals) * active[cols] * active[rows], integer)


def _exact_int_rowsum(n, rows, mag):
    out = np.zeros(n, dtype=np.int64)
    np.add.at(out, rows, mag.astype(np.int64))
    return out


def _sgn(x):
    return np.where(x > 0, 1, np.where(x < 0, -1, 0)).astype(np.int64)


def prune(inst) -> PruneResult:
    """Run Algorithm 1 to completion on ``inst`` (instances.Instance)."""
    from instances import Instance  # generator container only

    n = inst.n
    integer = inst.integer
    dt = np.int64 if integer else np.float64
    rows, cols, vals, pos = _entries(inst)
    vals = vals.astype(dt)
    # per-row slices of the entry list (rows are contiguous and ascending)
    starts = np.searchsorted(rows, np.arange(n), side="left")
    ends = np.searchsorted(rows, np.arange(n), side="right")

    h = inst.h.astype(dt).copy()
    h_mass = np.abs(inst.h).astype(np.float64)
    C_mass = 0.0
    absv = np.abs(vals).astype(np.float64)
    active = np.ones(n, dtype=bool)
    C = dt(0)
    kind = np.zeros(n, dtype=np.int8)
    round_of = np.full(n, -1, dtype=np.int32)
    fixed = np.zeros(n, dtype=np.int8)
    partner = np.full(n, -1, dtype=np.int64)
    sigma = np.zeros(n, dtype=np.int8)
    per_round = []
    rnd = 0
    ar = np.arange(n)
    while True:
        # 1. determined spins (the decision uses the fixed-order row sums)
        a = fixed_order_abs_rowsum(n, rows, cols, vals, pos, active, integer)
        D = active & (np.abs(h) > 2 * a)
        Didx = np.nonzero(D)[0]
        sD = -_sgn(h[Didx])
        s_full = np.zeros(n, dtype=dt)
        s_full[Didx] = sD
        # 2. fold D into C (terms h_i s_i + sum_{j in D} J_ij s_i s_j, i ascending, added to
        #    C one after another) and into the fields of the remaining active spins
        if Didx.size:
            dd = ascending_rowsum(n, rows, pos, vals * s_full[rows] * s_full[cols], integer)
            C = _ascending_sum(np.r_[np.asarray([C], dtype=dt), h[Didx] * sD + dd[Didx]], integer)
            inD = np.zeros(n, dtype=np.float64)
            inD[Didx] = 1.0
            C_mass += float((h_mass[Didx]).sum() + (absv * inD[rows] * inD[cols]).sum())
            keep = active & ~D
            F = ascending_rowsum(n, rows, pos, 2 * vals * s_full[cols], integer)
            h[keep] = h[keep] + F[keep]
            Fm = np.zeros(n)
            np.add.at(Fm, rows, 2 * absv * inD[cols])
            h_mass[keep] += Fm[keep]
            kind[Didx] = 1
            round_of[Didx] = rnd
            fixed[Didx] = sD
            active[Didx] = False
        # 3. semi-determined spins among the remaining active spins
        live = (vals != 0) & active[rows] & active[cols]
        deg = np.bincount(rows[live], minlength=n)
        cand = active & (deg == 1)
        nb = np.full(n, -1, dtype=np.int64)
        jv = np.zeros(n, dtype=dt)
        sel = live & cand[rows]
        nb[rows[sel]] = cols[sel]
        jv[rows[sel]] = vals[sel]
        cand &= (2 * np.abs(jv) >= np.abs(h))
        nbc = np.where(nb >= 0, nb, 0)
        mutual = cand & (nb >= 0) & cand[nbc] & (nb[nbc] == ar)
        S = cand & ~(mutual & (ar < nb))
        Sidx = np.nonzero(S)[0]
        # 4. fold S: h_i -= sum over k in S with n(k) = i of sgn(J_ik) h_k (k ascending);
        #    C -= 2 |J_k,n(k)| for k in S, one after another
        if Sidx.size:
            to_me = S[cols] & (nb[cols] == rows)
            G_ = ascending_rowsum(n, rows, pos, np.where(to_me, _sgn(vals) * h[cols], 0), integer)
            rest = active & ~S
            h[rest] = h[rest] - G_[rest]
            Gm = np.zeros(n)
            np.add.at(Gm, rows, np.where(to_me, h_mass[cols], 0.0))
            h_mass[rest] += Gm[rest]
            C = _ascending_sum(np.r_[np.asarray([C], dtype=dt), -2 * np.abs(jv[Sidx])], integer)
            C_mass += float(2 * np.abs(jv[Sidx]).astype(np.float64).sum())
            kind[Sidx] = 2
            round_of[Sidx] = rnd
            partner[Sidx] = nb[Sidx]
            sigma[Sidx] = _sgn(jv[Sidx])
            active[Sidx] = False
        per_round.append((int(Didx.size), int(Sidx.size)))
        rnd += 1
        if Didx.size == 0 and Sidx.size == 0:
            break

    G = np.nonzero(active)[0]
    h_G = h[G]
    remap = np.full(n, -1, dtype=np.int64)
    remap[G] = np.arange(G.size)
    if inst.is_dense:
        red = Instance(G.size, inst.name + "/G", h_G.copy(), inst.J[np.ix_(G, G)].astype(dt),
                       integer=integer)
    else:
        keepe = active[rows] & active[cols] & (vals != 0)
        r2, c2, v2 = remap[rows[keepe]], remap[cols[keepe]], vals[keepe]
        rp = np.zeros(G.size + 1, dtype=np.int64)
        np.add.at(rp, r2 + 1, 1)
        red = Instance(G.size, inst.name + "/G", h_G.copy(), None, np.cumsum(rp), c2, v2, integer)
    return PruneResult(n, G, h_G, C, red, kind, round_of, fixed, partner, sigma, rnd, per_round,
                       h_mass[G].copy(), C_mass)


def unprune(res: PruneResult, s_G) -> np.ndarray:
    """Full spin vector from the reduced-problem spins and the pruning record."""
    s = np.zeros(res.n, dtype=np.int64)
    s[res.G] = np.asarray(s_G, dtype=np.int64)
    for rnd in range(res.rounds - 1, -1, -1):
        here = res.round_of == rnd
        d = here & (res.kind == 1)
        s[d] = res.fixed[d]
        k = np.nonzero(here & (res.kind == 2))[0]
        s[k] = -res.sigma[k].astype(np.int64) * s[res.partner[k]]
    assert np.all(np.abs(s) == 1)
    return s.astype(np.int8)
