"""Seeded synthetic Ising instances and the random draws of domain selection.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
no arithmetic of the solver itself: it only builds couplings J, fields h and
uniform random numbers, so both implementations see identical inputs.

Conventions (paper, Sec. II, scalar energy form): the energy is
E(s) = s^T J s + h^T s with J symmetric and J_ii = 0.  Generators return J in
that convention; Table-1-shaped workloads are drawn as J-hat and halved, since
the paper defines J_ij = J-hat_ij / 2.

Sparse instances are stored as CSR with both directions of every edge present
and column indices ascending within each row.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# ---------------------------------------------------------------------------
# instance container
# ---------------------------------------------------------------------------


@dataclass
class Instance:
    """An Ising instance (J, h) in dense or CSR form.

    ``integer`` is True when every J_ij and h_i is an integer (values are then
    held in int64 arrays); otherwise values are float64.
    """

    n: int
    name: str
    h: np.ndarray
    J: Optional[np.ndarray] = None          # dense (n, n)
    row_ptr: Optional[np.ndarray] = None    # CSR (n+1,) int64
    col: Optional[np.ndarray] = None        # CSR (nnz,) int64, ascending per row
    val: Optional[np.ndarray] = None        # CSR (nnz,)
    integer: bool = False
    meta: dict = field(default_factory=dict)

    @property
    def is_dense(self) -> bool:
        return self.J is not None

    @property
    def nnz(self) -> int:
        if self.is_dense:
            return int(np.count_nonzero(self.J))
        return int(self.col.shape[0])

    def dense(self) -> np.ndarray:
        if self.is_dense:
            return self.J
        out = np.zeros((self.n, self.n), dtype=self.val.dtype)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        out[rows, self.col] = self.val
        return out

    def csr(self):
        """(row_ptr, col, val) of the nonzero couplings."""
        if not self.is_dense:
            return self.row_ptr, self.col, self.val
        rows, cols = np.nonzero(self.J)
        vals = self.J[rows, cols]
        row_ptr = np.zeros(self.n + 1, dtype=np.int64)
        np.add.at(row_ptr, rows + 1, 1)
        return np.cumsum(row_ptr), cols.astype(np.int64), vals

    def as_csr(self) -> "Instance":
        rp, c, v = self.csr()
        return Instance(self.n, self.name + "/csr", self.h.copy(), None, rp, c, v,
                        self.integer, dict(self.meta))

    def as_dense(self) -> "Instance":
        return Instance(self.n, self.name + "/dense", self.h.copy(), self.dense().copy(),
                        None, None, None, self.integer, dict(self.meta))


def _vals(x, integer):
    return np.asarray(x, dtype=np.int64 if integer else np.float64)


def _from_upper_edges(n, ei, ej, w, h, name, integer, meta=None) -> Instance:
    """Build a symmetric CSR instance from undirected edges (i < j) with weights."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    w = _vals(w, integer)
    keep = w != 0
    ei, ej, w = ei[keep], ej[keep], w[keep]
    rows = np.concatenate([ei, ej])
    cols = np.concatenate([ej, ei])
    vals = np.concatenate([w, w])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if dup.any():
            raise ValueError("duplicate edge")
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return Instance(n, name, _vals(h, integer), None, np.cumsum(row_ptr), cols, vals,
                    integer, meta or {})


def _dense_from_upper(upper, h, name, integer, meta=None) -> Instance:
    J = np.triu(upper, 1)
    J = J + J.T
    return Instance(J.shape[0], name, _vals(h, integer), _vals(J, integer), integer=integer,
                    meta=meta or {})


# ---------------------------------------------------------------------------
# workload generators (shapes of the paper's experiments and the configs)
# ---------------------------------------------------------------------------


def sk_pm1(n: int, seed: int) -> Instance:
    """Dense SK instance: J_ij = J_ji uniform on {-1, +1}, J_ii = 0, h = 0."""
    rng = np.random.default_rng(seed)
    upper = rng.choice(np.array([-1, 1], dtype=np.int64), size=(n, n))
    return _dense_from_upper(upper, np.zeros(n), f"sk_pm1_n{n}_s{seed}", True,
                             {"kind": "sk_pm1", "seed": seed})


def sk_gauss(n: int, seed: int, sigma: Optional[float] = None) -> Instance:
    """Dense SK instance with Gaussian couplings J_ij ~ N(0, 1/n) (default), h = 0."""
    rng = np.random.default_rng(seed)
    sigma = 1.0 / np.sqrt(n) if sigma is None else sigma
    upper = rng.normal(0.0, sigma, size=(n, n))
    return _dense_from_upper(upper, np.zeros(n), f"sk_gauss_n{n}_s{seed}", False,
                             {"kind": "sk_gauss", "seed": seed, "sigma": sigma})


def erdos_renyi(n: int, p: float, seed: int, weights: str = "pm1") -> Instance:
    """G(n, p) graph; weights 'pm1' (iid +-1) or 'one' (all +1); h = 0."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    mask = rng.random(iu.shape[0]) < p
    ei, ej = iu[mask], ju[mask]
    if weights == "pm1":
        w = rng.choice(np.array([-1, 1], dtype=np.int64), size=ei.shape[0])
    elif weights == "one":
        w = np.ones(ei.shape[0], dtype=np.int64)
    else:
        raise ValueError(weights)
    return _from_upper_edges(n, ei, ej, w, np.zeros(n), f"er_n{n}_p{p}_{weights}_s{seed}", True,
                             {"kind": "er", "p": p, "weights": weights, "seed": seed})


def torus(lx: int, ly: int, seed: int, weights: str = "pm1") -> Instance:
    """2D periodic lattice lx x ly (degree 4 when lx, ly >= 3); h = 0."""
    rng = np.random.default_rng(seed)
    n = lx * ly
    idx = np.arange(n).reshape(ly, lx)
    right = np.roll(idx, -1, axis=1)
    down = np.roll(idx, -1, axis=0)
    a = np.concatenate([idx.ravel(), idx.ravel()])
    b = np.concatenate([right.ravel(), down.ravel()])
    ei, ej = np.minimum(a, b), np.maximum(a, b)
    if weights == "pm1":
        w = rng.choice(np.array([-1, 1], dtype=np.int64), size=ei.shape[0])
    elif weights == "one":
        w = np.ones(ei.shape[0], dtype=np.int64)
    else:
        raise ValueError(weights)
    return _from_upper_edges(n, ei, ej, w, np.zeros(n), f"torus_{lx}x{ly}_{weights}_s{seed}", True,
                             {"kind": "torus", "lx": lx, "ly": ly, "weights": weights, "seed": seed})


def random_regular_edges(n: int, k: int, rng) -> tuple[np.ndarray, np.ndarray]:
    """Simple k-regular graph by the pairing (configuration) model with rejection."""
    if (n * k) % 2:
        raise ValueError("n*k must be even")
    for _ in range(10000):
        stubs = np.repeat(np.arange(n), k)
        rng.shuffle(stubs)
        a, b = stubs[0::2], stubs[1::2]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        key = lo * n + hi
        if np.unique(key).shape[0] != key.shape[0]:
            continue
        return lo, hi
    # fall back to edge switching repairs for large k
    raise RuntimeError("pairing model failed")


def _random_regular_switch(n: int, k: int, rng) -> tuple[np.ndarray, np.ndarray]:
    """k-regular graph: pairing model, then random double-edge swaps remove loops/multi-edges."""
    stubs = np.repeat(np.arange(n), k)
    rng.shuffle(stubs)
    a, b = list(stubs[0::2]), list(stubs[1::2])
    m = len(a)

    def bad(i):
        return a[i] == b[i]

    for _ in range(200 * m):
        seen = {}
        badset = []
        for e in range(m):
            lo, hi = min(a[e], b[e]), max(a[e], b[e])
            if lo == hi or (lo, hi) in seen:
                badset.append(e)
            else:
                seen[(lo, hi)] = e
        if not badset:
            break
        for e in badset:
            f = int(rng.integers(m))
            if f == e:
                continue
            # swap endpoints b[e] <-> b[f]
            a1, b1, a2, b2 = a[e], b[f], a[f], b[e]
            if a1 == b1 or a2 == b2:
                continue
            b[e], b[f] = b1, b2
    a, b = np.array(a), np.array(b)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = lo * n + hi
    if np.any(lo == hi) or np.unique(key).shape[0] != key.shape[0]:
        raise RuntimeError("could not build simple regular graph")
    return lo, hi


def random_regular(n: int, k: int, seed: int, weights: str = "pm1") -> Instance:
    """Random simple k-regular graph with iid +-1 (or all +1) weights, h = 0."""
    rng = np.random.default_rng(seed)
    try:
        ei, ej = random_regular_edges(n, k, rng) if k <= 4 else _random_regular_switch(n, k, rng)
    except RuntimeError:
        ei, ej = _random_regular_switch(n, k, rng)
    if weights == "pm1":
        w = rng.choice(np.array([-1, 1], dtype=np.int64), size=ei.shape[0])
    else:
        w = np.ones(ei.shape[0], dtype=np.int64)
    return _from_upper_edges(n, ei, ej, w, np.zeros(n), f"reg{k}_n{n}_{weights}_s{seed}", True,
                             {"kind": "regular", "k": k, "weights": weights, "seed": seed})


def table1_regular(n: int, k: int, dist: str, seed: int) -> Instance:
    """k-regular instance shaped like the pruning-rate workload (Sec. IV-A, Table 1).

    dist='uniform': J-hat ~ U(-1, 1), h-hat ~ U(-6, 6);
    dist='gaussian': J-hat ~ N(0, 1/3), h-hat ~ N(0, 12) (variances);
    dist='binary':  J-hat = +-1/sqrt(3), h-hat = +-2 sqrt(3);
    dist='binary_int': the binary case rescaled by 2 sqrt(3) and written in J terms,
    J = +-1, h = +-12, so that the tie 2 sum|J| = |h| is exact in integers.
    Real cases are drawn as J-hat and halved to J (paper, Sec. II).
    """
    rng = np.random.default_rng(seed)
    if k <= 4:
        ei, ej = random_regular_edges(n, k, rng)
    else:
        ei, ej = _random_regular_switch(n, k, rng)
    m = ei.shape[0]
    if dist == "uniform":
        jh = rng.uniform(-1.0, 1.0, size=m)
        hh = rng.uniform(-6.0, 6.0, size=n)
        return _from_upper_edges(n, ei, ej, jh / 2.0, hh, f"t1_uniform_n{n}_s{seed}", False,
                                 {"kind": "table1", "dist": dist, "seed": seed, "k": k})
    if dist == "gaussian":
        jh = rng.normal(0.0, np.sqrt(1.0 / 3.0), size=m)
        hh = rng.normal(0.0, np.sqrt(12.0), size=n)
        return _from_upper_edges(n, ei, ej, jh / 2.0, hh, f"t1_gaussian_n{n}_s{seed}", False,
                                 {"kind": "table1", "dist": dist, "seed": seed, "k": k})
    if dist == "binary":
        jh = rng.choice([-1.0, 1.0], size=m) / np.sqrt(3.0)
        hh = rng.choice([-1.0, 1.0], size=n) * 2.0 * np.sqrt(3.0)
        return _from_upper_edges(n, ei, ej, jh / 2.0, hh, f"t1_binary_n{n}_s{seed}", False,
                                 {"kind": "table1", "dist": dist, "seed": seed, "k": k})
    if dist == "binary_int":
        jv = rng.choice(np.array([-1, 1], dtype=np.int64), size=m)
        hv = rng.choice(np.array([-12, 12], dtype=np.int64), size=n)
        return _from_upper_edges(n, ei, ej, jv, hv, f"t1_binint_n{n}_s{seed}", True,
                                 {"kind": "table1", "dist": dist, "seed": seed, "k": k})
    raise ValueError(dist)


def random_integer_field(inst: Instance, seed: int, hmax: int) -> Instance:
    """Same couplings with an iid integer field h_i uniform on [-hmax, hmax]."""
    rng = np.random.default_rng(seed)
    h = rng.integers(-hmax, hmax + 1, size=inst.n).astype(np.int64)
    out = Instance(inst.n, inst.name + f"_h{hmax}", h, inst.J, inst.row_ptr, inst.col, inst.val,
                   inst.integer, dict(inst.meta))
    return out


def planted(inst: Instance, seed: int) -> tuple[Instance, np.ndarray]:
    """Unfrustrated copy with a known ground state tau.

    J_ij <- -tau_i tau_j |J_ij|, h_i <- -tau_i |h_i|: every term of the energy is
    minimised by s = tau at once, so E0 = -sum_ij |J_ij| - sum_i |h_i|.
    """
    rng = np.random.default_rng(seed)
    tau = rng.choice(np.array([-1, 1], dtype=np.int64), size=inst.n)
    h = -tau * np.abs(inst.h)
    if inst.is_dense:
        J = -np.outer(tau, tau) * np.abs(inst.J)
        out = Instance(inst.n, inst.name + "_planted", h.astype(inst.h.dtype), J.astype(inst.J.dtype),
                       integer=inst.integer, meta=dict(inst.meta))
    else:
        rows = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
        val = -tau[rows] * tau[inst.col] * np.abs(inst.val)
        out = Instance(inst.n, inst.name + "_planted", h.astype(inst.h.dtype), None, inst.row_ptr.copy(),
                       inst.col.copy(), val.astype(inst.val.dtype), inst.integer, dict(inst.meta))
    return out, tau


def from_edges(n: int, edges, h, name: str = "graph", integer: bool = True) -> Instance:
    """Small hand-made graphs: edges is a list of (i, j, w)."""
    if len(edges):
        e = np.asarray(edges)
        ei, ej, w = e[:, 0].astype(np.int64), e[:, 1].astype(np.int64), e[:, 2]
        lo, hi = np.minimum(ei, ej), np.maximum(ei, ej)
    else:
        lo = hi = np.zeros(0, dtype=np.int64)
        w = np.zeros(0)
    return _from_upper_edges(n, lo, hi, w, h, name, integer)


def random_forest_plus_cycles(n: int, seed: int, n_extra: int = 0, hmax: int = 0) -> Instance:
    """Random recursive forest (~3 trees) on n vertices plus n_extra chords, +-1 weights.

    Mixes tree components, which pruning peels to a centre, with cycles, which
    survive as a 2-core; an optional integer field exercises determined spins.
    """
    rng = np.random.default_rng(seed)
    edges = {}
    for v in range(1, n):
        if rng.random() < 0.08:
            continue  # start a new tree
        u = int(rng.integers(0, v))
        edges[(u, v)] = int(rng.choice([-1, 1]))
    added = 0
    while added < n_extra:
        u, v = sorted(int(x) for x in rng.integers(0, n, size=2))
        if u == v or (u, v) in edges:
            continue
        edges[(u, v)] = int(rng.choice([-1, 1]))
        added += 1
    h = rng.integers(-hmax, hmax + 1, size=n) if hmax > 0 else np.zeros(n, dtype=np.int64)
    e = [(u, v, w) for (u, v), w in sorted(edges.items())]
    return from_edges(n, e, h, f"forest_n{n}_s{seed}_x{n_extra}_h{hmax}", True)


# ---------------------------------------------------------------------------
# random draws of domain selection: a counter-based SplitMix64 stream
# ---------------------------------------------------------------------------

SPLITMIX_GAMMA = np.uint64(0x9E3779B97F4A7C15)
SPLITMIX_M1 = np.uint64(0xBF58476D1CE4E5B9)
SPLITMIX_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter: np.ndarray) -> np.ndarray:
    """Output number (counter + 1) of a SplitMix64 generator seeded with ``seed``.

    SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the state advances by the
    golden gamma 0x9E3779B97F4A7C15 and each output is the state passed through
    the mix z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
    z *= 0x94D049BB133111EB; z ^= z >> 31 (all modulo 2^64).
    """
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * SPLITMIX_GAMMA
        z = (z ^ (z >> np.uint64(30))) * SPLITMIX_M1
        z = (z ^ (z >> np.uint64(27))) * SPLITMIX_M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_draws(seed: int, replicas: int, n: int, replica_offset: int = 0) -> np.ndarray:
    """U[r, i] uniform on [-1, 1), keyed by (seed, replica r, spin i).

    Counter c = (r << 32) | i; U = 2 * (top 24 bits of splitmix64 / 2^24) - 1, a
    value exactly representable in float32, so every precision sees the same draw.
    """
    r = np.arange(replica_offset, replica_offset + replicas, dtype=np.uint64)[:, None]
    i = np.arange(n, dtype=np.uint64)[None, :]
    z = splitmix64(seed, (r << np.uint64(32)) | i)
    u24 = (z >> np.uint64(40)).astype(np.float64)
    return 2.0 * (u24 / 16777216.0) - 1.0


# ---------------------------------------------------------------------------
# serving request stream
# ---------------------------------------------------------------------------


def serving_stream(count: int, seed: int, rate: float, nmin: int = 64, nmax: int = 4096,
                   dense_frac: float = 0.5, avg_degree: float = 8.0,
                   replica_choices=(64, 128, 256, 512, 1024)):
    """Poisson stream of request descriptors (arrival time, kind, n, replicas, seed).

    n is log-uniform on [nmin, nmax]; half the requests are dense SK +-1, the
    rest Erdos-Renyi with p = avg_degree / (n - 1) and +-1 weights.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    n = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=count))).astype(np.int64)
    dense = rng.random(count) < dense_frac
    reps = rng.choice(np.asarray(replica_choices), size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return [dict(t=float(t[k]), kind="sk_pm1" if dense[k] else "er", n=int(n[k]),
                 replicas=int(reps[k]), seed=int(seeds[k]),
                 p=float(min(1.0, avg_degree / max(1, n[k] - 1))))
            for k in range(count)]


def make_request_instance(desc) -> Instance:
    if desc["kind"] == "sk_pm1":
        return sk_pm1(desc["n"], desc["seed"])
    return erdos_renyi(desc["n"], desc["p"], desc["seed"], "pm1")


# ---- problem descriptions of the Table-3 shapes (Sec. IV-D) -------------------------------
# These are inputs (edge lists, clauses, QUBO matrices); their conversion to Ising form is
# the front-ends' work.

def maxcut_regular_edges(n: int, k: int, seed: int) -> np.ndarray:
    """Edges (m, 2) of a simple k-regular graph (MaxCut-3: k = 3), unit weights implied."""
    rng = np.random.default_rng(seed)
    ei, ej = random_regular_edges(n, k, rng)
    return np.stack([ei, ej], axis=1)


def maxcut_dense_edges(n: int, p: float, seed: int) -> np.ndarray:
    """Edges (m, 2) of G(n, p) (MaxCut-D: p = 0.5)."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    mask = rng.random(iu.shape[0]) < p
    return np.stack([iu[mask], ju[mask]], axis=1)


def nae3sat_clauses(n: int, ratio: float, seed: int, planted: bool = False) -> np.ndarray:
    """Random NAE-3SAT clauses (round(ratio n), 3) over distinct variables, literals +-(v + 1).

    planted: clauses violated by a hidden assignment are redrawn, so it satisfies them all."""
    rng = np.random.default_rng(seed)
    m = int(round(ratio * n))
    hidden = rng.choice([-1, 1], size=n)
    out = np.zeros((m, 3), dtype=np.int64)
    k = 0
    while k < m:
        v = rng.choice(n, size=3, replace=False)
        sg = rng.choice([-1, 1], size=3)
        if planted:
            vals = sg * hidden[v]
            if vals[0] == vals[1] == vals[2]:
                continue
        out[k] = sg * (v + 1)
        k += 1
    return out


def sk_qubo_matrix(n: int, seed: int) -> np.ndarray:
    """SK-QUBO shape: symmetric Q with off-diagonal entries iid in {0, 1}, zero diagonal."""
    rng = np.random.default_rng(seed)
    upper = np.triu(rng.integers(0, 2, size=(n, n)), 1)
    return (upper + upper.T).astype(np.int64)
