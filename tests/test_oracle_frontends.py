"""Pins of the oracle's problem front-ends: exhaustive agreement with the problems' own definitions."""
import itertools

import numpy as np
import pytest

import instances as I
import oracle


def _all_spins(n):
    return np.array(list(itertools.product([-1, 1], repeat=n)), dtype=np.int64)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_qubo_value_is_energy_plus_offset_for_every_x(seed):
    rng = np.random.default_rng(seed)
    n = 9
    Q = rng.integers(-3, 4, size=(n, n)).astype(np.float64)   # not symmetric, nonzero diagonal
    c = rng.integers(-2, 3, size=n).astype(np.float64)
    inst, off = oracle.qubo_instance(Q, c)
    S = _all_spins(n)
    E = oracle.energies(inst, S.T)
    f = np.array([oracle.qubo_value(Q, c, (1 + s) // 2) for s in S])
    assert np.allclose(E + off, f, rtol=0, atol=1e-9)


def test_maxcut_energy_counts_the_cut_for_every_s():
    n = 10
    edges = I.maxcut_regular_edges(n, 3, 4)
    w = np.arange(1, len(edges) + 1)                           # distinct integer weights
    inst, W = oracle.maxcut_instance(n, edges, w)
    S = _all_spins(n)
    E = oracle.energies(inst, S.T)
    cuts = np.array([oracle.cut_of(n, edges, w, s) for s in S])
    assert np.array_equal(E, 2 * W - 4 * cuts)
    # unit weights on a 3-regular graph: E = 2 (m - 2 cut), the table's convention
    inst1, W1 = oracle.maxcut_instance(n, edges)
    assert W1 == len(edges) == 15


def test_nae3sat_energy_counts_violated_clauses_for_every_s():
    n = 8
    cl = I.nae3sat_clauses(n, 2.11, 5)
    cl = np.vstack([cl, [[1, -1, 3], [2, 2, -2]]])             # clauses that repeat a variable
    inst, base = oracle.nae3sat_instance(n, cl)
    S = _all_spins(n)
    E = oracle.energies(inst, S.T)
    U = np.array([oracle.nae_violated(cl, s) for s in S])
    assert np.array_equal(E + base, 8 * U)


def test_planted_nae3sat_is_satisfiable():
    n = 14
    cl = I.nae3sat_clauses(n, 2.11, 6, planted=True)
    inst, base = oracle.nae3sat_instance(n, cl)
    e_min, _, _ = oracle.brute_force_min(inst)
    assert (e_min + base) // 8 == 0


# ---- the library's front-ends (host code of the C ABI) against the oracle's -------------------

def test_library_qubo_matches_oracle():
    import paper_2312_05837_amd as P
    rng = np.random.default_rng(11)
    Q = rng.normal(size=(30, 30))
    c = rng.normal(size=30)
    J, h, off = P.ising_from_qubo(Q, c)
    Jo, ho, offo = oracle.qubo_to_ising(Q, c)
    assert np.allclose(J, Jo, rtol=1e-15, atol=0) and np.allclose(h, ho, rtol=1e-14, atol=1e-14)
    assert abs(off - offo) <= 1e-12 * (1 + abs(offo))


def test_library_maxcut_and_nae3sat_match_oracle():
    import paper_2312_05837_amd as P
    n = 200
    edges = I.maxcut_regular_edges(n, 3, 7)
    edges = np.vstack([edges, edges[:5]])                      # duplicates are summed
    rp, col, val, W = P.ising_from_maxcut(n, edges)
    inst, Wo = oracle.maxcut_instance(n, edges)
    assert W == Wo
    assert np.array_equal(rp, inst.row_ptr) and np.array_equal(col, inst.col) and np.array_equal(val, inst.val)
    cl = I.nae3sat_clauses(n, 2.11, 8)
    cl = np.vstack([cl, [[3, -3, 5]]])
    rp, col, val, base = P.ising_from_nae3sat(n, cl)
    inst, baseo = oracle.nae3sat_instance(n, cl)
    assert base == baseo
    assert np.array_equal(rp, inst.row_ptr) and np.array_equal(col, inst.col) and np.array_equal(val, inst.val)


def test_library_frontends_reject_bad_input():
    import paper_2312_05837_amd as P
    with pytest.raises(P.IsingError):
        P.ising_from_maxcut(4, [[0, 0]])                       # self-loop
    with pytest.raises(P.IsingError):
        P.ising_from_nae3sat(4, [[1, 2, 5]])                   # variable out of range
    with pytest.raises(P.IsingError):
        P.ising_from_qubo(np.array([[np.inf]]))
