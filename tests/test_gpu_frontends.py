"""Problem front-ends end to end on the GPU: MaxCut and NAE-3SAT (Sec. IV-D) built by the
library's front-ends, solved by ising_solve, read back in the problem's own terms."""
import numpy as np
import pytest

import instances as I
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2312_05837_amd as P
    c = P.ising_create(0)
    yield c
    P.ising_destroy(c)


def test_maxcut_reaches_brute_force_cut(ctx):
    import paper_2312_05837_amd as P
    n = 18
    edges = I.maxcut_regular_edges(n, 3, 2)
    rp, col, val, W = P.ising_from_maxcut(n, edges)
    st, keep = P.host_problem(n, row_ptr=rp, col=col, val=val.astype(np.int32))
    spins, E, Ei, stats = P.ising_solve(ctx, st, P.params(replicas=64, steps=500, seed=3))
    inst, _ = oracle.maxcut_instance(n, edges)
    e_min, _, _ = oracle.brute_force_min(inst)
    assert E == oracle.energy(inst, spins)
    assert oracle.cut_of(n, edges, None, spins) == (2 * W - E) / 4 == (2 * W - e_min) / 4


def test_planted_nae3sat_satisfied(ctx):
    import paper_2312_05837_amd as P
    n = 60
    cl = I.nae3sat_clauses(n, 2.11, 21, planted=True)
    rp, col, val, base = P.ising_from_nae3sat(n, cl)
    st, keep = P.host_problem(n, row_ptr=rp, col=col, val=val)
    spins, E, Ei, stats = P.ising_solve(ctx, st, P.params(replicas=256, steps=1000, seed=5))
    assert oracle.nae_violated(cl, spins) == (E + base) // 8 == 0


def test_qubo_through_the_solver(ctx):
    import paper_2312_05837_amd as P
    n = 16
    Q = I.sk_qubo_matrix(n, 9) - 0.6 * np.eye(n) * n    # a QUBO whose minimum is not x = 0
    J, h, off = P.ising_from_qubo(Q)
    st, keep = P.host_problem(n, J=J, h=h)
    spins, E, Ei, stats = P.ising_solve(ctx, st, P.params(replicas=64, steps=500, precision="fp64", seed=7))
    x = (1 + spins.astype(np.int64)) // 2
    inst, off_o = oracle.qubo_instance(Q)
    e_min, _, _ = oracle.brute_force_min(inst)
    assert abs(oracle.qubo_value(Q, None, x) - (E + off)) < 1e-9 * (1 + abs(E))
    assert abs(E - e_min) < 1e-9 * (1 + abs(e_min))
