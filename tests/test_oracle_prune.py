"""Pins of the oracle's pruning and retrieval (paper Sec. III-A, Algorithm 1, Fig. 1c)."""
import networkx as nx
import numpy as np
import pytest

import instances as I
import oracle


def _check_exact_for_all_sG(inst, pr, trials=20, seed=0):
    # E_full(unprune(s_G)) = E_G(s_G) + C for EVERY s_G (algebra of the reduced problem)
    rng = np.random.default_rng(seed)
    for _ in range(trials):
        sG = rng.choice([-1, 1], size=pr.G.size)
        s = oracle.unprune(pr, sG)
        lhs = oracle.energy(inst, s)
        rhs = (oracle.energy(pr.reduced, sG) if pr.G.size else 0) + pr.C
        if inst.integer:
            assert lhs == rhs
        else:
            scale = np.abs(inst.val).sum() + np.abs(inst.h).sum()
            assert abs(lhs - rhs) <= 1e-12 * scale


@pytest.mark.parametrize("seed", range(4))
def test_exact_for_every_reduced_state_integer(seed):
    inst = I.random_forest_plus_cycles(300, seed, n_extra=20, hmax=3)
    pr = oracle.prune(inst)
    assert 0 < pr.G.size < inst.n
    _check_exact_for_all_sG(inst, pr, seed=seed)


@pytest.mark.parametrize("dist", ["uniform", "gaussian"])
def test_exact_for_every_reduced_state_real(dist):
    inst = I.table1_regular(400, 6, dist, 7)
    pr = oracle.prune(inst)
    assert pr.eta > 0.2
    _check_exact_for_all_sG(inst, pr)


def test_dense_input_same_decisions():
    inst = I.random_forest_plus_cycles(120, 3, n_extra=10, hmax=2)
    a = oracle.prune(inst)
    b = oracle.prune(inst.as_dense())
    assert np.array_equal(a.G, b.G) and a.C == b.C
    assert np.array_equal(a.kind, b.kind) and np.array_equal(a.partner, b.partner)


@pytest.mark.parametrize("seed", range(5))
def test_optimum_preserved_brute_force(seed):
    kinds = [
        lambda: I.random_forest_plus_cycles(18, seed, n_extra=3, hmax=3),
        lambda: I.random_integer_field(I.erdos_renyi(16, 0.15, seed, "pm1"), seed, 4),
        lambda: I.table1_regular(16, 3, "uniform", seed),
    ]
    for mk in kinds:
        inst = mk()
        pr = oracle.prune(inst)
        e_full, _, _ = oracle.brute_force_min(inst)
        if pr.G.size:
            e_red, s_red, _ = oracle.brute_force_min(pr.reduced)
        else:
            e_red, s_red = 0, np.zeros(0, dtype=np.int8)
        if inst.integer:
            assert e_red + pr.C == e_full
            assert oracle.energy(inst, oracle.unprune(pr, s_red)) == e_full
        else:
            assert abs(e_red + pr.C - e_full) < 1e-9


@pytest.mark.parametrize("seed", range(3))
def test_zero_field_is_two_core_plus_tree_centres(seed):
    inst = I.random_forest_plus_cycles(400, seed, n_extra=6, hmax=0)
    pr = oracle.prune(inst)
    g = nx.Graph()
    g.add_nodes_from(range(inst.n))
    rp, col, val = inst.csr()
    for i in range(inst.n):
        for p in range(rp[i], rp[i + 1]):
            if i < col[p]:
                g.add_edge(i, int(col[p]), w=int(val[p]))
    core = set(nx.k_core(g, 2).nodes())
    expect = set(core)
    for comp in nx.connected_components(g):
        if comp & core:
            continue
        expect.add(min(nx.center(g.subgraph(comp))))
    assert set(pr.G.tolist()) == expect
    # every edge outside G x G was peeled at cost -2|J_e|
    Gs = set(pr.G.tolist())
    peeled = sum(abs(d["w"]) for u, v, d in g.edges(data=True) if not (u in Gs and v in Gs))
    assert pr.C == -2 * peeled
    assert np.all(pr.kind[pr.kind != 0] == 2)


def test_first_round_rate_closed_form():
    # Sec. IV-A bound-expectation equations: for J-hat ~ U(-1,1) on a 6-regular graph and
    # h-hat ~ U(-6,6), eta_1 = Pr(|h-hat| > sum_6 |J-hat|) = 1 - E[sum]/6 = 1/2 exactly.
    etas = []
    for seed in range(8):
        pr = oracle.prune(I.table1_regular(1000, 6, "uniform", seed))
        etas.append(pr.per_round[0][0] / 1000)
    assert abs(np.mean(etas) - 0.5) < 0.02


def test_binary_tie_prunes_nothing():
    # Table 1 binary row: 2 sum|J| = |h| exactly, the strict rule never fires, degree 6 => eta = 0
    for seed in range(3):
        pr = oracle.prune(I.table1_regular(200, 6, "binary_int", seed))
        assert pr.eta == 0.0 and pr.rounds == 1 and pr.C == 0


def test_hand_made_cases():
    # star, centre 0: leaves are semi-determined with partner 0
    star = I.from_edges(4, [(0, 1, 1), (0, 2, 1), (0, 3, 1)], np.zeros(4))
    pr = oracle.prune(star)
    assert pr.G.tolist() == [0] and pr.C == -6
    assert pr.partner[1:].tolist() == [0, 0, 0] and pr.sigma[1:].tolist() == [1, 1, 1]
    # isolated antiferro... ferromagnetic edge J = -1: mutual pair, larger index goes
    edge = I.from_edges(2, [(0, 1, -1)], np.zeros(2))
    pr = oracle.prune(edge)
    assert pr.G.tolist() == [0] and pr.kind[1] == 2 and pr.partner[1] == 0 and pr.sigma[1] == -1
    assert pr.C == -2
    s = oracle.unprune(pr, [1])
    assert s.tolist() == [1, 1]
    # edge with a strong field on spin 0: 0 determined, then 1 determined next round
    fe = I.from_edges(2, [(0, 1, 1)], np.array([3, 0]))
    pr = oracle.prune(fe)
    assert pr.G.size == 0 and pr.kind.tolist() == [1, 1] and pr.round_of.tolist() == [0, 1]
    assert pr.fixed.tolist() == [-1, 1] and pr.C == -5
    e, _, _ = oracle.brute_force_min(fe)
    assert e == -5
    # path of 4: leaves peeled, then the middle pair is mutual and the lower centre survives
    path = I.from_edges(4, [(0, 1, 1), (1, 2, 1), (2, 3, 1)], np.zeros(4))
    pr = oracle.prune(path)
    assert pr.G.tolist() == [1] and pr.round_of.tolist() == [0, -1, 1, 0]


def test_fixed_order_sum_is_the_stated_order():
    # one row of 150 entries: lanes take p = l, l+64, l+128; then xor 32..1 butterfly
    rng = np.random.default_rng(0)
    vals = rng.normal(size=150) * 10.0 ** rng.integers(-8, 8, size=150)
    rows = np.zeros(150, dtype=np.int64)
    cols = np.arange(150)
    active = np.ones(150, dtype=bool)
    got = oracle.fixed_order_abs_rowsum(150, rows, cols, vals, cols.copy(), active, False)[0]
    lanes = [0.0] * 64
    for p in range(150):
        lanes[p % 64] = lanes[p % 64] + abs(vals[p])
    for d in (32, 16, 8, 4, 2, 1):
        lanes = [lanes[i] + lanes[i ^ d] for i in range(64)]
    assert got == lanes[0]
    assert abs(got - np.abs(vals).sum()) <= 1e-13 * np.abs(vals).sum()


def _star_real(k, j_first, j_rest, h_first, h_rest, h_leaf):
    """Star with centre 0 and leaves 1..k (real couplings): leaf 1 has coupling j_first and
    field h_first, the others j_rest and h_rest; the centre's field is h_leaf.  The centre
    also sits on a triangle with spins k+1, k+2 (unit couplings, no field), which keeps it in
    G after its leaves are gone (two active neighbours, 2 sum|J| = 4 > |h_0|)."""
    edges = [(0, 1, j_first)] + [(0, i, j_rest) for i in range(2, k + 1)]
    edges += [(0, k + 1, 1.0), (0, k + 2, 1.0), (k + 1, k + 2, 1.0)]
    h = np.r_[h_leaf, h_first, np.full(k - 1, h_rest), 0.0, 0.0]
    return I.from_edges(k + 3, edges, h, "star_real", integer=False)


def test_determined_fold_is_a_plain_ascending_sum():
    # 70 determined leaves (|h| = 1 > 2|J|) fold into the free centre: the terms 2 J_0i s_i are
    # 0.8 (leaf 1) and then 69 terms of 2^-55, each below half an ulp of 0.8.  Added one after
    # another in ascending index they leave 0.8 unchanged; any grouping that sums the small
    # terms first (pairwise, 64 strided partials) moves the result by about 2^-49.
    inst = _star_real(70, 0.4, 2.0 ** -56, -1.0, -1.0, 0.0)
    pr = oracle.prune(inst)
    assert pr.G.tolist() == [0, 71, 72] and np.all(pr.kind[1:71] == 1) and pr.rounds == 2
    assert pr.h_G.tolist() == [0.8, 0.0, 0.0]
    assert 0.8 + 69 * 2.0 ** -55 != 0.8   # the small terms matter once grouped
    assert pr.C == -70.0                   # sum of h_i s_i = -|h_i|; no D-D couplings
    assert abs(pr.h_mass[0] - 0.8) < 1e-14 and pr.C_mass == 70.0   # magnitudes for error bounds


def test_semi_determined_fold_is_a_plain_ascending_sum():
    # 70 semi-determined leaves (one neighbour, 2|J| = 1 >= |h|): h_0 -= sum sgn(J_0k) h_k with
    # h_1 = 0.8 first and 69 fields of 2^-55 after it, one after another: exactly -0.8
    inst = _star_real(70, 0.5, 0.5, 0.8, 2.0 ** -55, 0.0)
    pr = oracle.prune(inst)
    assert pr.G.tolist() == [0, 71, 72] and np.all(pr.kind[1:71] == 2) and np.all(pr.partner[1:71] == 0)
    assert pr.h_G[0] == -0.8
    assert pr.C == -70.0                   # -2|J| per semi-determined leaf
    # exactness for every reduced state (Sec. III-A reduced problem) still holds
    for sG in ([1, 1, 1], [-1, 1, -1], [1, -1, -1]):
        s = oracle.unprune(pr, sG)
        assert oracle.energy(inst, s) == oracle.energy(pr.reduced, np.array(sG)) + pr.C
