"""Pins of the oracle's energy and brute force (paper Sec. II and Sec. III-A)."""
import itertools

import numpy as np
import pytest

import instances as I
import oracle


def _plain_energy(J, h, s):
    n = len(s)
    e = 0
    for i in range(n):
        for j in range(n):
            e += J[i][j] * s[i] * s[j]
        e += h[i] * s[i]
    return e


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_single_flip_identity(seed):
    # Sec. III-A: E(X_i s) - E(s) = -4 s_i sum_j J_ij s_j - 2 h_i s_i
    inst = I.random_integer_field(I.sk_pm1(24, seed), seed, 5)
    rng = np.random.default_rng(seed)
    s = rng.choice([-1, 1], size=inst.n)
    e0 = oracle.energy(inst, s)
    for i in range(inst.n):
        s2 = s.copy()
        s2[i] = -s2[i]
        field = sum(int(inst.J[i, j]) * int(s[j]) for j in range(inst.n))
        assert oracle.energy(inst, s2) - e0 == -4 * s[i] * field - 2 * inst.h[i] * s[i]


def test_single_flip_identity_real_csr():
    inst = I.table1_regular(60, 6, "uniform", 3)
    rng = np.random.default_rng(3)
    s = rng.choice([-1, 1], size=inst.n)
    e0 = oracle.energy(inst, s)
    Jd = inst.dense()
    for i in range(0, inst.n, 7):
        s2 = s.copy()
        s2[i] = -s2[i]
        d = -4 * s[i] * (Jd[i] @ s) - 2 * inst.h[i] * s[i]
        assert abs(oracle.energy(inst, s2) - e0 - d) < 1e-12


def test_two_and_three_spin_closed_forms():
    # E = 2 J s0 s1: antiferromagnetic pair has minimum -2 with 2 minimisers
    pair = I.from_edges(2, [(0, 1, 1)], np.zeros(2))
    e, s, cnt = oracle.brute_force_min(pair)
    assert e == -2 and cnt == 2 and s[0] == -s[1]
    # frustrated triangle, all +1: minimum 2(-1-1+1) = -2, six minimisers
    tri = I.from_edges(3, [(0, 1, 1), (1, 2, 1), (0, 2, 1)], np.zeros(3))
    e, s, cnt = oracle.brute_force_min(tri)
    assert e == -2 and cnt == 6


def test_brute_force_matches_plain_enumeration():
    inst = I.random_integer_field(I.sk_pm1(9, 5), 5, 3)
    J = inst.J.tolist()
    h = inst.h.tolist()
    best = min(_plain_energy(J, h, s) for s in itertools.product([-1, 1], repeat=9))
    e, s, cnt = oracle.brute_force_min(inst)
    assert e == best
    assert _plain_energy(J, h, list(s)) == best


@pytest.mark.parametrize("seed", [0, 1])
def test_planted_ground_state(seed):
    base = I.random_integer_field(I.erdos_renyi(16, 0.3, seed, "pm1"), seed, 2)
    inst, tau = I.planted(base, seed + 10)
    e0 = -np.abs(inst.val).sum() - np.abs(inst.h).sum()
    assert oracle.energy(inst, tau) == e0
    e, s, cnt = oracle.brute_force_min(inst)
    assert e == e0


def test_torus_checkerboard():
    # all-+1 even torus is bipartite: E0 = -4N at the checkerboard
    for lx, ly in [(4, 4), (20, 40)]:
        inst = I.torus(lx, ly, 0, "one")
        yy, xx = np.meshgrid(np.arange(ly), np.arange(lx), indexing="ij")
        s = np.where((xx + yy) % 2 == 0, 1, -1).ravel()
        assert oracle.energy(inst, s) == -4 * inst.n
    e, _, cnt = oracle.brute_force_min(I.torus(4, 4, 0, "one"))
    assert e == -64 and cnt == 2


def test_global_flip_symmetry_and_cut():
    inst = I.erdos_renyi(40, 0.2, 4, "pm1")
    rng = np.random.default_rng(0)
    W = inst.val.sum() // 2
    for _ in range(5):
        s = rng.choice([-1, 1], size=inst.n)
        e = oracle.energy(inst, s)
        assert e == oracle.energy(inst, -s)
        # E = 2 sum_{i<j} J_ij s_i s_j  =>  cut weight = (2W - E) / 4
        assert 4 * oracle.cut_value(inst, s) == 2 * W - e


def test_dense_and_csr_agree():
    inst = I.sk_gauss(30, 2)
    c = inst.as_csr()
    S = np.random.default_rng(1).choice([-1, 1], size=(30, 7))
    assert np.allclose(oracle.energies(inst, S), oracle.energies(c, S), rtol=0, atol=1e-12)
