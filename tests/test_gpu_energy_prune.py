"""GPU parity of the exact energy, pruning (Algorithm 1) and retrieval against the oracle."""
import numpy as np
import pytest

import instances as I
import oracle
from gpu_util import to_problem, as_float32_instance, energy_bound
from test_oracle_prune import _star_real

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2312_05837_amd as P
    c = P.ising_create(0)
    yield c
    P.ising_destroy(c)


ENERGY_CASES = [
    ("sk_pm1_64", lambda: I.sk_pm1(64, 0)),
    ("sk_pm1_h_300", lambda: I.random_integer_field(I.sk_pm1(300, 1), 1, 7)),
    ("er_800", lambda: I.erdos_renyi(800, 0.06, 2, "pm1")),
    ("torus_20x40", lambda: I.torus(20, 40, 3, "pm1")),
    ("reg3_2000", lambda: I.random_regular(2000, 3, 4, "pm1")),
    ("t1_uniform_1000", lambda: I.table1_regular(1000, 6, "uniform", 5)),
    ("gauss_dense_257", lambda: I.sk_gauss(257, 6)),
    ("empty_graph_h", lambda: I.from_edges(5, [], np.array([1, -2, 0, 3, 4]))),
]


@pytest.mark.parametrize("name,mk", ENERGY_CASES, ids=[c[0] for c in ENERGY_CASES])
def test_energy_matches_oracle(ctx, name, mk):
    import torch
    import paper_2312_05837_amd as P
    inst = mk()
    prob = to_problem(inst)
    rng = np.random.default_rng(0)
    S = rng.choice(np.array([-1, 1], dtype=np.int8), size=(17, inst.n))
    E, Ei = P.ising_energy_dev(ctx, prob, torch.tensor(S, device="cuda"))
    torch.cuda.synchronize()
    ref = oracle.energies(inst, S.T)
    if inst.integer:
        assert np.array_equal(Ei.cpu().numpy(), ref.astype(np.int64))
        assert np.array_equal(E.cpu().numpy(), ref.astype(np.float64))
    else:
        assert np.all(np.abs(E.cpu().numpy() - ref) <= 2 * energy_bound(inst))


def test_energy_float32_values(ctx):
    import torch
    import paper_2312_05837_amd as P
    inst = I.sk_gauss(190, 9)
    f32 = as_float32_instance(inst)
    prob = to_problem(inst, real_dtype=torch.float32)
    S = np.random.default_rng(1).choice(np.array([-1, 1], dtype=np.int8), size=(5, inst.n))
    E, _ = P.ising_energy_dev(ctx, prob, torch.tensor(S, device="cuda"))
    torch.cuda.synchronize()
    assert np.all(np.abs(E.cpu().numpy() - oracle.energies(f32, S.T)) <= 2 * energy_bound(f32))


PRUNE_CASES = [
    ("forest_csr", lambda: I.random_forest_plus_cycles(500, 0, n_extra=30, hmax=3)),
    ("forest_dense", lambda: I.random_forest_plus_cycles(130, 1, n_extra=8, hmax=2).as_dense()),
    ("forest_h0", lambda: I.random_forest_plus_cycles(700, 2, n_extra=10, hmax=0)),
    ("er_field", lambda: I.random_integer_field(I.erdos_renyi(400, 0.01, 3, "pm1"), 3, 4)),
    ("t1_uniform", lambda: I.table1_regular(1000, 6, "uniform", 4)),
    ("t1_gaussian", lambda: I.table1_regular(1000, 6, "gaussian", 5)),
    ("t1_uniform_dense", lambda: I.table1_regular(200, 6, "uniform", 6).as_dense()),
    ("t1_binary_int", lambda: I.table1_regular(600, 6, "binary_int", 7)),
    ("t1_binary_real", lambda: I.table1_regular(600, 6, "binary", 8)),
    ("torus_nothing", lambda: I.torus(20, 40, 9, "pm1")),
    ("star", lambda: I.from_edges(4, [(0, 1, 1), (0, 2, 1), (0, 3, 1)], np.zeros(4))),
    ("edge_field", lambda: I.from_edges(2, [(0, 1, 1)], np.array([3, 0]))),
    ("path4", lambda: I.from_edges(4, [(0, 1, 1), (1, 2, 1), (2, 3, 1)], np.zeros(4))),
    ("all_determined", lambda: I.from_edges(3, [(0, 1, 1)], np.array([5, -5, 2]))),
    ("long_path", lambda: I.from_edges(301, [(i, i + 1, 1 if i % 3 else -1) for i in range(300)], np.zeros(301))),
    # real folds whose value depends on the summation order (see the oracle's pins)
    ("star_real_D", lambda: _star_real(70, 0.4, 2.0 ** -56, -1.0, -1.0, 0.0)),
    ("star_real_S", lambda: _star_real(70, 0.5, 0.5, 0.8, 2.0 ** -55, 0.0)),
]


def _prune_gpu(ctx, inst):
    import torch
    import paper_2312_05837_amd as P
    prob = to_problem(inst)
    pr = P.ising_prune_dev(ctx, prob)
    info = P.ising_pruned_info(pr)
    rec = P.ising_pruned_record_dev(ctx, pr)
    red = P.ising_pruned_copy_dev(ctx, pr) if info["n_G"] > 0 else None
    torch.cuda.synchronize()
    return prob, pr, info, {k: v.cpu().numpy() for k, v in rec.items()}, red


@pytest.mark.parametrize("name,mk", PRUNE_CASES, ids=[c[0] for c in PRUNE_CASES])
def test_prune_bit_exact(ctx, name, mk):
    inst = mk()
    ref = oracle.prune(inst)
    prob, pr, info, rec, red = _prune_gpu(ctx, inst)
    assert info["n_G"] == ref.G.size
    assert info["rounds"] == ref.rounds
    assert np.array_equal(rec["kind"], ref.kind)
    assert np.array_equal(rec["round_of"], ref.round_of)
    assert np.array_equal(rec["fixed"], np.where(ref.kind == 1, ref.fixed, 0))
    assert np.array_equal(rec["partner"], ref.partner)
    assert np.array_equal(rec["sigma"], ref.sigma)
    assert np.array_equal(rec["G"], ref.G)
    if inst.integer:
        assert info["C"] == ref.C
        if ref.G.size:
            assert np.array_equal(rec["h_G"].astype(np.int64), ref.h_G.astype(np.int64))
    else:
        # The decisions above compare fields with row sums formed in one fixed order on both
        # sides; the folds into h and C are plain ascending sums in the oracle and the device's
        # own reduction order in the kernels, so h_G and C agree to the summation bound
        # gamma_k * (sum of the magnitudes of their terms), k = n + nnz terms at most.
        u = 2.0 ** -53
        k = inst.n + (inst.n * inst.n if inst.is_dense else inst.nnz)
        gamma = k * u / (1 - k * u)
        assert abs(info["C"] - ref.C) <= gamma * ref.C_mass, (info["C"], ref.C, ref.C_mass)
        if ref.G.size:
            err = np.abs(rec["h_G"] - ref.h_G)
            assert np.all(err <= gamma * ref.h_mass), (err.max(), (gamma * ref.h_mass).min())
    if ref.G.size and red is not None and ref.G.size < inst.n:
        if inst.is_dense:
            assert np.array_equal(red.J.cpu().numpy(), ref.reduced.J)
        else:
            assert np.array_equal(red.row_ptr.cpu().numpy(), ref.reduced.row_ptr)
            assert np.array_equal(red.col.cpu().numpy(), ref.reduced.col)
            assert np.array_equal(red.val.cpu().numpy(), ref.reduced.val)


@pytest.mark.parametrize("name,mk", PRUNE_CASES[:6] + PRUNE_CASES[10:], ids=[c[0] for c in PRUNE_CASES[:6] + PRUNE_CASES[10:]])
def test_unprune_bit_exact(ctx, name, mk):
    import torch
    import paper_2312_05837_amd as P
    inst = mk()
    ref = oracle.prune(inst)
    prob, pr, info, rec, red = _prune_gpu(ctx, inst)
    rng = np.random.default_rng(5)
    for _ in range(3):
        sG = rng.choice(np.array([-1, 1], dtype=np.int8), size=max(ref.G.size, 1))[:ref.G.size]
        s = P.ising_unprune_dev(ctx, pr, torch.tensor(sG, device="cuda") if sG.size else
                                torch.zeros(1, dtype=torch.int8, device="cuda"))
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), oracle.unprune(ref, sG))


def test_invalid_problems_rejected(ctx):
    import torch
    import paper_2312_05837_amd as P
    J = torch.tensor([[0, 1], [2, 0]], dtype=torch.int32, device="cuda")
    with pytest.raises(P.IsingError) as e:
        P.ising_prune_dev(ctx, P.dense_problem(J))
    assert e.value.status == P.ISING_EINVAL
    J = torch.tensor([[1, 1], [1, 0]], dtype=torch.int32, device="cuda")
    with pytest.raises(P.IsingError):
        P.ising_prune_dev(ctx, P.dense_problem(J))
    # unsorted CSR columns
    rp = torch.tensor([0, 2, 3, 4], dtype=torch.int32, device="cuda")
    col = torch.tensor([2, 1, 0, 0], dtype=torch.int32, device="cuda")
    val = torch.ones(4, dtype=torch.int32, device="cuda")
    with pytest.raises(P.IsingError):
        P.ising_prune_dev(ctx, P.csr_problem(rp, col, val))
    J = torch.tensor([[0.0, float("nan")], [float("nan"), 0.0]], dtype=torch.float64, device="cuda")
    with pytest.raises(P.IsingError):
        P.ising_prune_dev(ctx, P.dense_problem(J))
