"""Pins of the oracle's domain selection (paper Sec. III-B and Sec. IV-B)."""
import numpy as np
import pytest
import torch

import instances as I
import oracle


def test_vertex_identity():
    # at theta in {+-pi/2}^n, L = 1^T s ((J - mu I) s + h) = E(s) - mu n
    inst = I.random_integer_field(I.sk_pm1(30, 1), 1, 4)
    rng = np.random.default_rng(0)
    for mu in (0.0, 0.5, 3.0):
        s = rng.choice([-1, 1], size=(30, 5))
        theta = s * np.pi / 2
        L = oracle.ds_loss(inst, theta, np.where(np.sin(theta) >= 0, 1, -1), mu)
        E = oracle.energies(inst, s)
        assert np.allclose(L, E - mu * 30, rtol=0, atol=1e-9)


def test_gradient_matches_finite_difference():
    inst = I.sk_gauss(25, 3)
    inst.h[:] = np.random.default_rng(1).normal(size=25)
    rng = np.random.default_rng(2)
    theta = rng.uniform(-np.pi, np.pi, size=(25, 3))
    mu = 0.7
    s_fixed = np.where(np.sin(theta) >= 0, 1, -1)
    g = oracle.ds_grad(inst, theta, mu)
    d = 1e-6
    for i in range(25):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += d
        tm[i] -= d
        fd = (oracle.ds_loss(inst, tp, s_fixed, mu) - oracle.ds_loss(inst, tm, s_fixed, mu)) / (2 * d)
        assert np.allclose(fd, g[i], rtol=1e-6, atol=1e-7)


def _torch_reference(inst, U, steps, opt, lr, mu, thetas=None):
    """Autograd + torch.optim on L(theta) with s~ = sign(sin theta) (torch.sign has zero gradient).
    The angles are never wrapped; with ``thetas`` (a list) the angles after each step are kept."""
    J = torch.tensor(inst.dense().astype(np.float64))
    h = torch.tensor(inst.h.astype(np.float64))
    theta = torch.tensor(np.arcsin(U).T.copy(), requires_grad=True)
    optim = (torch.optim.Adam([theta], lr=lr, betas=(0.9, 0.999), eps=1e-8) if opt == "adam"
             else torch.optim.SGD([theta], lr=lr))
    sins = []
    for _ in range(steps):
        optim.zero_grad()
        x = torch.sin(theta)
        s = torch.where(x >= 0, 1.0, -1.0).to(torch.float64).detach()
        loss = (x * (J @ s - mu * s + h[:, None])).sum()
        loss.backward()
        optim.step()
        sins.append(torch.sin(theta).detach().numpy().T.copy())
        if thetas is not None:
            thetas.append(theta.detach().numpy().T.copy())
    return np.array(sins)


@pytest.mark.parametrize("opt,lr", [("adam", 0.05), ("gd", 0.01)])
def test_optimizer_matches_torch(opt, lr):
    inst = I.random_integer_field(I.sk_pm1(20, 4), 4, 2)
    U = I.uniform_draws(11, 6, 20)
    res = oracle.ds_run(inst, U, 25, opt=opt, lr=lr, mu=0.5, record_sin=True)
    ref = _torch_reference(inst, U, 25, opt, lr, 0.5)
    assert np.max(np.abs(res.sin_trace - ref)) < 1e-9


@pytest.mark.parametrize("name,mk,R", [("sk20_field", lambda: I.random_integer_field(I.sk_pm1(20, 4), 4, 2), 6),
                                       ("er60", lambda: I.erdos_renyi(60, 0.1, 1, "pm1"), 8)])
def test_wrap_matches_unwrapped_adam_at_paper_lr(name, mk, R):
    # ADAM at the paper's lr 6.0 (Sec. IV-B) moves an angle by about 6 rad in its first step, so
    # the wrap theta - 2 pi rint(theta / 2 pi) fires on most spins.  torch.optim.Adam on the same
    # loss, never wrapped, gives the same sin(theta) after every step: the wrap only picks
    # another representative of the same angle (a wrong period, e.g. pi, flips signs of sin).
    inst = mk()
    U = I.uniform_draws(19, R, inst.n)
    res = oracle.ds_run(inst, U, 5, opt="adam", lr=6.0, mu=0.5, record_sin=True)
    thetas = []
    ref = _torch_reference(inst, U, 5, "adam", 6.0, 0.5, thetas=thetas)
    thetas = np.array(thetas)
    assert (np.abs(thetas) > np.pi).mean() > 0.5          # the unwrapped angles leave (-pi, pi]
    assert np.all(np.abs(res.theta) <= np.pi)             # the oracle's stay inside it
    assert np.max(np.abs(res.sin_trace - ref)) < 1e-9
    # the wrap is a no-op on sin and cos and moves angles by whole turns only
    th = np.linspace(-40.0, 40.0, 8001)
    w = oracle.wrap_angle(th)
    assert np.all(np.abs(w) <= np.pi)
    assert np.allclose((th - w) / (2 * np.pi), np.rint((th - w) / (2 * np.pi)), atol=1e-12)
    assert np.allclose(np.sin(w), np.sin(th), atol=1e-13) and np.allclose(np.cos(w), np.cos(th), atol=1e-13)


def test_large_mu_freezes_spins():
    inst = I.sk_pm1(40, 2)
    U = I.uniform_draws(3, 8, 40)
    res = oracle.ds_run(inst, U, 200, opt="gd", lr=1e-4, mu=1000.0, record=True, record_sin=True)
    s0 = np.where(U >= 0, 1, -1)
    assert np.all(res.spin_trace == s0[None])


def test_l1_equivalence_large_mu():
    # L1-norm equations: for large enough mu, max_s ||(J - mu I)s + h||_1 = mu n - min_s E(s)
    inst = I.random_integer_field(I.sk_pm1(10, 6), 6, 3)
    mu = float(np.max(np.abs(inst.J).sum(1) + np.abs(inst.h))) + 1.0
    e_min, _, _ = oracle.brute_force_min(inst)
    codes = np.arange(1 << 10)
    S = 1 - 2 * ((codes[:, None] >> np.arange(10)[None]) & 1)
    l1 = np.abs(S @ (inst.J - mu * np.eye(10)) + inst.h).sum(1)
    assert np.isclose(l1.max(), mu * 10 - e_min)


def test_best_tracking_and_energy_trace_consistent():
    inst = I.erdos_renyi(60, 0.1, 1, "pm1")
    U = I.uniform_draws(5, 7, 60)
    res = oracle.ds_run(inst, U, 50, opt="adam", lr=6.0, mu=0.5, record=True, record_sin=True)
    for t in range(50):
        assert np.array_equal(res.energy_trace[t], oracle.energies(inst, res.spin_trace[t].T))
    assert np.array_equal(res.e_best, res.energy_trace.min(0))
    assert np.array_equal(res.best_step, res.energy_trace.argmin(0) + 1)
    assert np.array_equal(res.e_best, oracle.energies(inst, res.s_best.T))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_reaches_brute_force_optimum_n20(seed):
    # quality sanity (guards a flipped gradient sign): 32 replicas x 1000 steps on an
    # N = 20 SK instance reach the exhaustive minimum
    inst = I.sk_pm1(20, seed)
    e_min, _, _ = oracle.brute_force_min(inst)
    U = I.uniform_draws(seed, 32, 20)
    res = oracle.ds_run(inst, U, 1000, opt="adam", lr=6.0, mu=0.5)
    assert res.e_best.min() == e_min
    assert np.all(res.e_best >= e_min)


def _fp32_rounded_start(inst, U, steps, opt, lr):
    """Oracle run whose initial angles are rounded to float32: a perturbation of one float32 rounding."""
    import oracle.ds as D
    th0 = np.arcsin(U).astype(np.float32).astype(np.float64)
    U2 = np.sin(th0)   # asin(U2) == th0 up to one float64 rounding
    return D.ds_run(inst, U2, steps, opt=opt, lr=lr, mu=0.5, record_sin=True)


def test_adam_amplifies_rounding_gd_does_not():
    # property of the method that sets the iterate-parity horizon of any FP32 implementation:
    # one float32 rounding of theta_0 stays below 1e-5 for 100 GD steps (lr 0.01), while
    # ADAM (lr 0.02) carries it above 1e-5 before step 100
    inst = I.sk_pm1(64, 0)
    U = I.uniform_draws(11, 32, 64)
    base_gd = oracle.ds_run(inst, U, 100, opt="gd", lr=0.01, mu=0.5, record_sin=True)
    pert_gd = _fp32_rounded_start(inst, U, 100, "gd", 0.01)
    base_ad = oracle.ds_run(inst, U, 100, opt="adam", lr=0.02, mu=0.5, record_sin=True)
    pert_ad = _fp32_rounded_start(inst, U, 100, "adam", 0.02)

    def err(a, b):
        return (np.abs(a - b).max(axis=2) / np.abs(a).max(axis=2)).max(axis=1)

    e_gd = err(base_gd.sin_trace, pert_gd.sin_trace)
    e_ad = err(base_ad.sin_trace, pert_ad.sin_trace)
    assert e_gd.max() < 1e-5
    assert e_ad[:30].max() < 1e-5
    assert e_ad.max() > 1e-5


# ---- second reading of s~*: the relaxed vertex sin(theta) ------------------------------

def test_relaxed_vertex_identity():
    # at theta in {+-pi/2}^n the relaxed vertex is the vertex: L = s^T (J - mu I) s + h^T s = E(s) - mu n
    inst = I.random_integer_field(I.sk_pm1(30, 5), 5, 4)
    rng = np.random.default_rng(3)
    for mu in (0.0, 0.5, 3.0):
        s = rng.choice([-1, 1], size=(30, 5))
        L = oracle.ds_loss_relaxed(inst, s * np.pi / 2, mu)
        assert np.allclose(L, oracle.energies(inst, s) - mu * 30, rtol=0, atol=1e-9)


def test_relaxed_gradient_matches_finite_difference():
    inst = I.sk_gauss(25, 6)
    inst.h[:] = np.random.default_rng(7).normal(size=25)
    theta = np.random.default_rng(8).uniform(-np.pi, np.pi, size=(25, 3))
    mu = 0.7
    g = oracle.ds_grad_relaxed(inst, theta, mu)
    d = 1e-6
    for i in range(25):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += d
        tm[i] -= d
        fd = (oracle.ds_loss_relaxed(inst, tp, mu) - oracle.ds_loss_relaxed(inst, tm, mu)) / (2 * d)
        assert np.allclose(fd, g[i], rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("opt,lr", [("adam", 0.05), ("gd", 0.01)])
def test_relaxed_optimizer_matches_torch(opt, lr):
    # autograd of the smooth loss x^T (J - mu I) x + h^T x through torch.optim
    inst = I.random_integer_field(I.sk_pm1(20, 9), 9, 2)
    U = I.uniform_draws(9, 4, 20)
    mu = 0.5
    J = torch.tensor(inst.dense().astype(np.float64))
    h = torch.tensor(inst.h.astype(np.float64))
    theta = torch.tensor(np.arcsin(U).T.copy(), requires_grad=True)
    optim = (torch.optim.Adam([theta], lr=lr, betas=(0.9, 0.999), eps=1e-8) if opt == "adam"
             else torch.optim.SGD([theta], lr=lr))
    ref = []
    for _ in range(40):
        optim.zero_grad()
        x = torch.sin(theta)
        loss = (x * (J @ x - mu * x + h[:, None])).sum()
        loss.backward()
        optim.step()
        ref.append(torch.sin(theta).detach().numpy().T.copy())
    res = oracle.ds_run(inst, U, 40, opt=opt, lr=lr, mu=mu, record_sin=True, loss="relaxed")
    assert np.allclose(res.sin_trace, np.array(ref), rtol=0, atol=1e-10)


def test_relaxed_loss_trace_and_energy_consistent():
    # step t records the loss of theta_{t-1} and the energy of its vertex
    inst = I.random_integer_field(I.erdos_renyi(40, 0.2, 10, "pm1"), 10, 3)
    U = I.uniform_draws(10, 6, 40)
    T = 30
    res = oracle.ds_run(inst, U, T, opt="adam", lr=0.5, mu=0.5, record=True, loss="relaxed")
    prev = oracle.ds_run(inst, U, T - 1, opt="adam", lr=0.5, mu=0.5, loss="relaxed")
    for th, t in ((np.arcsin(U).T, 0), (prev.theta.T, T - 1)):
        assert np.allclose(res.loss_trace[t], oracle.ds_loss_relaxed(inst, th, 0.5), rtol=0, atol=1e-9)
        s = np.where(np.sin(th) >= 0, 1, -1)
        assert np.array_equal(res.energy_trace[t], oracle.energies(inst, s))


@pytest.mark.parametrize("seed", [0, 1])
def test_relaxed_reaches_brute_force_optimum_n20(seed):
    inst = I.sk_pm1(20, seed)
    e_min, _, _ = oracle.brute_force_min(inst)
    U = I.uniform_draws(seed + 20, 32, 20)
    res = oracle.ds_run(inst, U, 1000, opt="adam", lr=6.0, mu=0.5, loss="relaxed")
    assert res.e_best.min() == e_min


def test_relaxed_adam_amplifies_faster():
    # the horizon of the relaxed-loss ADAM parity cases: at the paper's lr 6.0 two FP64 runs one ulp
    # apart stay within 1e-7 for 10 steps and pass 1e-6 by step 20 (SK n = 64)
    inst = I.sk_pm1(64, 0)
    U = I.uniform_draws(13, 32, 64)
    a = oracle.ds_run(inst, U, 20, opt="adam", lr=6.0, mu=0.5, record_sin=True, loss="relaxed")
    b = oracle.ds_run(inst, np.nextafter(U, 2), 20, opt="adam", lr=6.0, mu=0.5, record_sin=True, loss="relaxed")

    def sep(t):
        return (np.abs(a.sin_trace[t - 1] - b.sin_trace[t - 1]).max(axis=1)
                / np.abs(a.sin_trace[t - 1]).max(axis=1)).max()
    assert sep(10) < 1e-7
    assert sep(20) > 1e-6


# ---- convergence test (Sec. IV-B): spread of the last 5 losses <= 0.005 |L_now - L_init| ----

def test_convergence_step_closed_forms():
    # constant losses: the spread is 0 as soon as 5 losses exist
    assert oracle.convergence_step([3.0] * 12) == 5
    # L_t = -t: spread 4 <= 0.005 (t - 1) first at t = 801
    assert oracle.convergence_step(-np.arange(1, 1200, dtype=float)) == 801
    # window 3, tol 0.5 on L = -t: spread 2 <= 0.5 (t - 1) first at t = 5
    assert oracle.convergence_step(-np.arange(1, 20, dtype=float), window=3, tol=0.5) == 5
    # switched off, or never met
    assert oracle.convergence_step([1.0] * 10, tol=0.0) == 0
    assert oracle.convergence_step([0.0, 1.0, 0.0, 1.0, 0.0, 1.0]) == 0


def test_converged_replicas_stop_with_their_state():
    inst = I.random_integer_field(I.erdos_renyi(60, 0.1, 14, "pm1"), 14, 2)
    U = I.uniform_draws(14, 16, 60)
    T = 300
    full = oracle.ds_run(inst, U, T, opt="adam", lr=6.0, mu=0.5, record=True, record_sin=True)
    conv = oracle.ds_run(inst, U, T, opt="adam", lr=6.0, mu=0.5, conv_tol=0.005, conv_window=5)
    assert np.all(conv.conv_step > 0)
    for r in range(16):
        t = conv.conv_step[r]
        # the step of convergence is the test applied to the losses of the run without it
        assert t == oracle.convergence_step(full.loss_trace[:, r])
        # state after that step, and the best vertex over steps 1..t
        assert np.array_equal(np.sin(conv.theta[r]), full.sin_trace[t - 1, r])
        assert conv.e_best[r] == full.energy_trace[:t, r].min()
        assert conv.best_step[r] == int(np.argmin(full.energy_trace[:t, r])) + 1


# ---- step sizes of the FP32 parity cases -----------------------------------------------------
#
# The FP32 iterate bar (1e-5 norm-wise over the first 100 steps) can only hold where the method
# itself keeps FP32 rounding below it.  Each case below is one the GPU parity tests run at a
# step size smaller than the standard one (GD 0.01, ADAM 0.02; the relaxed-loss ADAM cases over
# 20 steps): the same formulas evaluated in float32 (oracle.ds_run(dtype=np.float32), a model of
# any FP32 implementation's rounding, not of the kernels) on the same instance, draws and
# compared replicas already depart from the float64 oracle by more than 1e-5 at the standard
# step size, on replicas whose vertices never differ.  The paper's own step sizes are pinned
# the same way: GD lr 0.05 and ADAM lr 6.0 are far outside the FP32 horizon.

def _fp32_departure(inst, U, steps, opt, lr, loss="vertex"):
    base = oracle.ds_run(inst, U, steps, opt=opt, lr=lr, mu=0.5, record_sin=True, loss=loss)
    f32 = oracle.ds_run(inst, U, steps, opt=opt, lr=lr, mu=0.5, record_sin=True, loss=loss, dtype=np.float32)
    same = np.all(base.spin_trace == f32.spin_trace, axis=(0, 2))
    err = (np.abs(base.sin_trace - f32.sin_trace).max(axis=2) / np.abs(base.sin_trace).max(axis=2)).max(axis=0)
    return err[same].max() if same.any() else np.inf


def _compared(U):
    R = U.shape[0]
    return U[np.r_[0:64, R - 64:R]] if R > 128 else U


def _lowered_cases():
    import test_gpu_ds as T
    import test_gpu_dense as TD
    multi = {c[0]: c for c in T.MULTI}
    relaxed = {c[0]: c for c in T.RELAXED}
    rows = {c[0]: c for c in T.ROWS_ORACLE}
    pm = I.sk_pm1(300, 11)
    pm3 = I.Instance(300, "sk_pm3_field_300", np.random.default_rng(12).integers(-4, 5, size=300), pm.J * 3,
                     integer=True)
    return [
        # name, instance maker, replicas, draw seed, optimizer, rejected step size, steps, loss
        ("er_int3_mult_rg4", multi["er_int3_mult_rg4"][1], 1024, 11, "gd", 0.01, 100, "vertex"),
        ("er3000_rg2_ept4", multi["er3000_rg2_ept4"][1], 512, 11, "gd", 0.01, 100, "vertex"),
        ("split_er_int3", multi["er_int3_mult_rg4"][1], 1024, 43, "gd", 0.005, 100, "vertex"),
        ("rows_reg3_1500_field5", rows["reg3_1500_field5_block256_ept8"][1], 256, 43, "gd", 0.01, 100, "vertex"),
        ("torus100x200_field63", lambda: I.random_integer_field(I.torus(100, 200, 26, "pm1"), 26, 63), 4, 11,
         "gd", 0.001, 100, "vertex"),
        ("dense_sk_pm1_300", TD.CASES[0][1], 200, 5, "gd", 0.01, 100, "vertex"),
        ("dense_bf16_pm1_300", lambda: I.sk_pm1(300, 4), 64, 9, "gd", 0.01, 100, "vertex"),
        ("dense_fp8_pm3_field_300", lambda: pm3, 64, 14, "gd", 0.01, 100, "vertex"),
        ("dense_i8x1_int3_field_300", TD.int3_field_300, 64, 75, "gd", 0.01, 100, "vertex"),
        ("relaxed_sk64_dense", relaxed["sk64_dense"][1], 32, 13, "gd", 0.01, 100, "relaxed"),
        ("relaxed_er800_pm1_packed_rg4", relaxed["er800_pm1_packed_rg4"][1], 1024, 13, "gd", 0.01, 100,
         "relaxed"),
        ("relaxed_t1_uniform_real_csr_ept2", relaxed["t1_uniform_real_csr_ept2"][1], 8, 13, "adam", 0.02, 20,
         "relaxed"),
        # the paper's step sizes in FP32: GD 0.05 (SK, ER and the dense N = 2000 workload), ADAM 6.0
        ("paper_gd_sk64", lambda: I.sk_pm1(64, 0), 32, 11, "gd", 0.05, 100, "vertex"),
        ("paper_gd_er800", lambda: I.erdos_renyi(800, 0.06, 1, "pm1"), 64, 11, "gd", 0.05, 100, "vertex"),
        ("paper_gd_sk2000_gauss", lambda: I.sk_gauss(2000, 0), 256, 5, "gd", 0.05, 100, "vertex"),
        ("paper_adam_sk64", lambda: I.sk_pm1(64, 0), 32, 11, "adam", 6.0, 30, "vertex"),
    ]


_LOWERED_IDS = ["er_int3_mult_rg4", "er3000_rg2_ept4", "split_er_int3", "rows_reg3_1500_field5", "torus100x200_field63",
                "dense_sk_pm1_300",
                "dense_bf16_pm1_300", "dense_fp8_pm3_field_300", "dense_i8x1_int3_field_300", "relaxed_sk64_dense",
                "relaxed_er800_pm1_packed_rg4", "relaxed_t1_uniform_real_csr_ept2", "paper_gd_sk64",
                "paper_gd_er800", "paper_gd_sk2000_gauss", "paper_adam_sk64"]


@pytest.mark.parametrize("case", range(len(_LOWERED_IDS)), ids=_LOWERED_IDS)
def test_fp32_rounding_exceeds_the_bar_at_rejected_step_sizes(case):
    name, mk, R, seed, opt, lr, steps, loss = _lowered_cases()[case]
    assert name == _LOWERED_IDS[case]
    inst = mk()
    U = _compared(I.uniform_draws(seed, R, inst.n))
    dep = _fp32_departure(inst, U, steps, opt, lr, loss)
    assert dep > 1e-5, (name, opt, lr, dep)
