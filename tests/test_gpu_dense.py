"""GPU parity of the matrix-core (MFMA) domain-selection engine for dense couplings.

FP32 form: same bar as the persistent engine (norm-wise relative iterate error
<= 1e-5; GD over 100 steps, ADAM over its 30-step horizon).  +-1 couplings are
exact in BF16, so the BF16 and BF16X2 forms must reproduce the FP32 form bit
for bit on them.  Couplings of one integer magnitude w run the FP8 form (J / w and
the vertex exact in FP8, every product and sum an exact integer): it must equal
the BF16 form bit for bit where both are exact, and FP32 requests on such
couplings run it.  On Gaussian couplings the BF16 forms carry the representation
error of J: J_hi + J_lo has relative error <= 2^-16 per entry and J_hi alone
2^-8; their tolerances below are those bounds times the observed growth of the
GD map (x10 over 100 steps), and the measured errors are printed.
"""
import numpy as np
import pytest

import instances as I
import oracle
from gpu_util import to_problem, iterate_error, compare_trajectories, int8_represented

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2312_05837_amd as P
    c = P.ising_create(0)
    yield c
    P.ising_destroy(c)


def _run(ctx, inst, R, steps, opt, lr, prec, chunks, U):
    import torch
    import paper_2312_05837_amd as P
    prob = to_problem(inst)
    state = P.ds_state(inst.n, R, "fp32")
    prm = P.params(replicas=R, steps=steps, optimizer=opt, precision=prec, lr=lr, mu=0.5)
    per = steps // chunks
    thetas, et = [], []
    for c in range(chunks):
        st2 = dict(state)
        st2["energy_trace"] = torch.zeros((per, R), dtype=torch.float64, device="cuda")
        P.ising_ds_dense_dev(ctx, prob, prm, st2, t0=c * per, steps=per,
                             uniform=torch.tensor(U, dtype=torch.float32, device="cuda") if c == 0 else None)
        torch.cuda.synchronize()
        thetas.append(state["theta"].cpu().numpy().astype(np.float64))
        et.append(st2["energy_trace"].cpu().numpy())
    out = {k: v.cpu().numpy() for k, v in state.items()}
    out["thetas"] = thetas
    out["energy_trace"] = np.concatenate(et)
    return out


def _worst(inst, got, U, steps, opt, lr, chunks):
    ref = oracle.ds_run(inst, U, steps, opt=opt, lr=lr, mu=0.5, record=True, record_sin=True)
    per = steps // chunks
    worst = 0.0
    for c, th in enumerate(got["thetas"]):
        t = (c + 1) * per
        worst = max(worst, iterate_error(np.sin(th), ref.sin_trace[t - 1]).max())
    return worst, ref


CASES = [  # name, maker, replicas, (GD lr, ADAM lr): the standard 0.01 / 0.02 unless the formulas
    # evaluated in float32 depart from the float64 oracle by more than 1e-5 at the standard step
    # (sk_pm1_300 GD: 4.2e-5; test_oracle_ds.py::test_fp32_rounding_exceeds_the_bar_at_rejected_step_sizes)
    ("sk_pm1_300", lambda: I.sk_pm1(300, 1), 200, (0.002, 0.02)),
    ("gauss_300", lambda: I.sk_gauss(300, 2), 200, (0.01, 0.02)),
    ("gauss_field_130", lambda: I.Instance(130, "g130", np.random.default_rng(3).normal(size=130),
                                           I.sk_gauss(130, 3).J, integer=False), 70, (0.01, 0.02)),
    # tile edges: one spin past the first 128-spin tile with a single replica, and whole tiles
    # with no padding in either dimension
    ("gauss_129_R1", lambda: I.sk_gauss(129, 4), 1, (0.01, 0.02)),
    ("gauss_256_R256", lambda: I.sk_gauss(256, 6), 256, (0.01, 0.02))]


@pytest.mark.parametrize("opt,steps", [("gd", 100), ("adam", 30)])
@pytest.mark.parametrize("name,mk,R,lrs", CASES, ids=[c[0] for c in CASES])
def test_fp32_form_iterates(ctx, name, mk, R, lrs, opt, steps):
    inst = mk()
    U = I.uniform_draws(5, R, inst.n)
    lr = lrs[0] if opt == "gd" else lrs[1]
    chunks = 10 if steps == 100 else 3
    got = _run(ctx, inst, R, steps, opt, lr, "fp32", chunks, U)
    got["loss_trace"] = np.zeros_like(got["energy_trace"])
    worst, excl = compare_trajectories(inst, got, U, steps, opt, lr, chunks, check_loss=False)
    print(f"{name} {opt}: FP32 MFMA worst iterate error {worst:.2e}, excluded {excl}/{R}")


def test_bf16_forms_exact_on_pm1(ctx):
    # +-1/2 couplings: not integers, so FP32 requests keep the FP32 matrix-core form
    # (integer +-1 ones are routed to the BF16 form, which is exact for them)
    pm = I.sk_pm1(300, 4)
    inst = I.Instance(300, "sk_half_300", np.zeros(300), pm.J * 0.5, integer=False)
    U = I.uniform_draws(6, 130, inst.n)
    a = _run(ctx, inst, 130, 60, "adam", 6.0, "fp32", 1, U)
    for prec in ("bf16x2", "bf16"):
        b = _run(ctx, inst, 130, 60, "adam", 6.0, prec, 1, U)
        for k in ("theta", "m", "v", "s_best", "e_best", "best_step", "energy_trace"):
            assert np.array_equal(a[k], b[k]), (prec, k)
    # the integer +-1 instance in FP32 (routed to BF16) matches the oracle like the FP32 form, at GD
    # lr 0.002: at the standard 0.01 the formulas evaluated in float32 depart from the float64
    # oracle by 3.1e-5 on these draws (test_oracle_ds.py::test_fp32_rounding_exceeds_the_bar_at_rejected_step_sizes)
    U2 = I.uniform_draws(9, 64, pm.n)
    got = _run(ctx, pm, 64, 100, "gd", 0.002, "fp32", 10, U2)
    got["loss_trace"] = np.zeros_like(got["energy_trace"])
    compare_trajectories(pm, got, U2, 100, "gd", 0.002, 10, check_loss=False)


@pytest.mark.parametrize("n,R", [(129, 1), (256, 512), (384, 257)])
def test_bf16_forms_exact_on_pm1_at_tile_edges(ctx, n, R):
    # the same bitwise identity of the FP32, BF16X2 and BF16 forms on +-1/2 couplings at tile
    # edges: one spin past the first 128-spin tile with one replica, whole tiles with no padding
    # (BF16X2 on 128 x 256 tiles, the others on 128 x 128), and one replica past a whole tile
    pm = I.sk_pm1(n, 40 + n)
    inst = I.Instance(n, f"sk_half_{n}", np.zeros(n), pm.J * 0.5, integer=False)
    U = I.uniform_draws(41, R, n)
    a = _run(ctx, inst, R, 40, "adam", 6.0, "fp32", 1, U)
    for prec in ("bf16x2", "bf16"):
        b = _run(ctx, inst, R, 40, "adam", 6.0, prec, 1, U)
        for k in ("theta", "m", "v", "s_best", "e_best", "best_step", "energy_trace"):
            assert np.array_equal(a[k], b[k]), (prec, k)


@pytest.mark.parametrize("prec,tol,steps", [("bf16x2", 2e-4, 100), ("bf16", 5e-2, 20)])
def test_bf16_forms_gaussian_error_bound(ctx, prec, tol, steps):
    # a vertex may legitimately differ where the oracle's |sin theta| is below the form's
    # error; such replicas are excluded from later steps (at most a quarter of them).  With
    # J rounded to one BF16 (2^-8 relative) trajectories part after a few tens of steps, so
    # that form is compared over 20 steps; its long runs are judged by FP64 energies.
    inst = I.sk_gauss(300, 7)
    U = I.uniform_draws(8, 64, inst.n)
    chunks = steps // 10
    got = _run(ctx, inst, 64, steps, "gd", 0.01, prec, chunks, U)
    got["loss_trace"] = np.zeros_like(got["energy_trace"])
    worst, excl = compare_trajectories(inst, got, U, steps, "gd", 0.01, chunks, TOL=tol, check_loss=False,
                                       max_excluded=16, check_energy=(prec == "bf16x2"))
    print(f"{prec}: worst iterate error vs FP64 oracle {worst:.2e}, replicas excluded {excl}/64")


def test_solve_dense_engine_energy_recomputed_fp64(ctx):
    import torch
    import paper_2312_05837_amd as P
    inst = I.sk_gauss(400, 9)
    for prec in ("fp32", "bf16x2", "bf16", "i8x3", "i8x2"):
        s, E, Ei, st = P.ising_solve_dev(ctx, to_problem(inst), P.params(replicas=256, steps=200, precision=prec,
                                                                           optimizer="adam", lr=6.0, mu=0.5))
        torch.cuda.synchronize()
        s = s.cpu().numpy()
        assert abs(E.item() - oracle.energy(inst, s)) < 1e-9 * (np.abs(inst.J).sum())
        assert E.item() / 400 < -1.2  # SK ground states lie near E/N = -1.53 in this convention; random vertices near 0


def test_fp8_form_exact_on_uniform_integer_couplings(ctx):
    # J = +-3 (one integer magnitude) with integer fields, n = 300 (K padding and a ragged
    # spin tile), R = 130 (a ragged replica tile): FP8, BF16 and FP32 requests all give the
    # same iterates, energies and best vertices bit for bit (the FP32 request runs FP8)
    pm = I.sk_pm1(300, 11)
    h = np.random.default_rng(12).integers(-4, 5, size=300)
    inst = I.Instance(300, "sk_pm3_field_300", h, pm.J * 3, integer=True)
    U = I.uniform_draws(13, 130, inst.n)
    a = _run(ctx, inst, 130, 60, "adam", 6.0, "fp8", 2, U)
    for prec in ("bf16", "fp32"):
        b = _run(ctx, inst, 130, 60, "adam", 6.0, prec, 2, U)
        for k in ("theta", "m", "v", "s_best", "e_best", "best_step", "energy_trace"):
            assert np.array_equal(a[k], b[k]), (prec, k)
    # and it follows the FP64 oracle like the FP32 form (GD, 100 steps, lr 0.001: at the standard
    # 0.01 the formulas evaluated in float32 depart from the float64 oracle by 3.6e-2 on these
    # draws, test_oracle_ds.py::test_fp32_rounding_exceeds_the_bar_at_rejected_step_sizes)
    U2 = I.uniform_draws(14, 64, inst.n)
    got = _run(ctx, inst, 64, 100, "gd", 0.001, "fp8", 10, U2)
    got["loss_trace"] = np.zeros_like(got["energy_trace"])
    worst, excl = compare_trajectories(inst, got, U2, 100, "gd", 0.001, 10, check_loss=False)
    print(f"FP8 form: worst iterate error vs FP64 oracle {worst:.2e}, excluded {excl}/64")


@pytest.mark.parametrize("n,R", [(129, 1), (256, 256), (384, 257)])
def test_integer_forms_agree_at_tile_edges(ctx, n, R):
    # J = +-3 with integer fields at tile edges: the FP8 form (one magnitude), three INT8 digits
    # and BF16 give the same iterates, energies and best vertices bit for bit (each product and
    # sum is an exact integer in every form), and so does an FP32 request, which runs FP8
    pm = I.sk_pm1(n, 60 + n)
    h = np.random.default_rng(61).integers(-4, 5, size=n)
    inst = I.Instance(n, f"sk_pm3_field_{n}", h, pm.J * 3, integer=True)
    U = I.uniform_draws(62, R, n)
    a = _run(ctx, inst, R, 40, "adam", 6.0, "fp8", 2, U)
    for prec in ("i8x3", "bf16", "fp32"):
        b = _run(ctx, inst, R, 40, "adam", 6.0, prec, 2, U)
        for k in ("theta", "m", "v", "s_best", "e_best", "best_step", "energy_trace"):
            assert np.array_equal(a[k], b[k]), (prec, k)


def test_fp8_form_rejected_for_other_couplings(ctx):
    import torch
    import paper_2312_05837_amd as P
    inst = I.sk_gauss(300, 15)
    state = P.ds_state(inst.n, 64, "fp32")
    prm = P.params(replicas=64, steps=5, optimizer="adam", precision="fp8", lr=6.0, mu=0.5)
    with pytest.raises(P.IsingError) as e:
        P.ising_ds_dense_dev(ctx, to_problem(inst), prm, state, t0=0, steps=5)
    assert e.value.status == P.ISING_ENOTSUP
    # mixed integer magnitudes (+-1 and +-2) are not one magnitude either
    pm = I.sk_pm1(300, 16)
    mixed = I.Instance(300, "mixed", np.zeros(300), pm.J * np.where(np.arange(300)[:, None] % 2 == 0, 1, 2)
                       * np.where(np.arange(300)[None, :] % 2 == 0, 1, 2), integer=True)
    mixed.J = np.where(mixed.J != 0, mixed.J, 0)
    assert np.array_equal(mixed.J, mixed.J.T)
    with pytest.raises(P.IsingError):
        P.ising_ds_dense_dev(ctx, to_problem(mixed), prm, state, t0=0, steps=5)
    torch.cuda.synchronize()


def test_solve_fp8_form_integer_energy(ctx):
    import torch
    import paper_2312_05837_amd as P
    inst = I.sk_pm1(512, 17)
    res = {}
    for prec in ("fp8", "fp32", "bf16"):
        s, E, Ei, st = P.ising_solve_dev(ctx, to_problem(inst), P.params(replicas=256, steps=200, precision=prec,
                                                                           optimizer="adam", lr=6.0, mu=0.5))
        torch.cuda.synchronize()
        s = s.cpu().numpy()
        assert Ei.item() == oracle.energy(inst, s)
        res[prec] = (s.copy(), Ei.item())
    assert np.array_equal(res["fp8"][0], res["fp32"][0]) and np.array_equal(res["fp8"][0], res["bf16"][0])


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x2", 2e-4), ("i8x3", 1e-5), ("i8x2", 1e-5)])
def test_full_size_sk2000(ctx, prec, tol):
    # the precision-form workload at its own size: dense SK N = 2000, J ~ N(0, 1/N), R = 256
    # replicas (the oracle on the first and last 64), GD lr 0.01 over 100 steps in 10 calls.
    # FP32: the FP32 matrix-core form at the FP32 bar.  BF16X2: J as hi + lo BF16 parts
    # (relative error <= 2^-16 per entry) at the BF16X2 bar.  I8X3 and I8X2: the oracle on the
    # couplings they represent (2^e Jq) at the FP32 bar.
    import paper_2312_05837_amd as P
    inst = I.sk_gauss(2000, 0)
    ref_inst = int8_represented(inst, {"i8x3": 3, "i8x2": 2}[prec])[0] if prec.startswith("i8") else inst
    R = 256
    U = I.uniform_draws(5, R, inst.n)
    got = _run(ctx, inst, R, 100, "gd", 0.01, prec, 10, U)
    assert P.ising_last_kernel(ctx) == f"k_dense_step<{prec}>", P.ising_last_kernel(ctx)
    got["loss_trace"] = np.zeros_like(got["energy_trace"])
    worst, excl = compare_trajectories(ref_inst, got, U, 100, "gd", 0.01, 10, TOL=tol, check_loss=False,
                                       max_excluded=8)
    print(f"sk2000 {prec}: worst iterate error vs FP64 oracle {worst:.2e}, excluded {excl}/128")


# ---- INT8 forms: J = 2^e Jq, Jq of three (two) balanced INT8 digits, exact int32 products ------

def test_int8_forms_exact_on_integer_couplings(ctx):
    # J = +-3 with integer fields (n = 300: K padding and a ragged spin tile; R = 130: a ragged
    # replica tile): J / 2^e is an integer, so the products are exact and I8X3 and I8X2 requests
    # give the FP8 form's iterates, energies and best vertices bit for bit
    import paper_2312_05837_amd as P
    pm = I.sk_pm1(300, 11)
    h = np.random.default_rng(12).integers(-4, 5, size=300)
    inst = I.Instance(300, "sk_pm3_field_300", h, pm.J * 3, integer=True)
    U = I.uniform_draws(13, 130, inst.n)
    a = _run(ctx, inst, 130, 60, "adam", 6.0, "fp8", 2, U)
    for prec in ("i8x3", "i8x2"):
        b = _run(ctx, inst, 130, 60, "adam", 6.0, prec, 2, U)
        assert P.ising_last_kernel(ctx) == f"k_dense_step<{prec}>", P.ising_last_kernel(ctx)
        for k in ("theta", "m", "v", "s_best", "e_best", "best_step", "energy_trace"):
            assert np.array_equal(a[k], b[k]), (prec, k)


@pytest.mark.parametrize("n,R", [(300, 96), (129, 1), (256, 512)])
@pytest.mark.parametrize("prec,digits", [("i8x3", 3), ("i8x2", 2)])
@pytest.mark.parametrize("opt,lr,steps", [("gd", 0.01, 100), ("adam", 0.02, 30)])
def test_int8_forms_gaussian_iterates(ctx, prec, digits, opt, lr, steps, n, R):
    # Gaussian couplings with a field: the FP64 oracle run on the couplings the form represents
    # (2^e Jq) at the FP32 bar; its product is exact in int32 and y is rounded once, so only the
    # FP32 iterate arithmetic differs.  For two digits 2^e is about 2^-16 of max|J|, so a wrong
    # exponent or digit would show at this bar; three digits are compared the same way.  Shapes:
    # n = 300 with R = 96 (K padding, ragged tiles in both dimensions), one spin past the first
    # 128-spin tile with a single replica, and whole 128 x 256 tiles with no padding.
    base = I.sk_gauss(n, 21)
    inst = I.Instance(n, f"g{n}h", np.random.default_rng(22).normal(size=n), base.J, integer=False)
    rep, e = int8_represented(inst, digits)
    U = I.uniform_draws(23, R, inst.n)
    chunks = 10 if steps == 100 else 3
    got = _run(ctx, inst, R, steps, opt, lr, prec, chunks, U)
    got["loss_trace"] = np.zeros_like(got["energy_trace"])
    worst, excl = compare_trajectories(rep, got, U, steps, opt, lr, chunks, check_loss=False)
    rel = np.abs(rep.J - inst.J).max() / np.abs(inst.J).max()
    print(f"{prec} {opt} n={n} R={R}: e = {e}, max |J - 2^e Jq| / max|J| = {rel:.1e}, "
          f"worst iterate error vs FP64 oracle on 2^e Jq {worst:.2e}, excluded {excl}/{R}")


def test_int8_forms_rejected_for_sparse(ctx):
    import paper_2312_05837_amd as P
    inst = I.torus(10, 10, 1, "pm1")
    for prec in ("i8x3", "i8x2"):
        with pytest.raises(P.IsingError) as e:
            P.ising_solve_dev(ctx, to_problem(inst), P.params(replicas=64, steps=10, precision=prec))
        assert e.value.status == P.ISING_ENOTSUP


def int3_field_300():
    """SK sign pattern with integer magnitudes 1..3 and an integer field up to 5, n = 300."""
    pm = I.sk_pm1(300, 71)
    mag = np.random.default_rng(72).integers(1, 4, size=(300, 300))
    mag = np.triu(mag, 1) + np.triu(mag, 1).T
    h = np.random.default_rng(73).integers(-5, 6, size=300)
    return I.Instance(300, "sk_int3_field_300", h, pm.J * mag, integer=True)


def test_fp32_requests_on_integer_couplings_run_one_int8_digit(ctx):
    # integer couplings of several magnitudes (|J| in 1..3) with an integer field, n = 300 (K
    # padding, a ragged spin tile), R = 130 (a ragged replica tile): an FP32 request runs the
    # INT8 form with one digit (every product and sum an exact integer), and equals the BF16 and
    # I8X3 requests, which are exact on these couplings too, bit for bit
    import paper_2312_05837_amd as P
    inst = int3_field_300()
    U = I.uniform_draws(74, 130, inst.n)
    a = _run(ctx, inst, 130, 60, "adam", 6.0, "fp32", 2, U)
    assert P.ising_last_kernel(ctx) == "k_dense_step<i8x1>", P.ising_last_kernel(ctx)
    for prec in ("bf16", "i8x3"):
        b = _run(ctx, inst, 130, 60, "adam", 6.0, prec, 2, U)
        for k in ("theta", "m", "v", "s_best", "e_best", "best_step", "energy_trace"):
            assert np.array_equal(a[k], b[k]), (prec, k)
    # and it follows the FP64 oracle like the FP32 form (GD, 100 steps, lr 0.002: at the standard
    # 0.01 the formulas evaluated in float32 depart from the float64 oracle by 4.9e-3 on these
    # draws, test_oracle_ds.py::test_fp32_rounding_exceeds_the_bar_at_rejected_step_sizes)
    U2 = I.uniform_draws(75, 64, inst.n)
    got = _run(ctx, inst, 64, 100, "gd", 0.002, "fp32", 10, U2)
    got["loss_trace"] = np.zeros_like(got["energy_trace"])
    worst, excl = compare_trajectories(inst, got, U2, 100, "gd", 0.002, 10, check_loss=False)
    print(f"one INT8 digit: worst iterate error vs FP64 oracle {worst:.2e}, excluded {excl}/64")



@pytest.mark.parametrize("prec,digits,shift", [("i8x3", 3, 102), ("i8x2", 2, 110)])
def test_int8_forms_at_the_exponent_floor(ctx, prec, digits, shift):
    # Gaussian couplings scaled by 2^-shift (n = 300): the smallest fitting exponent lies below
    # -126, so the scale is held at 2^-126 (a normal float) and the couplings are represented
    # more coarsely; the FP64 oracle on the couplings the form represents (built by the documented
    # rule, which holds the exponent at -126 too) at the FP32 bar, GD over 30 steps
    base = I.sk_gauss(300, 81)
    inst = I.Instance(300, "g300_tiny", np.zeros(300), np.ldexp(base.J, -shift), integer=False)
    rep, e = int8_represented(inst, digits)
    assert e == -126
    U = I.uniform_draws(82, 64, inst.n)
    got = _run(ctx, inst, 64, 30, "gd", 0.01, prec, 3, U)
    got["loss_trace"] = np.zeros_like(got["energy_trace"])
    worst, excl = compare_trajectories(rep, got, U, 30, "gd", 0.01, 3, check_loss=False)
    print(f"{prec} at 2^-{shift}: e = {e}, worst iterate error vs FP64 oracle on 2^e Jq {worst:.2e}, excluded {excl}/64")
