"""Serving form: continuous batching of many solves on one GPU.

Checks: every served result equals the same request solved alone (bit for bit:
the mix never changes a request's arithmetic); served results equal the plain
per-instance solve; requests arriving while others run are admitted and
overlap; failure handling (rejected input, over-budget request, cancellation,
timeout) is forced from the host.
"""
import time

import numpy as np
import pytest

import instances as I
import oracle

pytestmark = pytest.mark.gpu


def _host(inst):
    import paper_2312_05837_amd as P
    if inst.is_dense:
        return P.host_problem(inst.n, J=inst.J.astype(np.int32),
                              h=inst.h.astype(np.int32) if np.any(inst.h) else None)
    return P.host_problem(inst.n, row_ptr=inst.row_ptr, col=inst.col, val=inst.val.astype(np.int32),
                          h=inst.h.astype(np.int32) if np.any(inst.h) else None)


def _requests(count, seed, steps=200):
    descs = I.serving_stream(count, seed, rate=1000.0, nmin=64, nmax=1200, replica_choices=(64, 128, 256))
    out = []
    for k, d in enumerate(descs):
        inst = I.make_request_instance(d)
        if k % 5 == 0:  # some requests carry an integer field, so pruning has work to do
            inst = I.random_integer_field(inst, d["seed"], 3)
        out.append((inst, d["replicas"], d["seed"]))
    return out


@pytest.fixture()
def ctx():
    import paper_2312_05837_amd as P
    c = P.ising_create(0)
    yield c
    P.ising_destroy(c)


def _serve(ctx, reqs, steps=200, chunk=50, **cfg):
    import paper_2312_05837_amd as P
    P.ising_serve_start(ctx, chunk_steps=chunk, **cfg)
    tickets = []
    keep = []
    for inst, R, seed in reqs:
        st, k = _host(inst)
        keep.append(k)
        tickets.append(P.ising_submit(ctx, st, P.params(replicas=R, steps=steps, optimizer="adam", lr=6.0, mu=0.5,
                                                         seed=seed, precision="fp32")))
    res = [P.ising_wait(ctx, t, inst.n) for t, (inst, _, _) in zip(tickets, reqs)]
    info = P.ising_serve_query(ctx)
    P.ising_serve_stop(ctx)
    return res, info


def test_alone_equals_mix_and_plain_solve(ctx):
    import torch
    import paper_2312_05837_amd as P
    from gpu_util import to_problem
    reqs = _requests(24, 5)
    mix, info = _serve(ctx, reqs, chunk=50, max_resident=16)
    assert info["completed"] == len(reqs) and info["failed"] == 0
    assert info["chunks"] < len(reqs) * 4  # requests shared chunks (4 chunks of 50 steps each if alone)
    for k in (0, 3, 7, 11, 19):
        inst, R, seed = reqs[k]
        alone, _ = _serve(ctx, [reqs[k]], chunk=50)
        assert alone[0][0] == P.ISING_OK and mix[k][0] == P.ISING_OK
        assert np.array_equal(alone[0][1], mix[k][1]), k
        assert alone[0][2] == mix[k][2]
        # the same request through the plain per-instance solve
        s, E, Ei, st = P.ising_solve_dev(ctx, to_problem(inst), P.params(replicas=R, steps=200, optimizer="adam",
                                                                          lr=6.0, mu=0.5, seed=seed,
                                                                          precision="fp32"))
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), mix[k][1]), k
        assert float(E.item()) == mix[k][2]
    for (inst, _, _), (status, spins, energy, stats) in zip(reqs, mix):
        assert status == P.ISING_OK
        assert energy == oracle.energy(inst, spins)
        assert stats["t_total_ms"] >= stats["t_ds_ms"] >= 0


def test_zero_step_requests(ctx):
    # T = 0 (no step to run): each request, dense or sparse, returns what the plain solve returns,
    # the all +1 reduced vertex retrieved through its pruning record, with its exact energy
    import torch
    import paper_2312_05837_amd as P
    from gpu_util import to_problem
    reqs = _requests(8, 13)
    assert any(inst.is_dense and inst.n > 256 for inst, _, _ in reqs) and any(not inst.is_dense for inst, _, _ in reqs)
    res, info = _serve(ctx, reqs, steps=0, chunk=50, max_resident=8)
    assert info["completed"] == len(reqs) and info["failed"] == 0
    for (inst, R, seed), (status, spins, energy, stats) in zip(reqs, res):
        assert status == P.ISING_OK
        pr = oracle.prune(inst)
        assert np.array_equal(spins, oracle.unprune(pr, np.ones(pr.G.size, dtype=np.int64)))
        assert energy == oracle.energy(inst, spins)
        s, E, Ei, st = P.ising_solve_dev(ctx, to_problem(inst), P.params(replicas=R, steps=0, optimizer="adam",
                                                                          lr=6.0, mu=0.5, seed=seed,
                                                                          precision="fp32"))
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), spins)
        assert float(E.item()) == energy


def test_unpruned_requests_equal_plain_solve(ctx):
    # prune = 0 in serving: the request runs on the whole instance and returns what the plain
    # solve with prune = 0 returns, bit for bit (sparse and dense requests, some with fields)
    import torch
    import paper_2312_05837_amd as P
    from gpu_util import to_problem
    reqs = _requests(6, 17)
    P.ising_serve_start(ctx, chunk_steps=50, max_resident=8)
    keep, tickets = [], []
    for inst, R, seed in reqs:
        st, kp = _host(inst)
        keep.append(kp)
        tickets.append(P.ising_submit(ctx, st, P.params(replicas=R, steps=150, seed=seed, prune=False)))
    res = [P.ising_wait(ctx, t, inst.n) for t, (inst, _, _) in zip(tickets, reqs)]
    P.ising_serve_stop(ctx)
    for (inst, R, seed), (status, spins, energy, stats) in zip(reqs, res):
        assert status == P.ISING_OK
        assert stats["n_G"] == inst.n
        s, E, Ei, st = P.ising_solve_dev(ctx, to_problem(inst), P.params(replicas=R, steps=150, seed=seed,
                                                                          prune=False))
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), spins)
        assert float(E.item()) == energy == oracle.energy(inst, spins)


def test_stop_while_a_wait_is_blocked(ctx):
    # a wait blocked on a running request when the server is stopped returns that request's
    # result (stop finishes it first and releases the server only after the wait has returned)
    import threading
    import paper_2312_05837_amd as P
    inst = I.erdos_renyi(300, 0.03, 21, "pm1")
    P.ising_serve_start(ctx, chunk_steps=100)
    st, keep = _host(inst)
    t = P.ising_submit(ctx, st, P.params(replicas=64, steps=1000000, seed=3))
    out = {}
    waiter = threading.Thread(target=lambda: out.setdefault("r", P.ising_wait(ctx, t, inst.n)))
    waiter.start()
    time.sleep(0.3)  # the wait is inside the library, blocked on the running request
    assert waiter.is_alive()
    assert P.ising_serve_stop(ctx) is None
    waiter.join(timeout=120)
    assert not waiter.is_alive()
    status, spins, energy, stats = out["r"]
    assert status == P.ISING_OK and energy == oracle.energy(inst, spins) and stats["steps"] == 1000000


def test_submit_while_stopping_refused(ctx):
    # once stop has begun (it is finishing a long request), a new submission is refused with
    # EBUSY instead of being queued behind a scheduler that is about to exit
    import threading
    import paper_2312_05837_amd as P
    inst = I.erdos_renyi(300, 0.03, 23, "pm1")
    P.ising_serve_start(ctx, chunk_steps=100)
    st, keep = _host(inst)
    P.ising_submit(ctx, st, P.params(replicas=64, steps=1000000, seed=5))
    stopper = threading.Thread(target=lambda: P.ising_serve_stop(ctx))
    stopper.start()
    time.sleep(0.3)
    assert stopper.is_alive()
    with pytest.raises(P.IsingError) as e:
        P.ising_submit(ctx, st, P.params(replicas=64, steps=10, seed=6))
    assert e.value.status == P.ISING_EBUSY
    stopper.join(timeout=120)
    assert not stopper.is_alive()


def test_two_waits_on_one_ticket(ctx):
    # one of them returns the result and consumes the ticket; the other returns EINVAL
    import threading
    import paper_2312_05837_amd as P
    inst = I.erdos_renyi(300, 0.03, 22, "pm1")
    P.ising_serve_start(ctx, chunk_steps=100)
    st, keep = _host(inst)
    t = P.ising_submit(ctx, st, P.params(replicas=64, steps=300000, seed=4))
    outs = []
    threads = [threading.Thread(target=lambda: outs.append(P.ising_wait(ctx, t, inst.n))) for _ in range(2)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    P.ising_serve_stop(ctx)
    statuses = sorted(o[0] for o in outs)
    assert statuses == [P.ISING_OK, P.ISING_EINVAL]
    status, spins, energy, _ = next(o for o in outs if o[0] == P.ISING_OK)
    assert energy == oracle.energy(inst, spins)


def test_submit_and_wait_from_several_threads(ctx):
    # submission and waiting are thread-safe: four threads each submit and collect their own
    # requests; every result equals the same request served alone from one thread
    import threading
    import paper_2312_05837_amd as P
    reqs = _requests(12, 19)
    P.ising_serve_start(ctx, chunk_steps=50, max_resident=8)
    results = [None] * len(reqs)
    keep = []
    lock = threading.Lock()

    def worker(ids):
        for k in ids:
            inst, R, seed = reqs[k]
            st, kp = _host(inst)
            with lock:
                keep.append(kp)
            t = P.ising_submit(ctx, st, P.params(replicas=R, steps=200, optimizer="adam", lr=6.0, mu=0.5,
                                                 seed=seed, precision="fp32"))
            results[k] = P.ising_wait(ctx, t, inst.n)

    threads = [threading.Thread(target=worker, args=(list(range(w, len(reqs), 4)),)) for w in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=300)
    P.ising_serve_stop(ctx)
    alone, _ = _serve(ctx, reqs, chunk=50, max_resident=8)
    for k, (inst, _, _) in enumerate(reqs):
        assert results[k][0] == P.ISING_OK, k
        assert np.array_equal(results[k][1], alone[k][1]) and results[k][2] == alone[k][2], k
        assert results[k][2] == oracle.energy(inst, results[k][1])


def test_requests_arriving_while_others_run_are_admitted(ctx):
    import paper_2312_05837_amd as P
    reqs = _requests(12, 7)
    P.ising_serve_start(ctx, chunk_steps=20, max_resident=8)
    keep, tickets = [], []
    for k, (inst, R, seed) in enumerate(reqs):
        st, kp = _host(inst)
        keep.append(kp)
        tickets.append(P.ising_submit(ctx, st, P.params(replicas=R, steps=400, seed=seed)))
        if k == 5:
            time.sleep(0.05)  # the first requests are already running when the rest arrive
    res = [P.ising_wait(ctx, t, inst.n) for t, (inst, _, _) in zip(tickets, reqs)]
    info = P.ising_serve_query(ctx)
    P.ising_serve_stop(ctx)
    assert all(r[0] == P.ISING_OK for r in res)
    assert info["admitted"] == len(reqs) and info["completed"] == len(reqs)
    # 12 requests x 20 chunks each would be 240 chunks one at a time
    assert info["chunks"] < 120


def test_failing_dense_group_leaves_the_others_running(ctx, monkeypatch):
    # A dense group whose launch fails marks only its own requests.  The failure is forced from
    # the host: with ISING_SERVE_TEST_FAIL_DENSE_STEPS=50 (read when the server starts) a dense
    # group advancing 50 steps in a chunk reports a launch failure instead of launching.  A
    # long sparse request keeps the server busy so that the two dense requests, submitted back
    # to back, are admitted at the same chunk boundary: request A (50 steps) forms the failing
    # group, request B (100 steps) its own group in the same chunk.
    import time as _t
    import paper_2312_05837_amd as P
    monkeypatch.setenv("ISING_SERVE_TEST_FAIL_DENSE_STEPS", "50")
    P.ising_serve_start(ctx, chunk_steps=100)
    monkeypatch.delenv("ISING_SERVE_TEST_FAIL_DENSE_STEPS")
    c = I.erdos_renyi(2000, 4.0 / 1999, 7, "pm1")
    a, b = I.sk_pm1(300, 8), I.sk_pm1(320, 9)
    stc, kc = _host(c)
    sta, ka = _host(a)
    stb, kb = _host(b)
    prm_b = P.params(replicas=128, steps=100, optimizer="adam", lr=6.0, mu=0.5, seed=3, precision="fp32")
    tc = P.ising_submit(ctx, stc, P.params(replicas=256, steps=3000, seed=1))
    _t.sleep(0.02)
    ta = P.ising_submit(ctx, sta, P.params(replicas=128, steps=50, optimizer="adam", lr=6.0, mu=0.5, seed=2))
    tb = P.ising_submit(ctx, stb, prm_b)
    ra, rb, rc = P.ising_wait(ctx, ta, a.n), P.ising_wait(ctx, tb, b.n), P.ising_wait(ctx, tc, c.n)
    info = P.ising_serve_query(ctx)
    P.ising_serve_stop(ctx)
    assert ra[0] == P.ISING_EDEVICE
    assert rb[0] == P.ISING_OK and rc[0] == P.ISING_OK
    assert info["failed"] == 1 and info["completed"] == 2
    # the surviving dense request's result is the plain solve's
    spins, energy, _, _ = P.ising_solve(ctx, stb, prm_b)
    assert np.array_equal(rb[1], spins) and rb[2] == energy == oracle.energy(b, spins)


def test_failures_forced_from_the_host(ctx):
    import paper_2312_05837_amd as P
    P.ising_serve_start(ctx, hbm_budget_bytes=4 << 20, max_resident=4, chunk_steps=10)
    # asymmetric J: rejected at admission
    J = np.array([[0, 1], [2, 0]], dtype=np.int32)
    st, keep1 = P.host_problem(2, J=J)
    t_bad = P.ising_submit(ctx, st, P.params(replicas=8, steps=10))
    assert P.ising_wait(ctx, t_bad, 2)[0] == P.ISING_EINVAL
    # a convergence window the kernels do not hold: rejected at admission
    tor = I.torus(8, 8, 3, "pm1")
    st0, keep0 = _host(tor)
    t_win = P.ising_submit(ctx, st0, P.params(replicas=8, steps=10, conv_tol=0.005, conv_window=9))
    assert P.ising_wait(ctx, t_win, tor.n)[0] == P.ISING_EINVAL
    # larger than the whole budget: refused with ENOMEM
    big = I.sk_pm1(1200, 1)
    st2, keep2 = _host(big)
    t_big = P.ising_submit(ctx, st2, P.params(replicas=1024, steps=10))
    assert P.ising_wait(ctx, t_big, big.n)[0] == P.ISING_ENOMEM
    # timeout on a long request, then cancellation
    inst = I.erdos_renyi(300, 0.03, 2, "pm1")
    st3, keep3 = _host(inst)
    t_long = P.ising_submit(ctx, st3, P.params(replicas=64, steps=200000))
    assert P.ising_wait(ctx, t_long, inst.n, timeout_ms=0)[0] == P.ISING_ETIMEDOUT
    P.ising_cancel(ctx, t_long)
    assert P.ising_wait(ctx, t_long, inst.n)[0] == P.ISING_ECANCELED
    # the server still works afterwards
    small = I.erdos_renyi(100, 0.05, 3, "pm1")
    st4, keep4 = _host(small)
    t_ok = P.ising_submit(ctx, st4, P.params(replicas=32, steps=50))
    status, spins, energy, _ = P.ising_wait(ctx, t_ok, small.n)
    assert status == P.ISING_OK and energy == oracle.energy(small, spins)
    info = P.ising_serve_query(ctx)
    P.ising_serve_stop(ctx)
    assert info["failed"] == 3 and info["canceled"] == 1 and info["completed"] == 1


def test_large_sparse_and_grouped_dense_requests(ctx):
    """Sparse requests that need the widest register form (several spins per lane,
    two words of vertex bits per lane) and dense requests of different lengths,
    which the server advances as one matrix-core group per step count."""
    import torch
    import paper_2312_05837_amd as P
    from gpu_util import to_problem
    reqs = [(I.erdos_renyi(3000, 8.0 / 2999, 11, "pm1"), 512, 101, 120),
            (I.erdos_renyi(2600, 8.0 / 2599, 12, "pm1"), 512, 102, 60),
            (I.sk_pm1(300, 13), 128, 103, 120),
            (I.sk_pm1(520, 14), 256, 104, 70),
            (I.sk_pm1(300, 15), 64, 105, 70)]
    P.ising_serve_start(ctx, chunk_steps=50, max_resident=8)
    keep, tickets = [], []
    for inst, R, seed, steps in reqs:
        st, kp = _host(inst)
        keep.append(kp)
        tickets.append(P.ising_submit(ctx, st, P.params(replicas=R, steps=steps, optimizer="adam", lr=6.0, mu=0.5,
                                                         seed=seed, precision="fp32")))
    res = [P.ising_wait(ctx, t, r[0].n) for t, r in zip(tickets, reqs)]
    info = P.ising_serve_query(ctx)
    P.ising_serve_stop(ctx)
    assert info["completed"] == len(reqs) and info["failed"] == 0, [r[0] for r in res]
    for (inst, R, seed, steps), (status, spins, energy, _) in zip(reqs, res):
        assert status == P.ISING_OK
        s, E, Ei, st = P.ising_solve_dev(ctx, to_problem(inst), P.params(replicas=R, steps=steps, optimizer="adam",
                                                                          lr=6.0, mu=0.5, seed=seed,
                                                                          precision="fp32"))
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), spins), inst.n
        assert float(E.item()) == energy
        assert energy == oracle.energy(inst, spins)


def test_dense_graph_replays_equal_eager_launches(ctx):
    """Dense groups replay a captured launch sequence while their shape and step count stay
    the same (here four replays per group, with eager descriptor uploads and the sparse
    requests' launches in between); every result equals the one-by-one launches bit for bit."""
    import paper_2312_05837_amd as P
    pm = I.sk_pm1(400, 21)
    reqs = [(I.sk_pm1(300, 22), 128, 201), (pm, 256, 202),
            (I.Instance(400, "sk_pm3", np.zeros(400, dtype=np.int64), pm.J * 3, integer=True), 64, 203),
            (I.erdos_renyi(600, 8.0 / 599, 23, "pm1"), 128, 204)]
    graphs, _ = _serve(ctx, reqs, steps=100, chunk=20, max_resident=8)
    eager, _ = _serve(ctx, reqs, steps=100, chunk=20, max_resident=8, graphs=False)
    for (inst, _, _), g, e in zip(reqs, graphs, eager):
        assert g[0] == P.ISING_OK and e[0] == P.ISING_OK
        assert np.array_equal(g[1], e[1]) and g[2] == e[2], inst.name
        assert g[3]["best_step"] == e[3]["best_step"] and g[3]["best_replica"] == e[3]["best_replica"]
        assert g[2] == oracle.energy(inst, g[1])


def test_convergence_test_in_serving(ctx):
    """Requests with the convergence test: each result (vector, energy, replicas stopped, mean
    steps run) equals the plain solve's, and a request whose replicas have all stopped is
    finished at the end of that chunk instead of running its full step count."""
    import torch
    import paper_2312_05837_amd as P
    from gpu_util import to_problem
    reqs = [(I.table1_regular(400, 6, "binary_int", 31), 64, 301), (I.table1_regular(600, 6, "binary_int", 32), 128, 302),
            (I.random_integer_field(I.erdos_renyi(500, 8.0 / 499, 33, "pm1"), 33, 3), 64, 303)]
    T = 1000
    P.ising_serve_start(ctx, chunk_steps=50, max_resident=8)
    keep, tickets = [], []
    for inst, R, seed in reqs:
        st, kp = _host(inst)
        keep.append(kp)
        tickets.append(P.ising_submit(ctx, st, P.params(replicas=R, steps=T, optimizer="adam", lr=6.0, mu=0.5,
                                                         seed=seed, precision="fp32", conv_tol=0.005)))
    res = [P.ising_wait(ctx, tk, r[0].n) for tk, r in zip(tickets, reqs)]
    info = P.ising_serve_query(ctx)
    P.ising_serve_stop(ctx)
    assert info["completed"] == len(reqs) and info["failed"] == 0
    full = [st["converged"] == R for (_, R, _), (_, _, _, st) in zip(reqs, res)]
    assert any(full)
    if all(full):
        assert info["chunks"] < T // 50  # finished before the full step count
    for (inst, R, seed), (status, spins, energy, stats) in zip(reqs, res):
        assert status == P.ISING_OK
        s, E, Ei, st = P.ising_solve_dev(ctx, to_problem(inst), P.params(replicas=R, steps=T, optimizer="adam",
                                                                          lr=6.0, mu=0.5, seed=seed,
                                                                          precision="fp32", conv_tol=0.005))
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), spins), inst.name
        assert float(E.item()) == energy == oracle.energy(inst, spins)
        assert stats["converged"] == st["converged"] and stats["mean_steps_run"] == st["mean_steps_run"]


def test_reduced_precision_dense_forms_in_serving(ctx):
    # Gaussian dense requests in the BF16X2, I8X3 and I8X2 forms (float64 couplings; pruning keeps
    # them whole) and an FP32 request on integer dense couplings of several magnitudes (one INT8
    # digit) served together with integer sparse requests: each served result equals the same
    # request served alone and the plain solve bit for bit, and its energy is the exact (integer)
    # or FP64 energy of its vector.
    import torch
    import paper_2312_05837_amd as P
    from gpu_util import to_problem
    import test_gpu_dense as TD
    dense = [(I.sk_gauss(300, 61), 128, 1, "bf16x2"), (I.sk_gauss(257, 62), 64, 2, "i8x3"),
             (I.sk_gauss(500, 63), 256, 3, "i8x2"), (I.sk_gauss(300, 64), 128, 4, "i8x3"),
             (TD.int3_field_300(), 96, 5, "fp32")]  # integer magnitudes 1..3: one INT8 digit
    sparse = [(inst, R, seed, "fp32") for inst, R, seed in _requests(4, 9)]
    reqs = dense + sparse

    def serve(batch):
        P.ising_serve_start(ctx, chunk_steps=50)
        keep, tickets = [], []
        for inst, R, seed, prec in batch:
            if inst.is_dense and not inst.integer:
                st, k = P.host_problem(inst.n, J=inst.J.astype(np.float64))
            else:
                st, k = _host(inst)
            keep.append(k)
            tickets.append(P.ising_submit(ctx, st, P.params(replicas=R, steps=200, optimizer="adam", lr=6.0,
                                                             mu=0.5, seed=seed, precision=prec)))
        res = [P.ising_wait(ctx, t, inst.n) for t, (inst, _, _, _) in zip(tickets, batch)]
        P.ising_serve_stop(ctx)
        return res

    mix = serve(reqs)
    for k, (inst, R, seed, prec) in enumerate(reqs):
        status, spins, energy, _ = mix[k]
        assert status == P.ISING_OK, (k, prec)
        if inst.integer:
            assert energy == oracle.energy(inst, spins)
        else:
            assert abs(energy - oracle.energy(inst, spins)) <= 1e-9 * np.abs(inst.J).sum()
    for k in range(len(dense)):
        inst, R, seed, prec = reqs[k]
        alone = serve([reqs[k]])[0]
        assert np.array_equal(alone[1], mix[k][1]) and alone[2] == mix[k][2], (k, prec)
        s, E, Ei, st = P.ising_solve_dev(ctx, to_problem(inst), P.params(replicas=R, steps=200, optimizer="adam",
                                                                          lr=6.0, mu=0.5, seed=seed,
                                                                          precision=prec))
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), mix[k][1]), (k, prec)
        assert float(E.item()) == mix[k][2], (k, prec)
