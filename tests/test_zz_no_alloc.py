"""The energy entry point that allocates nothing against the one that allocates.

ising_energy_dev_noalloc keeps its partial sums in the library's static device
scratch instead of a buffer allocated on demand; its results must equal
ising_energy_dev's bit for bit (same kernels, same summation order), on two
calls in a row, the second with a smaller input, and requests beyond the
scratch are rejected before any work is enqueued.
"""
import numpy as np
import pytest

import instances as I
import oracle
from gpu_util import to_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,mk,counts", [
    ("er800_int", lambda: I.random_integer_field(I.erdos_renyi(800, 0.06, 2, "pm1"), 2, 5), (300, 17)),
    ("gauss_dense_257", lambda: I.sk_gauss(257, 6), (64, 3)),
])
def test_noalloc_energy_equals_allocating_call(name, mk, counts):
    import torch
    import paper_2312_05837_amd as P
    ctx = P.ising_create(0)
    try:
        inst = mk()
        prob = to_problem(inst)
        rng = np.random.default_rng(11)
        for count in counts:
            S = torch.tensor(rng.choice(np.array([-1, 1], dtype=np.int8), size=(count, inst.n)), device="cuda")
            E_ref, Ei_ref = P.ising_energy_dev(ctx, prob, S)
            E = torch.full((count,), np.nan, dtype=torch.float64, device="cuda")
            Ei = torch.zeros(count, dtype=torch.int64, device="cuda") if inst.integer else None
            P.ising_energy_dev_noalloc(ctx, prob, S, E, Ei)
            torch.cuda.synchronize()
            assert torch.equal(E, E_ref)
            if inst.integer:
                assert torch.equal(Ei, Ei_ref)
                assert np.array_equal(Ei.cpu().numpy(), oracle.energies(inst, S.cpu().numpy().T).astype(np.int64))
    finally:
        P.ising_destroy(ctx)


def test_noalloc_energy_rejects_requests_beyond_the_scratch():
    import torch
    import paper_2312_05837_amd as P
    ctx = P.ising_create(0)
    try:
        inst = I.torus(100, 200, 0, "pm1")          # n = 20000: 5000 partials of 8 bytes per vector
        prob = to_problem(inst)
        S = torch.ones((210, inst.n), dtype=torch.int8, device="cuda")   # 8.4 MB > 8 MiB
        E = torch.zeros(210, dtype=torch.float64, device="cuda")
        with pytest.raises(P.IsingError) as e:
            P.ising_energy_dev_noalloc(ctx, prob, S, E)
        assert e.value.status == P.ISING_EINVAL
        # within the limit it runs (and the rejected call left nothing behind)
        E2 = torch.zeros(100, dtype=torch.float64, device="cuda")
        Ei2 = torch.zeros(100, dtype=torch.int64, device="cuda")
        P.ising_energy_dev_noalloc(ctx, prob, S[:100], E2, Ei2)
        torch.cuda.synchronize()
        assert np.all(Ei2.cpu().numpy() == oracle.energy(inst, np.ones(inst.n, dtype=np.int8)))
    finally:
        P.ising_destroy(ctx)
