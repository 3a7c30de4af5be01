"""Pins of the oracle's metrics (paper Sec. IV) and of the shared random draws."""
import os

import numpy as np

import instances as I
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_table2_arithmetic():
    # Table 2: estimated TTS and speed recomputed from the printed means of chi_hat and T
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table2_comparisons.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for name, chi, t, tts, v in rows:
        chi, t, tts, v = map(float, (chi, t, tts, v))
        assert abs(oracle.tts_hat(t, chi, 1000) / tts - 1) < 0.005, name
        assert abs(oracle.speed(chi, t) / v - 1) < 0.015, name


def test_chi_hat_endpoints_and_eta():
    inst = I.random_integer_field(I.sk_pm1(50, 0), 0, 3)
    emax = np.sqrt(50) * np.sqrt((inst.J.astype(float) ** 2).sum()) + np.abs(inst.h).sum()
    assert np.isclose(oracle.chi_hat(inst, -emax), 1.0)
    assert np.isclose(oracle.chi_hat(inst, emax), 0.0)
    assert np.isclose(oracle.chi_hat(inst, 0.0), 0.5)
    assert oracle.pruning_rate(1000, 51) == 1 - 51 / 1000


def test_splitmix64_published_values():
    # first outputs of SplitMix64 seeded with 0 (reference values of the published generator)
    z = I.splitmix64(0, np.arange(3, dtype=np.uint64))
    assert [int(x) for x in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_draws_are_exact_float32_and_uniform():
    U = I.uniform_draws(7, 64, 1000)
    assert np.array_equal(U.astype(np.float32).astype(np.float64), U)
    assert U.min() >= -1 and U.max() < 1
    assert abs(U.mean()) < 0.01 and abs(U.var() - 1 / 3) < 0.01
    # a replica subset is reproducible on its own
    assert np.array_equal(I.uniform_draws(7, 4, 1000, replica_offset=10), U[10:14])
