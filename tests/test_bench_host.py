"""Host-side checks of bench.py (no GPU): the one-GPU contract, the roofline's algorithmic
bytes, and that every committed traffic record still matches the kernel sources it was
taken on (a kernel change makes bench.py report traffic as null until the counters are
taken again)."""
import json
import os
import subprocess
import sys

import pytest

import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_sparse_roofline_bytes_torus_100x200():
    # per step: nnz (4-byte column + 1-byte +-1 value) + 4 (n + 1) row pointers + n R (2 + 4)
    # for the vertex operand read and the product written once
    import bench
    inst = I.torus(100, 200, 0, "pm1")
    nnz = int(inst.col.size)
    assert nnz == 80000
    rf = bench.sparse_roofline(inst, inst.n, nnz, 256, 10000, 52.0, "adam", "vertex", "no_such_workload")
    assert rf["algorithmic_bytes_per_step"] == 80000 * 5 + 4 * 20001 + 20000 * 256 * 6 == 31200004
    assert rf["frac"] == pytest.approx(31200004 * 10000 / 52.0e-3 / 8e12)
    assert rf["traffic"] is None  # no record for an unknown workload


def _traffic_records():
    out = []
    for f in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        if f.startswith("traffic_") and f.endswith(".md"):
            stem = f[len("traffic_"):-len(".md")]
            kernel = "k_dense_step" if stem.startswith("k_dense_step_") else "k_ds"
            out.append((kernel, stem[len(kernel) + 1:]))
    return out


@pytest.mark.parametrize("kernel,workload", _traffic_records(), ids=[f"{k}-{w}" for k, w in _traffic_records()])
def test_traffic_records_match_current_sources(kernel, workload):
    import bench
    assert bench.recorded_traffic(kernel, workload) is not None, (kernel, workload)
