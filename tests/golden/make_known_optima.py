"""Write known_optima.json: exhaustive ground-state energies of small seeded instances.

The values are computed by the oracle alone (oracle.brute_force_min, an exhaustive
search over all 2^n spin vectors) and serve as fixed time-to-target energies
of the benchmark.  Run from the repository root: python tests/golden/make_known_optima.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import instances as I  # noqa: E402
import oracle  # noqa: E402


def sk64_sub20():
    """Leading 20 x 20 principal submatrix of the SK N = 64 +-1 instance (seed 0): itself an SK instance."""
    sk = I.sk_pm1(64, 0)
    return I.Instance(20, "sk64_s0_sub20", np.zeros(20, dtype=np.int64), sk.J[:20, :20].copy(), integer=True)


def main():
    out = {}
    inst = sk64_sub20()
    e, _, count = oracle.brute_force_min(inst)
    out["sk64_s0_sub20"] = {"E_min": int(e), "minimisers": int(count),
                            "instance": "leading 20x20 principal submatrix of instances.sk_pm1(64, 0), h = 0",
                            "source": "oracle.brute_force_min (all 2^20 spin vectors)"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "known_optima.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
