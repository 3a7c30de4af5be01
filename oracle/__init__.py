"""Plain, slow, obviously correct CPU oracle of the pruning + domain-selection solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it, to check and time the GPU path.
It shares no code with the HIP implementation; the two only share the seeded
input generators in ``instances``.

Everything is float64 (int64 for integer instances), written as the paper's
definitions and algorithm steps with numpy primitives (matrix products, sums):

* ``energy``    -- E(s) = s^T J s + h^T s (Sec. II, scalar energy form).
* ``prune``     -- Algorithm 1 (Sec. III-A) with the determined-spin and
                   semi-determined-spin rules and the reduced problem (h_G, C).
* ``unprune``   -- retrieval of the full spin vector (Fig. 1c).
* ``ds_run``    -- domain selection (Sec. III-B): sin-theta relaxation of the
                   domain indicator, loss of the relaxed L1 maximisation,
                   gradient descent or ADAM (Sec. IV-B).
* ``metrics``   -- pruning rate, Hamiltonian-ratio estimate, estimated
                   time-to-solution and solution speed (Sec. IV).
* ``brute_force_min`` -- exhaustive ground state for n <= 22.

Readings taken where the paper is silent are stated in each function.
Parity-pinning status: every function here is pinned by tests under
``tests/test_oracle_*.py`` except the free-running domain-selection trajectory
itself, which the paper pins only through the identities those tests check.
"""
from .energy import energy, energies, cut_value, brute_force_min, local_fields
from .prune import prune, unprune, PruneResult, fixed_order_abs_rowsum
from .ds import (ds_run, ds_loss, ds_grad, ds_loss_relaxed, ds_grad_relaxed, wrap_angle, DSResult, converged,
                 convergence_step)
from .metrics import pruning_rate, chi_hat, tts_hat, speed
from .solve import solve
from .frontends import (qubo_value, qubo_to_ising, qubo_instance, maxcut_instance, cut_of,
                        nae3sat_instance, nae_violated)

__all__ = [
    "energy", "energies", "cut_value", "brute_force_min", "local_fields",
    "prune", "unprune", "PruneResult", "fixed_order_abs_rowsum",
    "ds_run", "ds_loss", "ds_grad", "ds_loss_relaxed", "ds_grad_relaxed", "wrap_angle", "DSResult",
    "converged", "convergence_step",
    "pruning_rate", "chi_hat", "tts_hat", "speed", "solve",
    "qubo_value", "qubo_to_ising", "qubo_instance", "maxcut_instance", "cut_of", "nae3sat_instance",
    "nae_violated",
]
