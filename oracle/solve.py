"""End-to-end solve (Fig. 1): pruning, domain selection, retrieval -- oracle only."""
from __future__ import annotations

import numpy as np

from .energy import energy
from .prune import prune, unprune
from .ds import ds_run


def solve(inst, U, steps, opt="adam", lr=6.0, mu=0.5, do_prune=True, **kw):
    """Returns dict(spins, energy, prune=PruneResult|None, ds=DSResult, replica).

    U holds the uniform draws of the reduced problem, shape (R, |G|).  The
    solution is the replica with the lowest best energy (ties: lowest index),
    mapped back through the pruning record; its energy is recomputed on the
    full instance.
    """
    pr = prune(inst) if do_prune else None
    red = pr.reduced if pr is not None else inst
    if red.n == 0:
        s = unprune(pr, np.zeros(0, dtype=np.int8))
        return dict(spins=s, energy=energy(inst, s), prune=pr, ds=None, replica=-1)
    ds = ds_run(red, U, steps, opt=opt, lr=lr, mu=mu, **kw)
    r = int(np.argmin(ds.e_best))  # argmin returns the first (lowest) index on ties
    s_G = ds.s_best[r]
    s = unprune(pr, s_G) if pr is not None else s_G.astype(np.int8)
    return dict(spins=s, energy=energy(inst, s), prune=pr, ds=ds, replica=r)
