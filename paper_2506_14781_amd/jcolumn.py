"""J-column parallel tempering, the baseline the paper sets against 2D-PT.

Standard PT over the same beta ladder, repeated J times at one fixed
penalty (the mean of the 2D-PT penalties), with the best feasible energy
among the J runs picked afterwards ("Ground-state optimization under
constraints", and the caption of Fig. 3).  It uses as many replicas and
sweeps as the I x J 2D-PT grid.

Each column is a problem of its own (an I x 1 grid, so it tracks its own
coldest replica, and a 1-column grid never attempts a P-swap); the columns
of all instances run together in one batch.  Columns draw from independent
random streams: column j of a run with seed s uses seed column_seed(s, j).
"""
from __future__ import annotations

import numpy as np

from . import tdpt as T


def mean_penalty_q(p_q) -> int:
    """The fixed penalty of J-column PT: the mean of the 2D-PT penalties
    (Q12, rounded half away from zero)."""
    m = float(np.mean(np.asarray(p_q, dtype=np.float64)))
    return int(np.sign(m) * np.floor(abs(m) + 0.5))


def column_seed(seed: int, j: int) -> int:
    return ((int(seed) << 8) + 1 + int(j)) & 0xFFFFFFFFFFFFFFFF


def column_configs(beta, p_q, *, mcs_per_swap: int, seed: int, f_target=None, trace_cap: int = 0):
    """The J run configurations of J-column PT for a 2D-PT grid (beta, p_q)."""
    p = mean_penalty_q(p_q)
    return [T.RunConfig(beta, [p], mcs_per_swap=mcs_per_swap, seed=column_seed(seed, j),
                        f_target=f_target, trace_cap=trace_cap)
            for j in range(len(p_q))]


def best_feasible(problems) -> int | None:
    """Best feasible energy (f_q) over the columns' coldest replicas, None if
    no column has found a feasible state yet."""
    fs = [p.query()["best_f_q"] for p in problems]
    fs = [f for f in fs if f < (1 << 62)]
    return min(fs) if fs else None


def first_hit(problems) -> int:
    """Earliest sweep at which any column's coldest replica hit the target
    (-1: none)."""
    hits = [p.query()["first_hit_sweep"] for p in problems]
    hits = [h for h in hits if h >= 0]
    return min(hits) if hits else -1
