"""Adaptive beta / penalty schedule for 2D-PT (Algorithm 2 of the paper).

A host loop over short population runs on the GPU sampler.  A population
at (beta, P) is n_chain independent Markov chains started from random
states, each run for `mcs` sweeps: one problem with a 1 x n_chain grid at
that beta and penalty, with P-swaps off (a single row has no beta-swaps),
so no chain ever exchanges with another.  From the chains' final states:
sigma_E (population standard deviation of E = f + P g, in energy units),
sigma_g (of the constraint g) and mean_g.

First column (penalty P0): starting at beta0, rows are added with
beta <- beta + alpha_beta / sigma_E while sigma_E > sigma_min (at most
i_max rows); each row also proposes the next column's penalty
P + alpha_P / (beta sigma_g), and the next column takes the median of the
proposals.  Further columns: the whole beta ladder is rebuilt from beta0 at
the column's penalty (same rule, fixed row count), each row again proposing
a next penalty; columns are added until the coldest row's mean_g < 0.5
(constraints satisfied) or j_max columns.  The final beta of each row is
the median over the columns' ladders.

Readings where the paper is silent: a row with sigma_g = 0 (every chain
with the same g) proposes no penalty, and if no row proposes one no column
is added; sigma_E = 0 counts as reaching sigma_min; the number of rows is
capped at i_max; population n (counted from 0 over the whole procedure)
uses seed + 1 + n.  Penalties are kept in energy units and rounded to Q12
(half away from zero) when a population runs and in the result.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import tdpt as T


def q12_scalar(x: float) -> int:
    return int(np.sign(x) * np.floor(abs(x) * 4096.0 + 0.5))


@dataclasses.dataclass
class Schedule:
    beta: np.ndarray            # float64[I], ascending
    p_q: np.ndarray             # int32[J], non-decreasing, Q12
    beta_ladders: list          # per column, the ladder it built (I + 1 values)
    populations: int            # population runs made


class _Sampler:
    def __init__(self, instance: "T.Instance", n_chain: int, mcs: int, seed: int, device: str):
        self.instance, self.n_chain, self.mcs, self.seed, self.device = instance, n_chain, mcs, seed, device
        self.count = 0

    def stats(self, beta: float, p: float):
        pq = q12_scalar(p)
        cfg = T.RunConfig([beta], [pq] * self.n_chain, mcs_per_swap=self.mcs,
                          seed=self.seed + 1 + self.count, flags=T.NO_PSWAP)
        self.count += 1
        prob = T.Problem(self.instance, cfg, device=self.device)
        prob.run(1)
        f, g = prob.energies()
        prob.close()
        e = (f.astype(np.float64) + float(pq) * g.astype(np.float64)) / 4096.0
        return float(np.std(e)), float(np.std(g.astype(np.float64))), float(np.mean(g))


def adaptive_schedule(instance: "T.Instance", *, beta0: float, p0: float, i_max: int, j_max: int,
                      sigma_min: float, alpha_beta: float = 1.0, alpha_p: float = 1.0,
                      n_chain: int = 64, mcs: int = 100, seed: int = 0, device: str = "cuda") -> Schedule:
    """Algorithm 2: beta ladder and penalties for a 2D-PT grid of at most
    i_max x j_max replicas."""
    S = _Sampler(instance, n_chain, mcs, seed, device)
    # first column
    ladder = [float(beta0)]
    proposals = []
    while len(ladder) <= i_max:
        b = ladder[-1]
        sig_e, sig_g, _ = S.stats(b, p0)
        if not sig_e > sigma_min:
            break
        ladder.append(b + alpha_beta / sig_e)
        if sig_g > 0:
            proposals.append(p0 + alpha_p / (b * sig_g))
    rows = min(len(ladder), i_max)
    ladders = [ladder]
    penalties = [float(p0)]
    # further columns
    while len(penalties) < j_max and proposals:
        p = float(np.median(proposals))
        lad = [float(beta0)]
        proposals = []
        mean_g = 0.0
        for i in range(rows):
            b = lad[i]
            sig_e, sig_g, mean_g = S.stats(b, p)
            lad.append(b + alpha_beta / sig_e if sig_e > 0 else b)
            if sig_g > 0:
                proposals.append(p + alpha_p / (b * sig_g))
        ladders.append(lad)
        penalties.append(p)
        if mean_g < 0.5:
            break
    beta = np.array([float(np.median([lad[i] for lad in ladders])) for i in range(rows)])
    p_q = np.array([q12_scalar(p) for p in penalties], dtype=np.int32)
    return Schedule(beta=beta, p_q=p_q, beta_ladders=ladders, populations=S.count)
