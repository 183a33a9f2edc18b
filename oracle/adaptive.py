"""Algorithm 2 (adaptive schedule for 2D-PT), written from the paper for the
oracle's sampler.

TEST INFRASTRUCTURE ONLY: used by the tests to check the library's adaptive
schedule; nothing in the library imports it.

Steps in the paper's order and notation.  A population at (beta, P) is
N_chain independent chains from random initial states after MCS sweeps (the
oracle run on a 1 x N_chain grid with P-swaps off); sigma_E, sigma_g are
population standard deviations of E = f + P g (energy units) and of g, and
mean_g the mean of g.

Readings where the paper is silent (the same ones the library takes): rows
with sigma_g = 0 give no candidate penalty and no column is added without a
candidate; in the first column sigma_E = 0 ends the rows like sigma_E <=
sigma_min, in later columns it leaves beta unchanged; at most I rows; the
k-th population drawn (from 0) uses seed + 1 + k; penalties are rounded to
Q12 half away from zero whenever a population runs and in the output.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def _q12(x):
    return int(np.sign(x) * np.floor(abs(x) * 4096.0 + 0.5))


def population(inst, beta, P, N_chain, MCS, seed):
    """sigma_E, sigma_g, mean_g of N_chain independent chains at (beta, P)
    after MCS sweeps from random initial states."""
    Pq = _q12(P)
    out = O.run(inst, np.array([beta]), np.array([Pq] * N_chain, dtype=np.int32), mcs_per_swap=MCS,
                n_rounds=1, seed=seed, flags=O.NO_PSWAP)
    f = out["f"].astype(np.float64)
    g = out["g"].astype(np.float64)
    E = (f + Pq * g) / 4096.0
    return np.std(E), np.std(g), np.mean(g)


def adaptive_schedule(inst, beta0, P0, I, J, sigma_min, alpha_beta, alpha_P, N_chain, MCS, seed):
    draws = [0]

    def population_k(beta, P):
        out = population(inst, beta, P, N_chain, MCS, seed + 1 + draws[0])
        draws[0] += 1
        return out

    # adaptive schedule on the first column, penalty P0
    beta_s = {(1, 1): beta0}
    P_s = {}
    i = 1
    while i <= I:
        sigma_E, sigma_g, _ = population_k(beta_s[(i, 1)], P0)
        if sigma_E > sigma_min:
            beta_s[(i + 1, 1)] = beta_s[(i, 1)] + alpha_beta / sigma_E
            if sigma_g > 0:
                P_s[(i, 2)] = P0 + alpha_P / (beta_s[(i, 1)] * sigma_g)
            i += 1
        else:
            break
    I = min(i, I)
    cand = [P_s[(r, 2)] for r in range(1, I + 1) if (r, 2) in P_s]
    P = {1: P0}
    if cand:
        P[2] = np.median(cand)

    # adaptive schedule for the remaining columns
    j = 2
    while j <= J and j in P:
        beta_s[(1, j)] = beta0
        for i in range(1, I + 1):
            sigma_E, sigma_g, mean_g = population_k(beta_s[(i, j)], P[j])
            beta_s[(i + 1, j)] = beta_s[(i, j)] + (alpha_beta / sigma_E if sigma_E > 0 else 0.0)
            if sigma_g > 0:
                P_s[(i, j + 1)] = P[j] + alpha_P / (beta_s[(i, j)] * sigma_g)
        if mean_g < 0.5:
            break
        cand = [P_s[(r, j + 1)] for r in range(1, I + 1) if (r, j + 1) in P_s]
        if j + 1 <= J and cand:
            P[j + 1] = np.median(cand)
        j += 1

    # final beta schedule: median over the columns, row by row
    cols = sorted(P)
    beta = np.array([np.median([beta_s[(r, c)] for c in cols]) for r in range(1, I + 1)])
    return beta, np.array([_q12(P[c]) for c in cols], dtype=np.int32), draws[0]
