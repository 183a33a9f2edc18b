"""Sampling quality of the last replica (the experiment of Fig. 2).

The empirical distribution of the bottom-right replica's logical state,
accumulated over the rounds of one run, against the Boltzmann distribution
of the logical problem; the paper measures it with the Kullback-Leibler
divergence, whose expected value for t independent samples approaches
(2^N - 1) / (2 t) (Appendix B).

A node's logical value is read from its lowest-numbered physical copy.
Logical states are indexed by sum_k ((x_k + 1) / 2) 2^k.
"""
from __future__ import annotations

import itertools

import numpy as np


def logical_index(states: np.ndarray, first_copy: np.ndarray) -> np.ndarray:
    """Index of the logical state read from physical states (rows)."""
    bits = (np.asarray(states)[..., first_copy] > 0).astype(np.int64)
    return bits @ (1 << np.arange(first_copy.shape[0], dtype=np.int64))


def first_copies(logical_of) -> np.ndarray:
    """Lowest-numbered physical spin of every logical node."""
    logical_of = np.asarray(logical_of)
    _, idx = np.unique(logical_of, return_index=True)
    return idx


def boltzmann_logical(J_logical_q, b_logical_q, beta: float) -> np.ndarray:
    """Exact distribution of the logical problem E = -sum_{i<j} J x x - sum b x
    (Q12 inputs) at inverse temperature beta, by enumeration."""
    J = np.asarray(J_logical_q, dtype=np.float64) / 4096.0
    N = J.shape[0]
    b = np.zeros(N) if b_logical_q is None else np.asarray(b_logical_q, dtype=np.float64) / 4096.0
    X = np.array(list(itertools.product([-1.0, 1.0], repeat=N)))[:, ::-1]  # row k: bits of k
    E = -0.5 * np.einsum("ki,ij,kj->k", X, J, X) - X @ b
    w = np.exp(-beta * (E - E.min()))
    return w / w.sum()


def kl_divergence(counts, target) -> float:
    """KL(empirical || target) in nats; empty states contribute 0."""
    counts = np.asarray(counts, dtype=np.float64)
    p = counts / counts.sum()
    m = p > 0
    return float(np.sum(p[m] * np.log(p[m] / np.asarray(target)[m])))


def sample_bottom_right(problem, rounds: int, first_copy: np.ndarray, checkpoints=()):
    """Count the bottom-right replica's logical state after each of `rounds`
    rounds of a fresh problem.  Returns the counts and, for each checkpoint
    (a number of samples), the counts at that point.

    A problem created with RunConfig(hist_logical=True) (and an instance
    with logical_of) counts on the device, in the library's per-round
    histogram: it runs from checkpoint to checkpoint and the counts are read
    there.  Otherwise the states are read back and counted on the host after
    every round."""
    ck = sorted(set(int(c) for c in checkpoints if 0 < int(c) <= rounds))
    snaps = {}
    if problem.cfg.hist_logical:
        done = 0
        for c in ck + [rounds]:
            if c > done:
                problem.run(c - done)
                done = c
            if c in ck and c not in snaps:
                snaps[c] = problem.histogram()[0].astype(np.int64)
        counts, samples = problem.histogram()
        if samples != rounds:
            raise ValueError("the problem had run before sampling started")
        return counts.astype(np.int64), snaps
    counts = np.zeros(1 << first_copy.shape[0], dtype=np.int64)
    for t in range(1, rounds + 1):
        problem.run(1)
        s = problem.states()[-1]
        counts[logical_index(s, first_copy)] += 1
        if t in ck:
            snaps[t] = counts.copy()
    return counts, snaps
