"""Small instances whose state space can be enumerated exactly, shared by tests."""
from __future__ import annotations

import itertools

import numpy as np

from synth.instances import instance_from_logical, q12


def tiny_instance(seed: int = 7, N: int = 5, degree_cap: int = 3, with_field: bool = True):
    """All-to-all logical problem on N nodes, couplings ~ N(0, 0.5^2) in Q12,
    sparsified with copy chains under `degree_cap` (N=5, cap 3: 2 copies per
    node, 10 physical spins, as in the paper's five-node example)."""
    rng = np.random.default_rng(seed)
    A = rng.normal(0.0, 0.5, size=(N, N))
    A = np.triu(A, 1)
    A = A + A.T
    Jq = q12(A)
    np.fill_diagonal(Jq, 0)
    b = q12(rng.normal(0.0, 0.3, size=N)) if with_field else None
    return instance_from_logical(Jq, b_logical_q=b, degree_cap=degree_cap)


def all_states(n: int) -> np.ndarray:
    return np.array(list(itertools.product([-1, 1], repeat=n)), dtype=np.int64)


def dense_physical(inst) -> np.ndarray:
    Jp = np.zeros((inst.n, inst.n), dtype=np.int64)
    rows = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
    Jp[rows, inst.col] = inst.J_q
    return Jp


def enumerate_fg(inst):
    """f and g of every physical state, computed in matrix form."""
    S = all_states(inst.n)
    Jp = dense_physical(inst)
    f = -(np.einsum("ki,ij,kj->k", S, Jp, S) // 2) - S @ inst.b_q.astype(np.int64)
    g = ((S[:, inst.copy_a] - S[:, inst.copy_b]) ** 2).sum(axis=1)
    return S, f, g


def boltzmann(f, g, beta, p_q):
    e = (f + int(p_q) * g) / 4096.0
    w = np.exp(-beta * (e - e.min()))
    return w / w.sum()
