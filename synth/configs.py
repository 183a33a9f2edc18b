"""Named synthetic workloads (sizes and schedules) and their seeded builders.

Each workload is a planted Wishart problem family sparsified with copy chains
under a degree cap, run on an I x J replica grid with geometric inverse
temperatures and linear penalties.  The sweep-per-swap ratio is 50 (the
ratio the paper uses for its Wishart study) unless the workload says
otherwise.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .constrained import planted_coloring
from .instances import (Instance, build_instance, geometric_betas, instance_from_logical,
                        linear_penalties_q, q12)


@dataclasses.dataclass
class Workload:
    name: str
    instance: Instance
    beta: np.ndarray           # float64[I], ascending
    p_q: np.ndarray            # int32[J], non-decreasing, Q12
    mcs_per_swap: int
    sweeps: int
    seed: int
    f_target_q: int | None = None   # a known optimum's f, when the family plants one

    @property
    def n_beta(self) -> int:
        return int(self.beta.shape[0])

    @property
    def n_p(self) -> int:
        return int(self.p_q.shape[0])

    @property
    def replicas(self) -> int:
        return self.n_beta * self.n_p

    @property
    def rounds(self) -> int:
        return self.sweeps // self.mcs_per_swap

    @property
    def updates_per_sweep(self) -> int:
        return self.replicas * self.instance.n


_CACHE: dict = {}


def _inst(N, alpha, seed, D):
    key = (N, alpha, seed, D)
    if key not in _CACHE:
        _CACHE[key] = build_instance(N, alpha, seed, degree_cap=D)
    return _CACHE[key]


def wishart_small(seed: int = 0) -> Workload:
    """N=12, alpha=0.5, degree cap 4, 8x4 grid (beta 0.1..5, P 0..4), 1e4 sweeps."""
    return Workload("wishart-N12-D4-8x4", _inst(12, 0.5, 0, 4),
                    geometric_betas(0.1, 5.0, 8), linear_penalties_q(0, 4, 4),
                    50, 10_000, seed)


def wishart_n200(seed: int = 0) -> Workload:
    """N=200, alpha=0.8, degree cap 8, 32x16 grid (beta 0.05..10, P 0..8), swap every sweep, 1e5 sweeps."""
    return Workload("wishart-N200-D8-32x16", _inst(200, 0.8, 0, 8),
                    geometric_betas(0.05, 10.0, 32), linear_penalties_q(0, 8, 16),
                    1, 100_000, seed)


def batched_sizes(count: int = 64, seed0: int = 0):
    """(N, alpha) of the batched family: N ~ U{50..400}, alpha ~ U{0.5, 0.8}."""
    out = []
    for k in range(count):
        rng = np.random.default_rng(10_000 + seed0 + k)
        N = int(rng.integers(50, 401))
        alpha = float(rng.choice([0.5, 0.8]))
        out.append((N, alpha, seed0 + k))
    return out


def batched_member(N: int, alpha: float, seed: int) -> Workload:
    """One member of the batched family: degree cap 6, 16x8 grid (beta 0.1..8, P 0..6), 5e4 sweeps."""
    return Workload(f"wishart-N{N}-D6-16x8-s{seed}", _inst(N, alpha, seed, 6),
                    geometric_betas(0.1, 8.0, 16), linear_penalties_q(0, 6, 8),
                    50, 50_000, seed)


def wishart_n1000(seed: int = 0) -> Workload:
    """N=1000, alpha=0.6, degree cap 6, 64x32 grid (beta 0.02..12, P 0..10), 2e5-sweep cap."""
    return Workload("wishart-N1000-D6-64x32", _inst(1000, 0.6, 0, 6),
                    geometric_betas(0.02, 12.0, 64), linear_penalties_q(0, 10, 32),
                    50, 200_000, seed)


def serving_grid(N: int):
    """Replica grid scaled with N: I = 8*2^round(0.75*(log2 N - 6)) in [8, 64], J = I/2."""
    I = 8 * 2 ** int(round(0.75 * (math.log2(N) - 6)))
    I = max(8, min(64, I))
    return I, I // 2


def serving_member(N: int, alpha: float, seed: int, sweeps: int) -> Workload:
    I, J = serving_grid(N)
    return Workload(f"serve-N{N}-D6-{I}x{J}-s{seed}", _inst(N, alpha, seed, 6),
                    geometric_betas(0.1, 8.0, I), linear_penalties_q(0, 6, J),
                    50, sweeps, seed)


def jcolumn_member(N: int, seed: int) -> Workload:
    """A planted Wishart instance as in the paper's 2D-PT vs J-column PT
    comparison: alpha 0.75, three copies per node, 50 sweeps per swap; a
    16 x 8 grid (beta geometric 0.1..8, P linear 0..6)."""
    inst = build_instance(N, 0.75, seed, copies=3)
    return Workload(f"wishart-N{N}-c3-16x8-s{seed}", inst, geometric_betas(0.1, 8.0, 16),
                    linear_penalties_q(0, 6, 8), 50, 0, seed)


def fig2_workload(seed: int = 0, rounds: int = 2000) -> Workload:
    """The sampling experiment of Fig. 2 on a stand-in instance: a 5-node
    all-to-all logical problem (couplings ~ N(0, 1), fields ~ N(0, 0.5^2),
    Q12; the paper's full-adder couplings are not given), two copies per node
    under degree cap 3 (10 physical spins), one row at beta = 1, penalties
    {2, 4, 6, 8}, a P-swap step every 500 sweeps."""
    rng = np.random.default_rng(1000 + seed)
    A = np.triu(rng.normal(0.0, 1.0, size=(5, 5)), 1)
    Jq = q12(A + A.T)
    np.fill_diagonal(Jq, 0)
    b = q12(rng.normal(0.0, 0.5, size=5))
    inst = instance_from_logical(Jq, b_logical_q=b, degree_cap=3)
    return Workload(f"fig2-standin-N5-s{seed}", inst, np.array([1.0]), q12([2.0, 4.0, 6.0, 8.0]),
                    500, 500 * rounds, seed)


def coloring_workload(seed: int = 0, V: int = 4000, k: int = 4, degree: int = 6) -> Workload:
    """General constraints: planted graph k-colouring in one-hot form (V
    nodes, k spins per node, at most `degree` neighbours per node, one
    one-hot term per node; 16,000 spins by default), on a 32 x 16 grid
    (beta geometric 0.2..5, P linear 0..4) with 50 sweeps per swap.  The
    planted colouring is a feasible optimum (f_target_q)."""
    key = ("coloring", V, k, degree, seed)
    if key not in _CACHE:
        _CACHE[key] = planted_coloring(V, k, degree, seed)
    pc = _CACHE[key]
    return Workload(f"coloring-V{V}-k{k}-d{degree}-32x16", pc.instance, geometric_betas(0.2, 5.0, 32),
                    linear_penalties_q(0, 4, 16), 50, 10_000, seed, f_target_q=pc.f_target_q)
