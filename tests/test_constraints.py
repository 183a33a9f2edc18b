"""Pins of the oracle's general-constraint path (g = sum_t (a_t.s + d_t)^2)
against what the constraints mean and against exact enumeration (CPU).

The copy-edge path is pinned elsewhere; here the term path is tied to it
(copy edges written as terms must give the same trajectory), the penalty is
checked against the violation it encodes (one-hot groups, a capacity limit
with slack bits), and the sampler against the exact Boltzmann distribution
of E = f + P g on instances small enough to enumerate.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from synth.configs import wishart_small
from synth.constrained import planted_coloring, slack_knapsack, terms_from_copies
from tests.tiny import all_states, boltzmann, dense_physical, tiny_instance


def _enumerate_f(inst):
    S = all_states(inst.n)
    Jp = dense_physical(inst)
    f = -(np.einsum("ki,ij,kj->k", S, Jp, S) // 2) - S @ inst.b_q.astype(np.int64)
    return S, f


def _knapsack_parts(inst):
    """Item weights and slack weights, capacity, from the single term."""
    coef = inst.term_coef.astype(np.int64)
    C = (int(coef.sum()) - int(inst.term_const[0])) // 2
    return coef, C


def _knapsack_g(inst, S):
    """4 (w.x + sum 2^l y - C)^2 from the bits x = (1 + s) / 2."""
    coef, C = _knapsack_parts(inst)
    X = (S + 1) // 2
    return 4 * (X @ coef - C) ** 2


def _coloring_g(V, k, S):
    """4 sum_u (number of colours of node u - 1)^2."""
    X = ((S + 1) // 2).reshape(S.shape[0], V, k)
    return 4 * ((X.sum(axis=2) - 1) ** 2).sum(axis=1)


def test_copy_edges_as_terms_give_the_same_trajectory():
    """(s_a - s_b)^2 is the term a = (1, -1), d = 0: the oracle's term path
    reproduces its copy-edge path bit for bit (states, energies, counters,
    tracking)."""
    w = wishart_small()
    t = terms_from_copies(w.instance)
    f_gs = O.energy(w.instance, w.instance.physical_state(w.instance.planted))[0]
    for seed in (0, 3):
        a = O.run(w.instance, w.beta, w.p_q, mcs_per_swap=5, n_rounds=40, seed=seed, f_target=f_gs,
                  trace=True)
        b = O.run(t, w.beta, w.p_q, mcs_per_swap=5, n_rounds=40, seed=seed, f_target=f_gs, trace=True)
        for key in a:
            assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key
    inst = tiny_instance()
    S = all_states(inst.n).astype(np.int8)
    ti = terms_from_copies(inst)
    for s in S[::7]:
        assert O.energy(inst, s) == O.energy(ti, s)


def test_slack_knapsack_penalty_is_the_capacity_violation():
    """Over every state: g = 4 (w.x + slack - C)^2, zero exactly when the
    slack bits make up the unused capacity, so a state with g = 0 never
    exceeds the capacity; every load up to C has such a slack setting."""
    inst = slack_knapsack(5, seed=2)
    S = all_states(inst.n)
    g = np.array([O.energy(inst, s.astype(np.int8))[1] for s in S])
    assert np.array_equal(g, _knapsack_g(inst, S))
    coef, C = _knapsack_parts(inst)
    X = (S + 1) // 2
    load = X[:, :5] @ coef[:5]
    assert np.all(load[g == 0] <= C)
    for x_items in {tuple(r) for r in X[load <= C][:, :5]}:
        rows = np.all(X[:, :5] == np.array(x_items), axis=1)
        assert np.any(g[rows] == 0)


def test_one_hot_penalty_counts_colours_per_node():
    """Random states of a small colouring instance: g = 4 sum_u (c_u - 1)^2
    with c_u the number of colours node u takes; zero exactly on
    assignments of one colour per node."""
    V, k = 12, 4
    pc = planted_coloring(V, k, degree=3, seed=5)
    rng = np.random.default_rng(0)
    S = rng.choice([-1, 1], size=(300, V * k))
    onehot = -np.ones((50, V * k), dtype=np.int64)
    onehot[np.arange(50)[:, None], np.arange(V) * k + rng.integers(0, k, size=(50, V))] = 1
    S = np.concatenate([S, onehot])
    g = np.array([O.energy(pc.instance, s.astype(np.int8))[1] for s in S])
    assert np.array_equal(g, _coloring_g(V, k, S))
    assert np.all(g[300:] == 0)


def test_coloring_cost_counts_monochromatic_edges():
    """On one-hot states f = weight (monochromatic edges - k |E| / 4); the
    planted colouring is feasible with f = f_target, and by brute force over
    every state of a 4-node, 3-colour instance no feasible state is below
    it."""
    V, k = 10, 3
    pc = planted_coloring(V, k, degree=3, seed=1)
    inst = pc.instance
    rows = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
    edges = {(min(a, b) // k, max(a, b) // k) for a, b in zip(rows, inst.col)}
    rng = np.random.default_rng(3)
    for _ in range(40):
        colours = rng.integers(0, k, size=V)
        s = -np.ones(inst.n, dtype=np.int8)
        s[np.arange(V) * k + colours] = 1
        mono = sum(colours[u] == colours[v] for u, v in edges)
        f, g = O.energy(inst, s)
        assert g == 0
        assert f == 4096 * mono - 4096 * k * len(edges) // 4
    f, g = O.energy(inst, pc.state)
    assert (f, g) == (pc.f_target_q, 0)
    small = planted_coloring(4, 3, degree=2, seed=0)
    S, fe = _enumerate_f(small.instance)
    ge = _coloring_g(4, 3, S)
    assert fe[ge == 0].min() == small.f_target_q
    # with a large enough penalty the minimum of E is a feasible optimum
    e = fe + 4096 * 8 * ge
    assert ge[np.argmin(e)] == 0 and fe[np.argmin(e)] == small.f_target_q


def _state_index(states):
    bits = (states > 0).astype(np.int64)
    n = states.shape[-1]
    return bits @ (1 << np.arange(n - 1, -1, -1))


@pytest.mark.parametrize("which", ["knapsack", "coloring"])
def test_general_constraint_grid_samples_boltzmann(which):
    """2x2 grid: over independent seeds the final state at every position
    has the mean f and g of the Boltzmann distribution of f + P g at that
    (beta, P) (g enumerated from the constraint's meaning), and each
    adjacent pair's swap acceptance equals sum pi_A pi_B min(1, e^x), all
    within 3 standard errors (acceptances from the attempts of 4 further
    rounds run from the final states: one independent Bernoulli sample per
    pair and seed after the burn-in)."""
    if which == "knapsack":
        inst = slack_knapsack(5, seed=2)
        S, f = _enumerate_f(inst)
        g = _knapsack_g(inst, S)
        beta, p_q = np.array([0.1, 0.3]), np.array([512, 2048], dtype=np.int32)
    else:
        inst = planted_coloring(3, 3, degree=2, seed=4).instance
        S, f = _enumerate_f(inst)
        g = _coloring_g(3, 3, S)
        beta, p_q = np.array([0.5, 1.5]), np.array([1024, 4096], dtype=np.int32)
    finals, pa, pt, ba, bt = [], [], [], [], []
    for sd in range(600):
        r = O.run(inst, beta, p_q, mcs_per_swap=2, n_rounds=24, seed=sd)
        finals.append(r["states"])
        pa.append(r["p_acc"]); pt.append(r["p_att"]); ba.append(r["b_acc"]); bt.append(r["b_att"])
        if sd < 20:
            idx = _state_index(r["states"])
            assert np.array_equal(r["f"], f[idx]) and np.array_equal(r["g"], g[idx])
    idx = _state_index(np.array(finals))
    pa, pt, ba, bt = map(np.array, (pa, pt, ba, bt))
    for i in range(2):
        for j in range(2):
            p = boltzmann(f, g, beta[i], p_q[j])
            for obs in (f, g):
                x = obs[idx[:, i * 2 + j]].astype(np.float64)
                mean = (p * obs).sum()
                sd = np.sqrt(max((p * obs ** 2).sum() - mean ** 2, 0.0))
                assert abs(x.mean() - mean) < 3 * sd / np.sqrt(len(x)) + 1e-9
    pa, pt, ba, bt = [], [], [], []
    for sd, s0 in enumerate(finals):
        r = O.run(inst, beta, p_q, mcs_per_swap=2, n_rounds=4, seed=10**6 + sd, s0=s0)
        pa.append(r["p_acc"]); pt.append(r["p_att"]); ba.append(r["b_acc"]); bt.append(r["b_att"])
    pa, pt, ba, bt = map(np.array, (pa, pt, ba, bt))
    for i in range(2):
        pA, pB = boltzmann(f, g, beta[i], p_q[0]), boltzmann(f, g, beta[i], p_q[1])
        x = beta[i] * (p_q[1] - p_q[0]) * (g[None, :] - g[:, None]) / 4096.0
        acc = (pA[:, None] * pB[None, :] * np.exp(np.minimum(x, 0))).sum()
        rate = pa[:, i, 0] / pt[:, i, 0]
        assert abs(rate.mean() - acc) < 3 * np.sqrt(acc * (1 - acc) / len(rate))
    for j in range(2):
        pA, pB = boltzmann(f, g, beta[0], p_q[j]), boltzmann(f, g, beta[1], p_q[j])
        e = f + int(p_q[j]) * g
        x = (beta[1] - beta[0]) * (e[None, :] - e[:, None]) / 4096.0
        acc = (pA[:, None] * pB[None, :] * np.exp(np.minimum(x, 0))).sum()
        rate = ba[:, j, 0] / bt[:, j, 0]
        assert abs(rate.mean() - acc) < 3 * np.sqrt(acc * (1 - acc) / len(rate))


@pytest.mark.parametrize("which", ["knapsack", "coloring"])
def test_general_constraint_long_run_batch_means(which):
    """One long chain per instance (4 x 10^4 rounds): every position's mean f
    and g (g enumerated from the constraint's meaning) and every pair's swap
    acceptance within 3 standard errors of the exact product-Boltzmann
    values, errors from 40 batch means after 10 % burn-in."""
    from tests.tiny import batch_means_check, exact_grid_expectations, oracle_long_run
    if which == "knapsack":
        inst = slack_knapsack(5, seed=2)
        S, f = _enumerate_f(inst)
        g = _knapsack_g(inst, S)
        beta, p_q = np.array([0.1, 0.3]), np.array([512, 2048], dtype=np.int32)
    else:
        inst = planted_coloring(3, 3, degree=2, seed=4).instance
        S, f = _enumerate_f(inst)
        g = _coloring_g(3, 3, S)
        beta, p_q = np.array([0.5, 1.5]), np.array([1024, 4096], dtype=np.int32)
    fs, gs, acc, att = oracle_long_run(O, inst, beta, p_q, chunks=10000, mcs=2, seed=5)
    fails = batch_means_check(fs, gs, acc, att, exact_grid_expectations(inst, beta, p_q, fg=(f, g)))
    assert not fails, "\n".join(fails)


def test_one_replica_with_terms_is_a_gibbs_chain():
    """I = J = 1 on the knapsack instance: the state histogram over seeds
    matches Boltzmann of f + P g (KL within 3x the sampling bias)."""
    inst = slack_knapsack(5, seed=2)
    S, f = _enumerate_f(inst)
    g = _knapsack_g(inst, S)
    beta, p_q = np.array([0.2]), np.array([1024], dtype=np.int32)
    finals = [O.run(inst, beta, p_q, mcs_per_swap=3, n_rounds=6, seed=sd)["states"][0]
              for sd in range(3000)]
    idx = _state_index(np.array(finals))
    p = boltzmann(f, g, beta[0], p_q[0])
    hist = np.bincount(idx, minlength=len(p)) / len(idx)
    nz = hist > 0
    kl = float((hist[nz] * np.log(hist[nz] / p[nz])).sum())
    k_eff = int((p > 1e-6).sum())
    assert kl < 3 * (k_eff - 1) / (2 * len(idx))
