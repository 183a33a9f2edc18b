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


# ------------------------------------------------------------------
# Long runs against the exact stationary distribution of the grid.
#
# The stationary distribution of 2D-PT is the product over grid positions of
# the Boltzmann distributions at (beta_i, P_j) (Appendix A), so every
# position's mean f and g and every adjacent pair's swap acceptance
# sum_{s,t} pi_A(s) pi_B(t) min(1, e^x) (x of Eq. 2 or Eq. 3 with s at the
# left/upper and t at the right/lower position) are known exactly by
# enumeration.

def exact_grid_expectations(inst, beta, p_q, fg=None):
    """Exact mean f, mean g per position [I, J] and acceptance per P pair
    [I, J-1] and beta pair [J, I-1], and the standard deviations of f and g
    per position.  fg: (f, g) of every state when g is not the copy
    constraint (enumerated from the constraint's meaning)."""
    f, g = fg if fg is not None else enumerate_fg(inst)[1:]
    I, J = len(beta), len(p_q)
    mf = np.zeros((I, J))
    mg = np.zeros((I, J))
    sf = np.zeros((I, J))
    sg = np.zeros((I, J))
    pi = {}
    for i in range(I):
        for j in range(J):
            p = boltzmann(f, g, beta[i], p_q[j])
            pi[i, j] = p
            mf[i, j] = (p * f).sum()
            mg[i, j] = (p * g).sum()
            sf[i, j] = np.sqrt(max((p * (f - mf[i, j]) ** 2).sum(), 0.0))
            sg[i, j] = np.sqrt(max((p * (g - mg[i, j]) ** 2).sum(), 0.0))
    accp = np.zeros((I, max(J - 1, 0)))
    for i in range(I):
        for k in range(J - 1):
            x = beta[i] * (int(p_q[k + 1]) - int(p_q[k])) * (g[None, :] - g[:, None]) / 4096.0
            accp[i, k] = (pi[i, k][:, None] * pi[i, k + 1][None, :] * np.exp(np.minimum(x, 0.0))).sum()
    accb = np.zeros((J, max(I - 1, 0)))
    for j in range(J):
        e = f + int(p_q[j]) * g
        for k in range(I - 1):
            x = (beta[k + 1] - beta[k]) * (e[None, :] - e[:, None]) / 4096.0
            accb[j, k] = (pi[k, j][:, None] * pi[k + 1, j][None, :] * np.exp(np.minimum(x, 0.0))).sum()
    return mf, mg, accp, accb, sf, sg


def batch_means_check(samples_f, samples_g, acc, att, exact, n_batches=40, burn=0.1, z=3.0):
    """Batch-means comparison of a long run with the exact expectations.

    samples_f, samples_g: [T, I, J] per-position f and g, one row per sample
    (consecutive samples of one chain); acc, att: [T, ...] per-sample
    increments of the accept / attempt counters of the P pairs and beta pairs
    (tuples (P, beta)).  After dropping the first `burn` fraction the samples
    are cut into n_batches consecutive batches; the standard error of each
    estimate is the standard deviation of its batch means over
    sqrt(n_batches), but never below the error of as many independent
    samples (the exact standard deviation over sqrt(samples); for an
    acceptance rate a, sqrt(a (1 - a) / attempts)), which a positively
    correlated chain cannot beat and which keeps events rarer than one per
    run (all batch means equal) from claiming a zero error.  Returns a list
    of failures (empty when every estimate is within z standard errors of
    its exact value)."""
    mf, mg, accp, accb, sf, sg = exact
    T = samples_f.shape[0]
    t0 = int(T * burn)
    L = (T - t0) // n_batches
    assert L >= 1, "not enough samples for the batches"

    def bm(x):
        x = x[t0:t0 + L * n_batches]
        return x.reshape((n_batches, L) + x.shape[1:]).mean(axis=1)

    fails = []

    def check(name, batch_est, want, floor):
        est = batch_est.mean(axis=0)
        se = np.maximum(batch_est.std(axis=0, ddof=1) / np.sqrt(n_batches), floor)
        bad = np.abs(est - want) > z * se + 1e-12
        for idx in zip(*np.nonzero(bad)):
            fails.append(f"{name}{tuple(int(v) for v in idx)}: {est[idx]:.6g} vs exact {want[idx]:.6g} "
                         f"(se {se[idx]:.3g})")
    n = L * n_batches
    check("mean f", bm(samples_f.astype(np.float64)), mf, sf / np.sqrt(n))
    check("mean g", bm(samples_g.astype(np.float64)), mg, sg / np.sqrt(n))
    for name, a, t, want in (("P acceptance", acc[0], att[0], accp), ("beta acceptance", acc[1], att[1], accb)):
        if want.size == 0:
            continue
        ba, bt = bm(a.astype(np.float64)), bm(t.astype(np.float64))
        attempts = bt.sum(axis=0) * L
        check(name, ba / np.maximum(bt, 1e-300), want,
              np.sqrt(want * (1.0 - want) / np.maximum(attempts, 1.0)))
    return fails


def oracle_long_run(O, inst, beta, p_q, chunks, mcs, seed):
    """One long 2D-PT chain from the oracle module O, sampled every 4 rounds.

    The chain runs in chunks of 4 rounds (one full period of Algorithm 1's
    schedule: P odd pairs, P even pairs, beta odd pairs, beta even pairs),
    each chunk continuing from the previous chunk's final configurations
    with a fresh random stream (seed * 10^6 + chunk): every chunk applies
    the same transition kernel, so the sequence of chunk-end states is one
    Markov chain with the product-Boltzmann stationary distribution.
    Returns f, g [chunks, I, J] and the counter increments ((P acc, beta acc),
    (P att, beta att)) of every chunk."""
    I, J = len(beta), len(p_q)
    fs = np.zeros((chunks, I, J), np.int64)
    gs = np.zeros((chunks, I, J), np.int64)
    pa = np.zeros((chunks, I, max(J - 1, 0)), np.int64)
    pt = np.zeros_like(pa)
    ba = np.zeros((chunks, J, max(I - 1, 0)), np.int64)
    bt = np.zeros_like(ba)
    s = None
    for c in range(chunks):
        r = O.run(inst, beta, p_q, mcs_per_swap=mcs, n_rounds=4, seed=seed * 10**6 + c, s0=s)
        s = r["states"]
        fs[c] = r["f"].reshape(I, J)
        gs[c] = r["g"].reshape(I, J)
        pa[c], pt[c], ba[c], bt[c] = r["p_acc"], r["p_att"], r["b_acc"], r["b_att"]
    return fs, gs, (pa, ba), (pt, bt)
