"""General constraint functions on the GPU vs the CPU oracle, bit-exact,
through the C ABI (g = sum_t (a_t.s + d_t)^2 instead of copy edges).

Cases: a capacity limit with slack spins (one term over every spin, unequal
coefficients, nonzero constant), one-hot colouring problems (many small
terms), copy chains written as terms (must reproduce the copy-edge path),
wide constraint rows, both drivers, batches that mix constraint kinds, and
the colouring workload the benchmark times (bit-exact on a sub-grid,
invariants on the full grid).
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from synth.configs import coloring_workload, wishart_small
from synth.constrained import planted_coloring, slack_knapsack, terms_from_copies
from tests.test_gpu_parity import _say, _with_env, assert_same, both, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2506_14781_amd as T
    return T


@pytest.mark.parametrize("I,J,mcs", [(1, 1, 3), (2, 2, 2), (3, 5, 1)])
def test_slack_knapsack(T, I, J, mcs):
    inst = slack_knapsack(5, seed=2)
    beta = np.geomspace(0.05, 0.8, I)
    p_q = np.linspace(256, 4096, J).astype(np.int32)
    both(T, inst, beta, p_q, mcs=mcs, rounds=30, seed=4, label=f"knapsack {I}x{J}")


def test_wide_constraint_rows(T):
    """A knapsack over 24 items (30 spins in one term: 29 constraint
    neighbours per spin, rows streamed 4 at a time) and a 10-colour
    problem."""
    inst = slack_knapsack(24, seed=1)
    both(T, inst, np.geomspace(0.01, 0.2, 4), np.array([0, 64, 128, 256], np.int32), mcs=2, rounds=20,
         seed=7, label="knapsack-24")
    pc = planted_coloring(30, 10, degree=4, seed=2)
    both(T, pc.instance, np.geomspace(0.2, 3.0, 4), np.array([0, 2048, 4096], np.int32), mcs=3, rounds=20,
         seed=1, f_target=pc.f_target_q, label="coloring-30x10")


@pytest.mark.parametrize("driver", ["0", "1"])
def test_planted_coloring_both_drivers(T, driver):
    pc = planted_coloring(200, 4, degree=5, seed=3)
    beta = np.geomspace(0.3, 4.0, 8)
    p_q = np.linspace(0, 8192, 4).astype(np.int32)
    o, P = _with_env("TDPT_PERSISTENT", driver, lambda: both(
        T, pc.instance, beta, p_q, mcs=5, rounds=40, seed=2, f_target=pc.f_target_q,
        label=f"coloring-200x4 driver {driver}"))
    assert P.query()["driver"] == int(driver)


def test_copy_chains_as_terms_match_copy_edges(T):
    """The N=12 Wishart workload with its copy edges given as terms runs the
    same trajectory on the GPU as through the copy-edge layout (and as the
    oracle)."""
    w = wishart_small()
    t = terms_from_copies(w.instance)
    f_gs = O.energy(w.instance, w.instance.physical_state(w.instance.planted))[0]
    o, P = both(T, t, w.beta, w.p_q, mcs=w.mcs_per_swap, rounds=200, seed=5, f_target=f_gs,
                label="wishart-N12 as terms")
    Q = run_gpu(T, w.instance, w.beta, w.p_q, mcs=w.mcs_per_swap, rounds=200, seed=5, f_target=f_gs)
    assert np.array_equal(P.states(), Q.states())
    assert all(np.array_equal(a, b) for a, b in zip(P.energies(), Q.energies()))
    assert P.query()["first_hit_sweep"] == Q.query()["first_hit_sweep"]


def test_batch_mixes_constraint_kinds(T):
    """Copy-edge and general-constraint problems in one batch, each equal to
    its own oracle run."""
    w = wishart_small()
    members = [
        ("wishart-N12", w.instance, w.beta, w.p_q, 5, 11),
        ("wishart-N12 terms", terms_from_copies(w.instance), w.beta, w.p_q, 5, 11),
        ("knapsack", slack_knapsack(6, seed=0), np.array([0.1, 0.4]), np.array([512, 2048], np.int32), 2, 3),
        ("coloring", planted_coloring(40, 3, degree=4, seed=1).instance, np.geomspace(0.3, 3, 4),
         np.array([0, 4096], np.int32), 3, 8),
    ]
    rounds = 20
    probs = []
    for name, inst, beta, p_q, mcs, seed in members:
        cfg = T.RunConfig(beta, p_q, mcs_per_swap=mcs, seed=seed, trace_cap=rounds)
        probs.append(T.Problem(T.Instance.from_synth(inst), cfg))
    B = T.Batch(4)
    B.set_members(probs)
    B.run(rounds)
    for (name, inst, beta, p_q, mcs, seed), P in zip(members, probs):
        _say(f"[constraints] batch member {name}")
        o = O.run(inst, beta, p_q, mcs_per_swap=mcs, n_rounds=rounds, seed=seed, trace=True)
        assert_same(o, P, name)


def test_coloring_workload_sub_grid_bit_exact(T):
    """The benchmark's colouring instance (16,000 spins) on a 4x4 corner of
    its grid for 2 rounds of 50 sweeps."""
    w = coloring_workload()
    both(T, w.instance, w.beta[-4:], w.p_q[-4:], mcs=w.mcs_per_swap, rounds=2, seed=0,
         f_target=w.f_target_q, label="coloring workload 4x4 corner")


def test_coloring_workload_full_grid_invariants(T):
    """The full 32x16 grid in the benchmark's launch configuration: every
    spin stays +-1, the f and g the library carries equal the oracle's
    energy of the states it returns, the grid permutation stays a
    permutation, swap counters are consistent, and any best state reported
    is feasible with the reported f."""
    w = coloring_workload()
    inst = T.Instance.from_synth(w.instance)
    cfg = T.RunConfig(w.beta, w.p_q, mcs_per_swap=w.mcs_per_swap, seed=1, f_target=w.f_target_q)
    P = T.Problem(inst, cfg)
    _say("[constraints] coloring workload full grid, 6 rounds")
    P.run(6)
    st = P.states()
    assert set(np.unique(st)) <= {-1, 1}
    f, g = P.energies()
    for p in range(0, st.shape[0], 37):
        assert (f[p], g[p]) == O.energy(w.instance, st[p])
    perm = P.perm()
    assert sorted(perm.tolist()) == list(range(st.shape[0]))
    pa, pc, ba, bc = P.counters()
    assert np.all(pc <= pa) and np.all(bc <= ba)
    q = P.query()
    if q["best_f_q"] < 2**62:
        s, bf, _ = P.best()
        assert O.energy(w.instance, s) == (bf, 0)


def test_autotuned_coloring_matches_oracle(T):
    pc = planted_coloring(200, 4, degree=5, seed=3)
    beta = np.geomspace(0.3, 4.0, 8)
    p_q = np.linspace(0, 8192, 4).astype(np.int32)
    P = T.Problem(T.Instance.from_synth(pc.instance),
                  T.RunConfig(beta, p_q, mcs_per_swap=5, seed=2, f_target=pc.f_target_q, trace_cap=30))
    rep = P.autotune(3)
    _say(f"[constraints] autotune coloring-200x4: driver {rep['driver']} block {rep['block']}")
    P.run(30)
    o = O.run(pc.instance, beta, p_q, mcs_per_swap=5, n_rounds=30, seed=2, f_target=pc.f_target_q, trace=True)
    assert_same(o, P, "tuned coloring")


def test_degenerate_constraints(T):
    """No terms (g = 0: plain PT on every column, every P-swap accepted) and a
    term without spins (g = d^2 everywhere: nothing is ever feasible), each
    bit-exact against the oracle."""
    from synth.constrained import with_terms
    base = slack_knapsack(5, seed=2)
    beta = np.array([0.1, 0.3])
    p_q = np.array([512, 2048], np.int32)
    free = with_terms(base, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32),
                      np.zeros(0, np.int32))
    o, P = both(T, free, beta, p_q, mcs=2, rounds=24, seed=3, label="no terms")
    pa, pc, _, _ = P.counters()
    assert np.all(o["g"] == 0) and np.array_equal(pa, pc) and pa.sum() > 0
    const = with_terms(base, np.array([0, 0], np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32),
                       np.array([3], np.int32))
    o, P = both(T, const, beta, p_q, mcs=2, rounds=24, seed=3, label="constant term")
    assert np.all(o["g"] == 9) and P.query()["best_f_q"] == 2**63 - 1


def test_large_constraint_field_without_penalty(T):
    """A term with coefficients of 5000 (pair weights of 2.5e7, above the
    packed layout's 24-bit products) on a ladder whose penalties are all 0:
    g does not steer the sampling but is still tracked exactly, so the
    library must keep such a problem off the packed layout and bound each
    lane's per-phase g sums by the constraint field."""
    from synth.constrained import with_terms
    base = slack_knapsack(5, seed=2)
    n = base.n
    idx = np.arange(n, dtype=np.int32)
    coef = np.full(n, 5000, np.int32)
    inst = with_terms(base, np.array([0, n], np.int32), idx, coef, np.array([7], np.int32))
    assert T.Instance.from_synth(inst).info()["narrow"] == 1  # problem rows would fit
    o, P = both(T, inst, np.array([0.05, 0.2]), np.array([0, 0], np.int32), mcs=3, rounds=12, seed=6,
                label="large constraint field, P = 0")
    assert np.abs(o["g"]).max() > (1 << 23)


@pytest.mark.parametrize("driver", ["0", "1"])
def test_constraint_beyond_32_bits(T, driver):
    """One term over 30 spins with constant 65539, so g = (sum s + 65539)^2
    straddles 2^32, and a field that pushes the P_q = 1 column above 2^32
    and the P_q = 2 column below it: every P-swap (Eq. 2) and beta-swap
    (Eq. 3, E = f + P g) compares g values on both sides of 2^32.  Both
    drivers must carry g at full width between swap partners and match the
    oracle bit for bit."""
    from synth.constrained import with_terms
    from synth.instances import Instance
    n = 30
    base = Instance(n=n, row_ptr=np.zeros(n + 1, np.int32), col=np.zeros(0, np.int32),
                    J_q=np.zeros(0, np.int32), b_q=np.full(n, 196608, np.int32),
                    copy_a=np.zeros(0, np.int32), copy_b=np.zeros(0, np.int32),
                    color=np.zeros(n, np.int32), logical_of=np.arange(n, dtype=np.int32), N=n)
    inst = with_terms(base, np.array([0, n], np.int32), np.arange(n, dtype=np.int32),
                      np.ones(n, np.int32), np.array([65536 + 3], np.int32))
    beta = np.array([0.002, 0.004, 0.008])
    p_q = np.array([1, 2], np.int32)
    o, P = _with_env("TDPT_PERSISTENT", driver, lambda: both(
        T, inst, beta, p_q, mcs=1, rounds=200, seed=3, label=f"g beyond 2^32, driver {driver}"))
    assert P.query()["driver"] == int(driver)
    tg = o["trace_g"]
    assert (tg >= 2**32).any() and (tg < 2**32).any()
