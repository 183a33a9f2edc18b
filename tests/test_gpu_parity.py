"""GPU path vs CPU oracle, bit-exact, through the C ABI.

Every case runs the same seeded inputs through the oracle and through the
gfx950 library and compares every output element by element: final spins
of every grid position, f and g per position, swap attempt/accept counters
of every pair, the bottom-right trace, best state, best energy and
first-hit sweep.  Integers are compared exactly; the two double-precision
decisions (heat bath, swap) use the same expression on both sides, so the
trajectories are identical.
"""
from __future__ import annotations

import dataclasses
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from synth.configs import batched_member, wishart_n200, wishart_small
from synth.instances import build_instance, instance_from_logical, q12, random_spins
from tests.tiny import tiny_instance

pytestmark = pytest.mark.gpu

INT64_MAX = 2**63 - 1


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2506_14781_amd as T
    return T


def run_gpu(T, inst, beta, p_q, *, mcs, rounds, seed, s0=None, f_target=None, flags=0,
            trace=True, split=None):
    I = T.Instance.from_synth(inst)
    cfg = T.RunConfig(beta, p_q, mcs_per_swap=mcs, seed=seed, s0=s0, f_target=f_target,
                      flags=flags, trace_cap=rounds if trace else 0)
    P = T.Problem(I, cfg)
    if split is None:
        P.run(rounds)
    else:
        for part in split:
            P.run(part)
    return P


def assert_same(o, P, label):
    st = P.states()
    if not np.array_equal(st, o["states"]):
        bad = np.argwhere(st != o["states"])
        p, v = bad[0]
        raise AssertionError(f"{label}: states differ at {len(bad)} spins; first: position {p}, "
                             f"spin {v} (gpu {st[p, v]}, oracle {o['states'][p, v]})")
    f, g = P.energies()
    assert np.array_equal(f, o["f"]), f"{label}: f differs"
    assert np.array_equal(g, o["g"]), f"{label}: g differs"
    pa, pc, ba, bc = P.counters()
    assert np.array_equal(pa, o["p_att"]) and np.array_equal(pc, o["p_acc"]), f"{label}: P counters"
    assert np.array_equal(ba, o["b_att"]) and np.array_equal(bc, o["b_acc"]), f"{label}: beta counters"
    q = P.query()
    assert q["first_hit_sweep"] == o["first_hit"], label
    assert q["best_f_q"] == o["best_f"], label
    assert q["best_sweep"] == o["best_sweep"], label
    if o["best_f"] != INT64_MAX:
        s, bf, bw = P.best()
        assert np.array_equal(s, o["best_state"]), f"{label}: best state"
    if len(o["trace_f"]):
        tf, tg = P.trace()
        assert np.array_equal(tf, o["trace_f"]) and np.array_equal(tg, o["trace_g"]), label


def both(T, inst, beta, p_q, *, mcs, rounds, seed, label, **kw):
    _say(f"[parity] {label}: n={inst.n} grid={len(beta)}x{len(p_q)} mcs={mcs} rounds={rounds} seed={seed}")
    o = O.run(inst, beta, p_q, mcs_per_swap=mcs, n_rounds=rounds, seed=seed,
              s0=kw.get("s0"), f_target=kw.get("f_target"), flags=kw.get("flags", 0),
              trace=True)
    P = run_gpu(T, inst, beta, p_q, mcs=mcs, rounds=rounds, seed=seed, **kw)
    assert_same(o, P, label)
    return o, P


def test_initial_energies_match(T):
    w = wishart_small()
    rng = np.random.default_rng(0)
    s0 = random_spins(rng, w.replicas * w.instance.n)
    both(T, w.instance, w.beta, w.p_q, mcs=50, rounds=0, seed=0, s0=s0, label="round0-s0")
    both(T, w.instance, w.beta, w.p_q, mcs=50, rounds=0, seed=9, label="round0-philox-s0")


def test_small_wishart_full_run(T):
    """N=12 planted Wishart, 8x4 grid, 1e4 sweeps: the whole run is bit-exact,
    including the planted ground-state hit."""
    w = wishart_small()
    inst = w.instance
    f_gs = O.energy(inst, inst.physical_state(inst.planted))[0]
    for seed in (0, 5):
        o, P = both(T, inst, w.beta, w.p_q, mcs=w.mcs_per_swap, rounds=w.rounds, seed=seed,
                    f_target=f_gs, label=f"wishart-N12 seed {seed}")
    assert o["first_hit"] > 0  # seed 5 reaches the planted ground state


def test_packed_per_round_single_problem(T):
    """Small bipartite replicas with long rounds run per-round launches by
    default: one spin per lane (a lone problem is latency-bound), each
    lane's structure held in registers for the round; with TDPT_SPIN=0 one
    quad per lane, four N=12 replicas per wave.  Both are bit-exact against
    the oracle, as is the persistent driver asked for instead.  The 10-spin
    instance (fields) and an instance with colour classes of 1 and 3 quads
    (lanes holding spins of both classes, one or none) run both shapes."""
    w = wishart_small()
    o, P = both(T, w.instance, w.beta, w.p_q, mcs=20, rounds=12, seed=3, label="spin lanes N12")
    q = P.query()
    assert (q["driver"], q["spin"], q["slots"]) == (0, 1, 1)
    Q = _with_env("TDPT_SPIN", "0", lambda: run_gpu(T, w.instance, w.beta, w.p_q, mcs=20, rounds=12, seed=3))
    assert (Q.query()["driver"], Q.query()["spin"], Q.query()["slots"]) == (0, 0, 4)
    assert_same(o, Q, "quad lanes N12")
    Q = _with_env("TDPT_PERSISTENT", "1", lambda: run_gpu(T, w.instance, w.beta, w.p_q, mcs=20, rounds=12, seed=3))
    assert Q.query()["driver"] == 1
    assert_same(o, Q, "N12 persistent")
    inst = tiny_instance()
    beta = np.geomspace(0.3, 3.0, 5)
    p_q = q12(np.linspace(0.5, 3.0, 7))
    o, P = _with_env("TDPT_PERSISTENT", "0", lambda: both(T, inst, beta, p_q, mcs=16, rounds=10, seed=4,
                                                          label="spin lanes tiny 5x7"))
    assert (P.query()["driver"], P.query()["spin"], P.query()["slots"]) == (0, 1, 8)
    Q = _with_env("TDPT_PERSISTENT", "0", lambda: _with_env("TDPT_SPIN", "0", lambda: run_gpu(
        T, inst, beta, p_q, mcs=16, rounds=10, seed=4)))
    assert (Q.query()["spin"], Q.query()["slots"]) == (0, 16)
    assert_same(o, Q, "quad lanes tiny 5x7")
    # classes of unequal size (1 and 3 quads, the last ones partly dead)
    inst = _unequal_classes()
    beta, p_q = np.geomspace(0.3, 3.0, 4), q12([0.0, 1.0, 2.0])
    o, P = both(T, inst, beta, p_q, mcs=20, rounds=12, seed=5, label="spin lanes unequal classes")
    assert (P.query()["driver"], P.query()["spin"], P.query()["slots"]) == (0, 1, 4)
    Q = _with_env("TDPT_SPIN", "0", lambda: run_gpu(T, inst, beta, p_q, mcs=20, rounds=12, seed=5))
    assert (Q.query()["driver"], Q.query()["spin"], Q.query()["slots"]) == (0, 0, 16)
    assert_same(o, Q, "quad lanes unequal classes")
    # three and four colour classes held in registers at one spin per lane:
    # a ladder-ordered N=6 instance (18 spins) and the three-copy N=16
    # J-column member (48 spins, ELL width 6, its own 16 x 8 grid)
    inst = build_instance(6, 0.5, 1, degree_cap=3, order="ascending")
    assert inst.n_colors == 3
    o, P = both(T, inst, np.geomspace(0.3, 3.0, 3), q12([0.0, 1.0, 2.0]), mcs=20, rounds=10, seed=6,
                label="spin lanes, 3 classes")
    assert (P.query()["driver"], P.query()["spin"], P.query()["slots"]) == (0, 1, 8)
    from synth.configs import jcolumn_member
    jc = jcolumn_member(16, 20000)
    o, P = both(T, jc.instance, jc.beta, jc.p_q, mcs=20, rounds=8, seed=7, label="spin lanes, 4 classes")
    assert (P.query()["driver"], P.query()["spin"], P.query()["slots"]) == (0, 1, 4)


def _unequal_classes():
    """Bipartite instance without fields: 3 centres (colour 0) with 3 leaves
    each (colour 1), two of the leaves copies of centres; Q12 couplings."""
    from synth.instances import Instance
    rng = np.random.default_rng(21)
    n = 12
    edges = [(c, 3 + 3 * c + k) for c in range(3) for k in range(3)]
    J = np.zeros((n, n), np.int32)
    for a, b in edges:
        J[a, b] = J[b, a] = int(rng.integers(-3000, 3000))
    row_ptr = np.zeros(n + 1, np.int32)
    cols, vals = [], []
    for i in range(n):
        nb = np.flatnonzero(J[i])
        cols += nb.tolist()
        vals += J[i, nb].tolist()
        row_ptr[i + 1] = len(cols)
    copy_a, copy_b = np.array([0, 1], np.int32), np.array([6, 9], np.int32)
    logical_of = np.array([0, 1, 2, 3, 4, 5, 0, 6, 7, 1, 8, 9], np.int32)
    color = np.array([0, 0, 0] + [1] * 9, np.int32)
    return Instance(n=n, row_ptr=row_ptr, col=np.array(cols, np.int32), J_q=np.array(vals, np.int32),
                    b_q=np.zeros(n, np.int32), copy_a=copy_a, copy_b=copy_b, color=color,
                    logical_of=logical_of, N=10)


@pytest.mark.parametrize("I,J,mcs", [(1, 1, 3), (1, 4, 2), (4, 1, 2), (2, 2, 1), (3, 5, 2)])
def test_tiny_grids(T, I, J, mcs):
    inst = tiny_instance()
    beta = np.geomspace(0.3, 3.0, I)
    p_q = q12(np.linspace(0.5, 3.0, J))
    both(T, inst, beta, p_q, mcs=mcs, rounds=40, seed=11, label=f"tiny {I}x{J}")


def test_no_pswap_flag(T):
    w = wishart_small()
    both(T, w.instance, w.beta, np.full(4, 8192, np.int32), mcs=10, rounds=30, seed=2,
         flags=O.NO_PSWAP, label="J-column PT")


def test_caller_initial_state(T):
    w = wishart_small()
    rng = np.random.default_rng(4)
    s0 = random_spins(rng, w.replicas * w.instance.n)
    both(T, w.instance, w.beta, w.p_q, mcs=7, rounds=25, seed=3, s0=s0, label="given s0")


def test_wide_layout(T):
    """Couplings beyond 16 bits take the 32-bit structure layout."""
    rng = np.random.default_rng(8)
    A = np.triu(rng.normal(0, 10.0, size=(6, 6)), 1)
    Jq = q12(A + A.T)
    np.fill_diagonal(Jq, 0)
    inst = instance_from_logical(Jq, degree_cap=3)
    assert np.abs(inst.J_q).max() > 32767
    T_inst = T.Instance.from_synth(inst)
    assert T_inst.info()["narrow"] == 0
    both(T, inst, np.array([0.001, 0.003]), q12([0.0, 40.0]), mcs=2, rounds=30, seed=1,
         label="wide")


@pytest.mark.parametrize("N,driver", [(48, "1"), (64, "0"), (64, "1")])
def test_streamed_structure_rows(T, N, driver):
    """More than 8 problem neighbours per spin (three copies per node: 16 at
    N = 48, 24 at N = 64): structure rows streamed in chunks."""
    from synth.configs import jcolumn_member
    w = jcolumn_member(N, 20000)
    o, P = _with_env("TDPT_PERSISTENT", driver, lambda: both(
        T, w.instance, w.beta[:6], w.p_q[:4], mcs=3, rounds=8, seed=2,
        label=f"three copies N={N} driver {driver}"))
    assert P.query()["driver"] == int(driver)


@pytest.mark.parametrize("N,driver", [(150, "0"), (200, "1")])
def test_rows_wider_than_48(T, N, driver):
    """Three copies per node at N = 150 and 200 (50 and 67 problem
    neighbours per spin, ELL widths 56 and 72): the run-time-width sweep,
    bit-exact against the oracle."""
    from synth.configs import jcolumn_member
    w = jcolumn_member(N, 20000)
    assert T.Instance.from_synth(w.instance).info()["max_degree"] in (50, 67)
    o, P = _with_env("TDPT_PERSISTENT", driver, lambda: both(
        T, w.instance, w.beta[:4], w.p_q[:3], mcs=3, rounds=6, seed=5,
        label=f"three copies N={N} driver {driver}"))
    assert P.query()["driver"] == int(driver)


def test_streamed_rows_wide_layout(T):
    """Couplings beyond int16 (32-bit structure) with 12+ neighbours."""
    rng = np.random.default_rng(21)
    A = np.triu(rng.normal(0, 12.0, size=(26, 26)), 1)
    Jq = q12(A + A.T)
    np.fill_diagonal(Jq, 0)
    inst = instance_from_logical(Jq, copies=2)
    assert np.abs(inst.J_q).max() > 32767 and np.diff(inst.row_ptr).max() > 8
    both(T, inst, np.array([0.0005, 0.002, 0.004]), q12([0.0, 30.0]), mcs=2, rounds=6, seed=4,
         label="wide, streamed")


def test_chains_only_no_couplings(T):
    inst = instance_from_logical(np.zeros((4, 4), np.int32), copies=3)
    both(T, inst, np.array([0.5, 1.5]), q12([0.0, 1.0]), mcs=3, rounds=20, seed=6,
         label="chains only")


def test_ragged_colour_classes(T):
    """Colour classes whose sizes are not multiples of 4 leave dead lanes in
    the last quad of each class."""
    inst = build_instance(23, 0.75, 4, degree_cap=5, order="ascending")
    sizes = np.bincount(inst.color)
    assert inst.n_colors == 5
    assert np.any(sizes % 4 != 0)
    both(T, inst, np.geomspace(0.2, 4, 3), q12([0, 1, 2.5]), mcs=4, rounds=20, seed=7,
         label="ragged classes")


def test_split_runs(T):
    """run(13) + run(0) + run(27) is the same trajectory as 40 rounds at once."""
    w = wishart_small()
    o = O.run(w.instance, w.beta, w.p_q, mcs_per_swap=5, n_rounds=40, seed=12, trace=True)
    P = run_gpu(T, w.instance, w.beta, w.p_q, mcs=5, rounds=40, seed=12, split=[13, 0, 27])
    assert_same(o, P, "split 13+0+27")


def test_checkpoint_rejects_other_shape(T):
    w = wishart_small()
    A = run_gpu(T, w.instance, w.beta, w.p_q, mcs=5, rounds=3, seed=12)
    other = run_gpu(T, w.instance, w.beta[:4], w.p_q, mcs=5, rounds=0, seed=12)
    with pytest.raises(T.TdptError):
        other.load(A.save())


def test_checkpoint_resume_is_bit_exact(T):
    w = wishart_small()
    I = T.Instance.from_synth(w.instance)
    cfg = T.RunConfig(w.beta, w.p_q, mcs_per_swap=5, seed=21, trace_cap=40)
    straight = T.Problem(I, cfg)
    straight.run(40)
    first = T.Problem(I, cfg)
    first.run(17)
    blob = first.save()
    resumed = T.Problem(I, cfg)
    resumed.load(blob)
    resumed.run(23)
    assert np.array_equal(straight.states(), resumed.states())
    assert all(np.array_equal(a, b) for a, b in zip(straight.energies(), resumed.energies()))
    assert all(np.array_equal(a, b) for a, b in zip(straight.counters(), resumed.counters()))
    assert all(np.array_equal(a, b) for a, b in zip(straight.trace(), resumed.trace()))
    assert straight.query() == resumed.query()


def _with_env(key, value, fn):
    old = os.environ.get(key)
    os.environ[key] = value
    try:
        return fn()
    finally:
        if old is None:
            del os.environ[key]
        else:
            os.environ[key] = old


def test_n200_prefix_bit_exact(T):
    """N=200 planted Wishart (6800 spins), 32x16 grid, a swap every sweep:
    the first rounds are bit-exact in the launch configuration the benchmark
    times (the persistent driver)."""
    w = wishart_n200()
    o, P = both(T, w.instance, w.beta, w.p_q, mcs=1, rounds=40, seed=1,
                label="wishart-N200 prefix")
    assert P.query()["driver"] == 1


def test_n200_prefix_per_round_driver(T):
    """The same prefix through the one-launch-pair-per-round driver."""
    w = wishart_n200()
    o, P = _with_env("TDPT_PERSISTENT", "0", lambda: both(
        T, w.instance, w.beta, w.p_q, mcs=1, rounds=12, seed=1, label="wishart-N200 per-round"))
    assert P.query()["driver"] == 0


def test_drivers_agree_on_the_small_workload(T):
    w = wishart_small()
    a = run_gpu(T, w.instance, w.beta, w.p_q, mcs=5, rounds=60, seed=8)
    b = _with_env("TDPT_PERSISTENT", "0", lambda: run_gpu(
        T, w.instance, w.beta, w.p_q, mcs=5, rounds=60, seed=8))
    assert a.query()["driver"] == 1 and b.query()["driver"] == 0
    assert np.array_equal(a.states(), b.states())
    assert all(np.array_equal(x, y) for x, y in zip(a.counters(), b.counters()))
    assert all(np.array_equal(x, y) for x, y in zip(a.trace(), b.trace()))
    qa, qb = a.query(), b.query()
    for k in ("driver", "slots", "spin"):  # the launch shape; results must not depend on it
        qa.pop(k), qb.pop(k)
    assert qa == qb
    assert np.array_equal(a.best()[0], b.best()[0])


@pytest.mark.parametrize("driver,block", [("0", "64"), ("0", "256"), ("0", "1024"),
                                          ("1", "64"), ("1", "192"), ("1", "512")])
def test_block_size_does_not_change_results(T, driver, block):
    """Threads per workgroup (so quads per lane) is a launch choice only."""
    w = wishart_n200()

    def go():
        return _with_env("TDPT_BLOCK", block, lambda: both(
            T, w.instance, w.beta[:8], w.p_q[:4], mcs=2, rounds=6, seed=3,
            label=f"driver {driver} block {block}"))
    o, P = _with_env("TDPT_PERSISTENT", driver, go)
    assert P.query()["driver"] == int(driver)


def test_batched_family_member(T):
    w = batched_member(64, 0.5, 3)
    both(T, w.instance, w.beta, w.p_q, mcs=w.mcs_per_swap, rounds=3, seed=2,
         label="batched member N=64")


def test_n200_long_run_invariants(T):
    """At full size over many rounds: every spin stays +-1, the energies the
    library carries equal those of the states it returns (no drift in the
    incremental bookkeeping), the position permutation stays a permutation
    and swap counters add up."""
    w = wishart_n200()
    _say("[invariants] wishart-N200 2000 rounds")
    P = run_gpu(T, w.instance, w.beta, w.p_q, mcs=1, rounds=2000, seed=4, trace=False)
    st = P.states()
    assert np.all(np.abs(st) == 1)
    f, g = P.energies()
    rng = np.random.default_rng(0)
    for pos in rng.choice(w.replicas, size=24, replace=False):
        assert O.energy(w.instance, st[pos]) == (f[pos], g[pos])
    perm = P.perm()
    assert np.array_equal(np.sort(perm), np.arange(w.replicas))
    pa, pc, ba, bc = P.counters()
    assert pa.sum() + ba.sum() == sum(
        (w.n_beta * ((w.n_p - (r % 2 == 0)) // 2)) if ((r - 1) // 2) % 2 == 0
        else (w.n_p * ((w.n_beta - (r % 2 == 0)) // 2)) for r in range(1, 2001))
    assert np.all(pc <= pa) and np.all(bc <= ba)


# ------------------------------------------------------ bit-packed layout

def _bits_form(T, inst, cfg, form, fn):
    """fn() with the bit-packed layout forced in the given form ("pair": two
    replicas per word, 16-bit coupling sums; "plain": one replica per word),
    after checking that the library reports that form for the problem."""
    def go():
        lay = T.Instance.from_synth(inst).layout(cfg)
        assert lay["bits"] == 1 and lay["pair16"] == (1 if form == "pair" else 0)
        return fn()
    return _with_env("TDPT_LAYOUT", "bits",
                     lambda: _with_env("TDPT_PAIR16", "1" if form == "pair" else "0", go))


@pytest.mark.parametrize("form", ["pair", "plain"])
@pytest.mark.parametrize("I,J,mcs", [(8, 4, 5), (3, 5, 2), (1, 1, 3)])
def test_bit_packed_layout_small(T, I, J, mcs, form):
    """The bit-packed layout (4 replicas per workgroup as bits), forced on
    small instances in both its forms: grids whose replica count is not a
    multiple of 4 (a pair word then holds one live replica), the instance
    with fields, the N=12 workload; 2 sweeps per round follow f and g
    update by update, 3 and 5 recompute them at the round's end."""
    for inst, name in [(tiny_instance(), "tiny+fields"), (wishart_small().instance, "wishart-N12")]:
        beta = np.geomspace(0.3, 3.0, I)
        p_q = q12(np.linspace(0.5, 3.0, J))
        _bits_form(T, inst, T.RunConfig(beta, p_q, mcs_per_swap=mcs, seed=13), form, lambda: both(
            T, inst, beta, p_q, mcs=mcs, rounds=30, seed=13, label=f"bits {form} {name} {I}x{J}"))


def test_bit_packed_large_couplings_take_the_plain_form(T):
    """Couplings whose row sums reach 2^14 cannot be summed in 16-bit halves:
    the library keeps such bit-packed problems in the plain form by itself,
    and the results equal the oracle's."""
    base = tiny_instance()
    inst = dataclasses.replace(base, J_q=np.asarray(base.J_q, dtype=np.int32) * 4)
    beta, p_q = np.geomspace(0.02, 0.3, 3), q12(np.linspace(0.5, 3.0, 2))
    cfg = T.RunConfig(beta, p_q, mcs_per_swap=5, seed=3)

    def go():
        assert T.Instance.from_synth(inst).layout(cfg)["pair16"] == 0
        both(T, inst, beta, p_q, mcs=5, rounds=20, seed=3, label="bits large couplings")
    _with_env("TDPT_LAYOUT", "bits", go)


def test_bit_packed_ragged_and_batched(T):
    inst = build_instance(23, 0.75, 4, degree_cap=5, order="ascending")
    _with_env("TDPT_LAYOUT", "bits", lambda: both(
        T, inst, np.geomspace(0.2, 4, 3), q12([0, 1, 2.5]), mcs=4, rounds=20, seed=7,
        label="bits ragged classes"))
    w = wishart_small()
    o = O.run(w.instance, w.beta, w.p_q, mcs_per_swap=5, n_rounds=12, seed=2, trace=True)
    P = _with_env("TDPT_LAYOUT", "bits", lambda: run_gpu(
        T, w.instance, w.beta, w.p_q, mcs=5, rounds=0, seed=2, trace=False))
    B = T.Batch(2)
    B.set_members([P])
    B.run(12)
    st = P.states()
    assert np.array_equal(st, o["states"])
    # one member in each form (a group, and a kernel, of its own each)
    o2 = O.run(w.instance, w.beta, w.p_q, mcs_per_swap=5, n_rounds=12, seed=9, trace=True)
    Pa = _with_env("TDPT_LAYOUT", "bits", lambda: _with_env("TDPT_PAIR16", "0", lambda: run_gpu(
        T, w.instance, w.beta, w.p_q, mcs=5, rounds=0, seed=2, trace=False)))
    Pb = _with_env("TDPT_LAYOUT", "bits", lambda: run_gpu(
        T, w.instance, w.beta, w.p_q, mcs=5, rounds=0, seed=9, trace=False))
    B2 = T.Batch(2)
    B2.set_members([Pa, Pb])
    B2.run(12)
    assert np.array_equal(Pa.states(), o["states"])
    assert np.array_equal(Pb.states(), o2["states"])
    for oo, PP in ((o, Pa), (o2, Pb)):
        f, g = PP.energies()
        assert np.array_equal(f, oo["f"]) and np.array_equal(g, oo["g"])


@pytest.mark.parametrize("form", ["pair", "plain"])
def test_n1000_instance_bit_exact_on_a_sub_grid(T, form):
    """The N=1000 planted-Wishart instance (250,000 spins per replica, bit-packed
    layout chosen automatically, in its pair form unless TDPT_PAIR16=0) on a
    2x2 sub-grid: one round of 50 sweeps is bit-exact against the oracle."""
    from synth.configs import wishart_n1000
    w = wishart_n1000()
    P0 = T.Instance.from_synth(w.instance)
    assert P0.info()["n"] == 250000
    beta = w.beta[[0, -1]]
    p_q = w.p_q[[0, -1]]

    def go():
        lay = P0.layout(T.RunConfig(beta, p_q, mcs_per_swap=50, seed=4))
        assert lay["bits"] == 1 and lay["pair16"] == (1 if form == "pair" else 0)
        both(T, w.instance, beta, p_q, mcs=50, rounds=1, seed=4, label=f"wishart-N1000 2x2 {form}")
    _with_env("TDPT_PAIR16", "1" if form == "pair" else "0", go)


def test_caller_initial_state_in_several_uploads(T):
    """A given initial state larger than one upload chunk (80 replicas of
    250,000 spins, about 20 MB) arrives whole: the states read back equal
    it, and the initial energies of replicas in the first and the last chunk
    equal the oracle's."""
    from synth.configs import wishart_n1000
    w = wishart_n1000()
    beta = np.geomspace(0.1, 3.0, 4)
    p_q = np.linspace(0, 8192, 20).astype(np.int32)
    R = len(beta) * len(p_q)
    s0 = random_spins(np.random.default_rng(12), R * w.instance.n).reshape(R, w.instance.n)
    _say("[s0] wishart-N1000 4x20 given state, 0 rounds")
    P = T.Problem(T.Instance.from_synth(w.instance), T.RunConfig(beta, p_q, mcs_per_swap=1, seed=0, s0=s0))
    assert np.array_equal(P.states(), s0)
    f, g = P.energies()
    for r in (0, 66, 67, R - 1):
        assert O.energy(w.instance, s0[r]) == (f[r], g[r])


def test_n1000_full_grid_invariants(T):
    """Full 64x32 grid of the N=1000 instance, two rounds of 50 sweeps: every
    spin +-1, f and g of sampled positions equal their recomputation, the
    permutation is a permutation."""
    from synth.configs import wishart_n1000
    w = wishart_n1000()
    _say("[invariants] wishart-N1000 64x32, 2 rounds x 50 sweeps")
    P = run_gpu(T, w.instance, w.beta, w.p_q, mcs=50, rounds=2, seed=0, trace=False)
    assert P.query()["driver"] == 0
    st = P.states()
    assert np.all(np.abs(st) == 1)
    f, g = P.energies()
    rng = np.random.default_rng(1)
    for pos in rng.choice(w.replicas, size=6, replace=False):
        assert O.energy(w.instance, st[pos]) == (f[pos], g[pos])
    assert np.array_equal(np.sort(P.perm()), np.arange(w.replicas))


# ----------------------------------------------------------------- autotuner

def test_autotune_leaves_results_unchanged(T):
    """The autotuner times launch shapes on the problem itself and restores
    its state: the state right after tuning equals the state before, and a
    tuned run is bit-identical to an untuned one (and to the oracle)."""
    w = wishart_small()

    def make():
        P = T.Problem(T.Instance.from_synth(w.instance),
                      T.RunConfig(w.beta, w.p_q, mcs_per_swap=5, seed=8, trace_cap=70))
        P.run(30)
        return P
    a, b = make(), make()
    before = (b.states(), b.energies(), b.query())
    rep = b.autotune(3)
    _say(f"[parity] autotune N12: {rep['driver']} {rep['block']} from {len(rep['trials'])} trials")
    assert len(rep["trials"]) >= 2
    assert (rep["driver"], rep["block"], rep["slots"]) in {(d, k, r) for d, k, r, _ in rep["trials"]}
    assert any(r > 1 for _, _, r, _ in rep["trials"])  # packed shapes are among the candidates
    assert np.array_equal(before[0], b.states())
    assert all(np.array_equal(x, y) for x, y in zip(before[1], b.energies()))
    assert before[2]["rounds_done"] == b.query()["rounds_done"]
    a.run(40)
    b.run(40)
    assert b.query()["driver"] == rep["driver"]
    assert np.array_equal(a.states(), b.states())
    assert all(np.array_equal(x, y) for x, y in zip(a.counters(), b.counters()))
    o = O.run(w.instance, w.beta, w.p_q, mcs_per_swap=5, n_rounds=70, seed=8, trace=True)
    assert_same(o, b, "tuned N12")


def test_autotune_n200_and_bits(T):
    """Tuning the N=200 workload and a forced bit-packed problem picks an
    admissible shape and keeps results bit-exact."""
    w = wishart_n200()
    P = T.Problem(T.Instance.from_synth(w.instance),
                  T.RunConfig(w.beta, w.p_q, mcs_per_swap=1, seed=1, trace_cap=40))
    rep = P.autotune(20)
    _say(f"[parity] autotune N200: {rep}")
    assert rep["block"] % 64 == 0 and 64 <= rep["block"] <= 1024
    P.run(40)
    o = O.run(w.instance, w.beta, w.p_q, mcs_per_swap=1, n_rounds=40, seed=1, trace=True)
    assert_same(o, P, "tuned N200")

    def bits():
        ws = wishart_small()
        Q = T.Problem(T.Instance.from_synth(ws.instance),
                      T.RunConfig(ws.beta, ws.p_q, mcs_per_swap=5, seed=2, trace_cap=20))
        r = Q.autotune(2)
        assert all(d == 0 and k <= 512 and n == 1 for d, k, n, _ in r["trials"])
        Q.run(20)
        return Q
    Q = _with_env("TDPT_LAYOUT", "bits", bits)
    ws = wishart_small()
    o = O.run(ws.instance, ws.beta, ws.p_q, mcs_per_swap=5, n_rounds=20, seed=2, trace=True)
    assert_same(o, Q, "tuned bits")


@pytest.mark.parametrize("form", ["pair", "plain"])
@pytest.mark.parametrize("mcs,block", [(5, "1024"), (5, "256"), (2, "1024")])
def test_bit_packed_block_sizes(T, mcs, block, form):
    """Bit-packed replicas at 1024 threads (allowed when f and g are
    recomputed at the round's end, from 4 sweeps per round), at 256, and
    capped at 768 when they follow every update (2 sweeps per round), in
    both forms: the same results as the oracle."""
    w = batched_member(100, 0.8, 5)

    def go():
        return _with_env("TDPT_BLOCK", block, lambda: both(
            T, w.instance, w.beta[:4], w.p_q[:4], mcs=mcs, rounds=5, seed=7,
            label=f"bits {form} mcs {mcs} block {block}"))
    _bits_form(T, w.instance, T.RunConfig(w.beta[:4], w.p_q[:4], mcs_per_swap=mcs, seed=7), form, go)


@pytest.mark.parametrize("order", ["7,3", "31,5", "1,17"])
def test_persistent_slot_order_does_not_matter(T, order):
    """The persistent driver's exchange must not depend on which workgroup
    (so which compute unit and XCD) serves which replica slot: with the
    slots assigned to workgroups in another order the run equals the
    oracle, for one problem and inside a persistent batch."""
    w = wishart_small()
    f_gs = O.energy(w.instance, w.instance.physical_state(w.instance.planted))[0]

    def go():
        o, P = both(T, w.instance, w.beta, w.p_q, mcs=5, rounds=60, seed=8, f_target=f_gs,
                    label=f"slot order {order}")
        assert P.query()["driver"] == 1
        m = batched_member(64, 0.8, 3)
        cfgs = [T.RunConfig(w.beta, w.p_q, mcs_per_swap=5, seed=9, trace_cap=30),
                T.RunConfig(m.beta[:8], m.p_q[:4], mcs_per_swap=3, seed=4, trace_cap=30)]
        insts = [w.instance, m.instance]
        probs = [T.Problem(T.Instance.from_synth(i), c) for i, c in zip(insts, cfgs)]
        B = T.Batch(2)
        B.set_members(probs)
        assert B.driver() == 1
        B.run(30)
        B.close()
        for i, c, P in zip(insts, cfgs, probs):
            o = O.run(i, c.beta, c.p_q, mcs_per_swap=c.mcs_per_swap, n_rounds=30, seed=c.seed, trace=True)
            assert_same(o, P, f"batch slot order {order}")
    _with_env("TDPT_PERSISTENT", "1", lambda: _with_env("TDPT_SLOT_ORDER", order, go))


def test_persistent_slot_order_n200(T):
    """The N=200 workload (512 workgroups over every compute unit) with slots
    assigned in a scattered order: the first rounds equal the oracle."""
    w = wishart_n200()
    _with_env("TDPT_SLOT_ORDER", "251,100", lambda: both(
        T, w.instance, w.beta, w.p_q, mcs=1, rounds=12, seed=2, label="N200 slot order 251,100"))
