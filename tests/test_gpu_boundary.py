"""The boundary's newer calls on the GPU, through the C ABI: the decoded
logical best state, the per-round device histogram of the bottom-right
replica's logical state, reads into device buffers, and the rules of batch
membership (TDPT_E_BUSY while a batch run is in flight, TDPT_E_STATE after a
member leaves)."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from synth.configs import fig2_workload, wishart_small

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2506_14781_amd as T
    return T


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


@pytest.mark.parametrize("layout", ["bytes", "bits"])
def test_logical_best_and_async_reads(T, layout):
    """N=12 planted Wishart, seed 5 (reaches the planted ground state): the
    logical best state is the best state read at each variable's first copy,
    it is the planted state up to the global flip, and every _async read
    equals its synchronous twin and the oracle."""
    import torch
    w = wishart_small()
    inst = w.instance
    f_gs = O.energy(inst, inst.physical_state(inst.planted))[0]
    rounds = 200
    _say(f"[boundary] logical best + async reads, {layout} layout")
    cfg = T.RunConfig(w.beta, w.p_q, mcs_per_swap=w.mcs_per_swap, seed=5, f_target=f_gs)
    P = _with_env("TDPT_LAYOUT", layout, lambda: T.Problem(T.Instance.from_synth(inst, logical=True), cfg))
    P.run(rounds)
    o = O.run(inst, w.beta, w.p_q, mcs_per_swap=w.mcs_per_swap, n_rounds=rounds, seed=5, f_target=f_gs)
    assert o["first_hit"] > 0 and o["best_f"] == f_gs
    s, bf, bw = P.best()
    x, xf, xw = P.best_logical()
    first = np.array([np.flatnonzero(inst.logical_of == k)[0] for k in range(inst.N)])
    assert np.array_equal(x, s[first]) and (xf, xw) == (bf, bw) == (o["best_f"], o["best_sweep"])
    assert np.array_equal(x, inst.planted) or np.array_equal(x, -inst.planted)
    dev = torch.device("cuda")
    fd = torch.zeros(P.R, dtype=torch.int64, device=dev)
    gd = torch.zeros(P.R, dtype=torch.int64, device=dev)
    sd = torch.zeros((P.R, P.n), dtype=torch.int8, device=dev)
    bd = torch.zeros(P.n, dtype=torch.int8, device=dev)
    bfs = torch.zeros(2, dtype=torch.int64, device=dev)
    words = torch.zeros(4, dtype=torch.int64, device=dev)
    P.energies_async(fd, gd)
    P.states_async(sd)
    P.best_async(bd, bfs)
    P.query_async(words)
    torch.cuda.synchronize()
    f, g = P.energies()
    assert np.array_equal(fd.cpu().numpy(), f) and np.array_equal(gd.cpu().numpy(), g)
    assert np.array_equal(f, o["f"]) and np.array_equal(g, o["g"])
    assert np.array_equal(sd.cpu().numpy(), P.states()) and np.array_equal(P.states(), o["states"])
    assert np.array_equal(bd.cpu().numpy(), s) and np.array_equal(s, o["best_state"])
    assert bfs.cpu().tolist() == [bf, bw]
    q = P.query()
    assert words.cpu().tolist() == [q["rounds_done"], q["first_hit_sweep"], q["best_f_q"], q["best_sweep"]]
    # only one of the energy outputs
    gd.zero_()
    P.energies_async(None, gd)
    torch.cuda.synchronize()
    assert np.array_equal(gd.cpu().numpy(), g)
    P.close()


def _host_histogram(T, inst, w, rounds, seed, flags):
    """The bottom-right replica's logical state counted on the host, one
    round at a time."""
    from paper_2506_14781_amd import sampling as S
    P = T.Problem(T.Instance.from_synth(inst),
                  T.RunConfig(w.beta, w.p_q, mcs_per_swap=w.mcs_per_swap, seed=seed, flags=flags))
    counts, _ = S.sample_bottom_right(P, rounds, S.first_copies(inst.logical_of))
    P.close()
    return counts


@pytest.mark.parametrize("driver", ["0", "1"])
def test_device_histogram_equals_host_count(T, driver):
    """The Fig. 2 workload (1 x 4 grid, 500 sweeps per round) with P-swaps and
    without: the device histogram after 120 rounds equals the bottom-right
    logical states read back and counted on the host round by round, in
    both drivers, and reading it mid-run leaves the run unchanged."""
    w = fig2_workload(rounds=120)
    inst = w.instance
    for flags in (0, T.NO_PSWAP):
        _say(f"[boundary] histogram driver {driver} flags {flags}")
        want = _host_histogram(T, inst, w, 120, 3, flags)
        cfg = T.RunConfig(w.beta, w.p_q, mcs_per_swap=w.mcs_per_swap, seed=3, flags=flags, hist_logical=True)
        P = _with_env("TDPT_PERSISTENT", driver,
                      lambda: T.Problem(T.Instance.from_synth(inst, logical=True), cfg))
        assert P.query()["driver"] == int(driver)
        P.run(50)
        mid, k = P.histogram()
        assert k == 50 and mid.sum() == 50
        P.run(70)
        got, k = P.histogram()
        assert k == 120 and np.array_equal(got.astype(np.int64), want)
        P.close()


def test_device_histogram_in_a_batch(T):
    """Histogrammed problems inside a batch with an ordinary one: the same
    counts as alone."""
    w = fig2_workload(rounds=40)
    inst = w.instance
    lone = []
    for seed in (1, 2):
        cfg = T.RunConfig(w.beta, w.p_q, mcs_per_swap=w.mcs_per_swap, seed=seed, hist_logical=True)
        P = T.Problem(T.Instance.from_synth(inst, logical=True), cfg)
        P.run(40)
        lone.append(P.histogram()[0])
        P.close()
    probs = [T.Problem(T.Instance.from_synth(inst, logical=True),
                       T.RunConfig(w.beta, w.p_q, mcs_per_swap=w.mcs_per_swap, seed=seed, hist_logical=True))
             for seed in (1, 2)]
    ws = wishart_small()
    other = T.Problem(T.Instance.from_synth(ws.instance), T.RunConfig(ws.beta, ws.p_q, mcs_per_swap=5, seed=0))
    B = T.Batch(4)
    B.set_members(probs + [other])
    for driver in (-1, 0):
        B.set_driver(driver)
        B.run(20)
    for P, want in zip(probs, lone):
        got, k = P.histogram()
        assert k == 40 and np.array_equal(got, want)
    B.close()


def test_batch_membership_rules(T):
    """While a batch run is in flight its members refuse to run, load or
    autotune on their own (TDPT_E_BUSY) and accept it once the run is done;
    destroying a member, or naming it in another batch, leaves the batch
    refusing to run (TDPT_E_STATE) until its members are set again; the
    remaining members' results equal their runs alone."""
    w = wishart_small()
    inst = T.Instance.from_synth(w.instance)
    long_run = 2000  # about 2000 launch pairs: in flight far longer than a few host calls

    def make(seed):
        return T.Problem(inst, T.RunConfig(w.beta, w.p_q, mcs_per_swap=50, seed=seed, trace_cap=64))
    alone = []
    for seed in range(3):
        P = make(seed)
        P.run(long_run + 20)
        alone.append((P.states(), *P.energies()))
        P.close()
    probs = [make(seed) for seed in range(3)]
    B = T.Batch(4)
    B.set_members(probs)
    B.set_driver(0)  # per-round launches
    blob = probs[0].save()
    B.run(long_run)
    codes = []
    for fn in (lambda: probs[0].run(1), lambda: probs[0].load(blob), lambda: probs[0].autotune(1)):
        with pytest.raises(T.TdptError) as ei:
            fn()
        codes.append(ei.value.code)
    _say(f"[boundary] codes while in flight: {codes}")
    assert codes == [T.E_BUSY] * 3
    probs[0].query()  # waits for the batch
    probs[0].run(20)  # allowed now
    B.set_members(probs[1:])
    B.run(20)
    for P, a in zip(probs, alone):
        assert np.array_equal(P.states(), a[0])
        f, g = P.energies()
        assert np.array_equal(f, a[1]) and np.array_equal(g, a[2])
    # a member destroyed: the batch must be given its members again
    probs[2].close()
    with pytest.raises(T.TdptError) as ei:
        B.run(1)
    assert ei.value.code == T.E_STATE
    B.set_members(probs[:2])
    B.run(1)
    # a member moved to another batch
    C = T.Batch(2)
    C.set_members([probs[1]])
    with pytest.raises(T.TdptError) as ei:
        B.run(1)
    assert ei.value.code == T.E_STATE
    C.run(1)
    B.set_members([probs[0]])
    B.run(1)
    assert probs[0].query()["rounds_done"] == long_run + 22
    assert probs[1].query()["rounds_done"] == long_run + 22
    B.close()
    C.close()


def test_stage_trace_of_the_persistent_driver(T):
    """Stage timestamps for 12 rounds of a persistent run: every slot's four
    stamps are ordered within each round, rounds follow one another, rounds
    past the cap stay unwritten, and the run's results equal the oracle's."""
    import torch
    from tests.test_gpu_parity import assert_same
    w = wishart_small()
    cfg = T.RunConfig(w.beta, w.p_q, mcs_per_swap=5, seed=4, trace_cap=30)
    P = _with_env("TDPT_PERSISTENT", "1", lambda: T.Problem(T.Instance.from_synth(w.instance), cfg))
    assert P.query()["driver"] == 1
    P.run(6)
    buf = torch.zeros(16 * P.R * 4, dtype=torch.int64, device="cuda")
    P.set_stage_trace(buf, 12)
    P.run(24)
    P.set_stage_trace(None, 0)
    t = buf.view(16, P.R, 4).cpu().numpy()
    assert (t[:12] > 0).all() and (t[12:] == 0).all()
    assert (np.diff(t[:12], axis=2) >= 0).all()
    assert (t[1:12, :, 0] >= t[:11, :, 3]).all()
    o = O.run(w.instance, w.beta, w.p_q, mcs_per_swap=5, n_rounds=30, seed=4, trace=True)
    assert_same(o, P, "with stage trace")


def test_batch_poll_equals_member_queries(T):
    """One batch-wide poll returns every member's rounds, first hit, best f
    and best sweep in the order the members were given (the batch keeps them
    sorted by layout internally), synchronously and into a device buffer."""
    import torch
    from synth.configs import batched_member
    w = wishart_small()
    f_gs = O.energy(w.instance, w.instance.physical_state(w.instance.planted))[0]
    m = batched_member(100, 0.8, 5)
    probs = [T.Problem(T.Instance.from_synth(m.instance), T.RunConfig(m.beta[:4], m.p_q[:4], mcs_per_swap=3,
                                                                       seed=1)),
             T.Problem(T.Instance.from_synth(w.instance), T.RunConfig(w.beta, w.p_q, mcs_per_swap=50, seed=5,
                                                                       f_target=f_gs)),
             T.Problem(T.Instance.from_synth(w.instance), T.RunConfig(w.beta, w.p_q, mcs_per_swap=50, seed=7,
                                                                       f_target=f_gs))]
    B = T.Batch(4)
    B.set_members(probs)
    B.run(200)
    words = B.query()
    dev = torch.zeros((3, 4), dtype=torch.int64, device="cuda")
    B.query_async(dev)
    torch.cuda.synchronize()
    for row, drow, P in zip(words, dev.cpu().numpy(), probs):
        q = P.query()
        want = [q["rounds_done"], q["first_hit_sweep"], q["best_f_q"], q["best_sweep"]]
        assert row.tolist() == want and drow.tolist() == want
    assert words[1][1] > 0  # seed 5 reaches the planted ground state within 1e4 sweeps
    B.set_members([probs[2], probs[0]])
    B.run(2)
    assert B.query()[:, 0].tolist() == [202, 202]
    B.close()
