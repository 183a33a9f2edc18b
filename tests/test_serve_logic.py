"""Host scheduling of the serving loop (continuous batching) on the CPU:
the library's problems and batch are replaced by stand-ins that count rounds,
so admission under the memory budget and the running-work cap, retirement at
the cap or at a hit, and the order of completion can be checked without a
GPU.  The sampling itself is covered by the GPU tests."""
from __future__ import annotations

import types

import numpy as np
import pytest

import paper_2506_14781_amd.serve as S


class _Cfg:
    def __init__(self, replicas, mcs=1):
        self.replicas = replicas
        self.mcs_per_swap = mcs


class _Inst:
    def __init__(self, n):
        self.n = n


class _World:
    """Stand-ins for the library: problems advance only inside batch.run;
    a problem 'hits' its target at a chosen round (or never)."""

    def __init__(self, hit_round=None):
        self.hit_round = hit_round or {}
        self.live = []
        self.max_live = 0
        self.max_work = 0
        self.log = []

    def module(self):
        world = self

        class Problem:
            def __init__(self, instance, cfg, device="cuda"):
                self.instance, self.cfg, self.rounds = instance, cfg, 0
                self.closed = False
                world.live.append(self)
                world.max_live = max(world.max_live, len(world.live))
                world.max_work = max(world.max_work, sum(p.cfg.replicas * p.instance.n for p in world.live))

            def query(self):
                h = world.hit_round.get(id(self.instance))
                hit = h is not None and self.rounds >= h
                return {"rounds_done": self.rounds, "best_f_q": 0 if hit else (1 << 63) - 1,
                        "first_hit_sweep": h * self.cfg.mcs_per_swap if hit else -1}

            def close(self):
                assert not self.closed
                self.closed = True
                world.live.remove(self)

        class Batch:
            def __init__(self, cap, device="cuda", stream=None):
                self.members = []

            def set_members(self, probs):
                assert all(not p.closed for p in probs)
                self.members = list(probs)

            def run(self, n):
                assert n > 0 and self.members
                for p in self.members:
                    p.rounds += n
                world.log.append((n, len(self.members)))

            def query(self):
                rows = []
                for p in self.members:
                    q = p.query()
                    rows.append([q["rounds_done"], q["first_hit_sweep"], q["best_f_q"], -1])
                return np.array(rows, dtype=np.int64).reshape(-1, 4)

            def close(self):
                pass

        return types.SimpleNamespace(Problem=Problem, Batch=Batch,
                                     workspace_bytes=lambda inst, cfg: cfg.replicas * inst.n)


@pytest.fixture
def world(monkeypatch):
    import torch
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(torch.cuda, "Stream", lambda *a, **k: None)
    w = _World()
    monkeypatch.setattr(S, "T", w.module())
    return w


def _req(name, n, replicas, rounds, arrival=0.0):
    return S.Request(name=name, instance=_Inst(n), cfg=_Cfg(replicas), max_rounds=rounds, arrival=arrival)


def test_every_request_runs_exactly_its_cap(world):
    reqs = [_req(f"r{k}", 100 * (k + 1), 4, rounds=3 + k) for k in range(6)]
    S.serve(reqs, chunk=2, budget_bytes=10 ** 9)
    for r in reqs:
        assert r.rounds_done == r.max_rounds and r.end is not None and r.hit_time is None
    assert not world.live  # every problem closed


def test_memory_budget_bounds_the_running_batch(world):
    reqs = [_req(f"r{k}", 1000, 4, rounds=5) for k in range(5)]  # 4,000 bytes each
    S.serve(reqs, chunk=10, budget_bytes=8_000)
    assert world.max_live == 2
    assert all(r.rounds_done == 5 for r in reqs)


def test_work_cap_serves_in_arrival_order(world):
    """With the running work capped below two requests, they run one at a
    time and finish in arrival order; without it they share the batch."""
    reqs = [_req(f"r{k}", 1000, 8, rounds=4) for k in range(4)]
    S.serve(reqs, chunk=10, budget_bytes=10 ** 9, max_work=12_000)
    assert world.max_live == 1
    ends = [r.end for r in reqs]
    assert ends == sorted(ends)
    assert all(m == 1 for _, m in world.log)


def test_work_cap_admits_into_an_empty_batch(world):
    """A request larger than the cap still runs (alone)."""
    reqs = [_req("big", 10_000, 16, rounds=2), _req("small", 10, 1, rounds=2)]
    S.serve(reqs, chunk=10, budget_bytes=10 ** 9, max_work=1_000)
    assert all(r.rounds_done == 2 for r in reqs)
    assert world.max_live == 1


def test_without_cap_all_share_the_batch(world):
    reqs = [_req(f"r{k}", 1000, 8, rounds=4) for k in range(4)]
    S.serve(reqs, chunk=10, budget_bytes=10 ** 9)
    assert world.max_live == 4


def test_hit_retires_a_request_early(world):
    reqs = [_req("a", 100, 2, rounds=50), _req("b", 100, 2, rounds=6)]
    world.hit_round[id(reqs[0].instance)] = 3
    S.serve(reqs, chunk=2, budget_bytes=10 ** 9)
    a, b = reqs
    assert a.hit_sweep == 3 and a.hit_time is not None
    assert a.rounds_done < a.max_rounds  # retired at the chunk that hit
    assert b.rounds_done == 6 and b.hit_time is None


def test_request_over_budget_is_rejected(world):
    with pytest.raises(ValueError):
        S.serve([_req("huge", 10_000, 4, rounds=1)], chunk=1, budget_bytes=1_000)


def test_summary_counts_hits_and_updates():
    reqs = [_req("a", 10, 2, rounds=4), _req("b", 10, 2, rounds=4)]
    reqs[0].hit_time, reqs[0].hit_sweep, reqs[0].rounds_done = 0.5, 3, 3
    reqs[1].rounds_done = 4
    s = S.summarize(reqs, 2.0)
    assert s["hit_fraction"] == 0.5 and s["tts_p50_s"] == 0.5
    assert s["spin_updates"] == (3 + 4) * 1 * 2 * 10
    assert np.isclose(s["spin_updates_per_s"], s["spin_updates"] / 2.0)


def test_late_arrival_runs_exactly_its_cap(world):
    """A request that arrives while others run is set up (possibly during a
    chunk) and joins at a round boundary: it runs exactly its own rounds."""
    reqs = [_req("first", 100, 2, rounds=6), _req("late", 100, 2, rounds=2, arrival=0.02)]
    S.serve(reqs, chunk=2, budget_bytes=10 ** 9)
    assert [r.rounds_done for r in reqs] == [6, 2]
    assert reqs[1].start >= reqs[1].arrival
    assert not world.live


def test_cancelled_request_is_dropped_at_a_round_boundary(world):
    """A request cancelled while it runs leaves the batch at the next round
    boundary with the rounds it ran; the others run to their caps."""
    reqs = [_req("a", 100, 2, rounds=40), _req("b", 100, 2, rounds=12)]

    def on_chunk(now, active, pending):
        if reqs[0].rounds_done >= 4:
            reqs[0].cancelled = True
    S.serve(reqs, chunk=2, budget_bytes=10 ** 9, on_chunk=on_chunk)
    a, b = reqs
    assert a.status == "cancelled" and a.rounds_done == 4 and a.end is not None
    assert b.status == "cap" and b.rounds_done == 12
    assert not world.live


def test_cancelled_before_admission_never_runs(world):
    reqs = [_req("a", 100, 2, rounds=6), _req("b", 100, 2, rounds=6, arrival=0.05)]
    reqs[1].cancelled = True
    S.serve(reqs, chunk=2, budget_bytes=10 ** 9)
    assert reqs[1].status == "cancelled" and reqs[1].rounds_done == 0 and reqs[1].problem is None
    assert reqs[0].status == "cap" and reqs[0].rounds_done == 6


def test_deadline_drops_running_and_waiting_requests(world, monkeypatch):
    """Time limits: a running request past its limit is dropped at a round
    boundary; a waiting one (held back by the memory budget) never starts."""
    clock = {"t": 0.0}
    monkeypatch.setattr(S.time, "perf_counter", lambda: clock["t"])
    monkeypatch.setattr(S.time, "sleep", lambda dt: clock.__setitem__("t", clock["t"] + max(dt, 1e-3)))
    reqs = [_req("slow", 1000, 4, rounds=100), _req("waits", 1000, 4, rounds=5)]
    reqs[0].deadline = 1.0
    reqs[1].deadline = 0.5

    def on_chunk(now, active, pending):
        clock["t"] += 0.1  # every chunk takes 0.1 s
    S.serve(reqs, chunk=2, budget_bytes=4_000, on_chunk=on_chunk)  # room for one at a time
    slow, waits = reqs
    assert slow.status == "timeout" and 0 < slow.rounds_done < 100
    assert waits.status == "timeout" and waits.rounds_done == 0 and waits.start is None
    assert not world.live


def test_status_of_finished_requests(world):
    reqs = [_req("a", 100, 2, rounds=50), _req("b", 100, 2, rounds=6)]
    world.hit_round[id(reqs[0].instance)] = 3
    S.serve(reqs, chunk=2, budget_bytes=10 ** 9)
    assert [r.status for r in reqs] == ["hit", "cap"]
    s = S.summarize(reqs, 1.0)
    assert s["dropped"] == {"timeout": 0, "cancelled": 0}
