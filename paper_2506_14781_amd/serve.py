"""Host drivers over the C ABI: plain, batched and continuously batched runs.

All sampling work runs in the library's kernels; this module only decides
which problems run when, and measures wall time to the planted ground state.

* plain   — one problem at a time, each until its target is hit or its sweep
            cap is reached, the next starting when the previous stops;
* batched — every problem in one batch from t = 0, solved ones retired;
* serving — requests arrive over time; a request is admitted into the running
            batch as soon as its device footprint fits the memory budget,
            joins at the next round boundary, and retires when it hits its
            target or reaches its cap, or is dropped when it is cancelled
            or its time limit runs out.  Requests already on the GPU keep
            running while new ones are admitted (continuous batching).

A result does not depend on the mode: random streams are keyed per problem.
Hit times: the hit sweep is exact; its wall time is interpolated inside the
chunk of rounds in which it happened.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import tdpt as T


@dataclasses.dataclass
class Request:
    """One solve: an instance, its run configuration, a round cap."""
    name: str
    instance: "T.Instance"
    cfg: "T.RunConfig"
    max_rounds: int
    arrival: float = 0.0            # seconds after the start of the job
    # filled in by the drivers
    start: float | None = None
    end: float | None = None
    hit_time: float | None = None   # seconds after arrival, None if censored
    hit_sweep: int = -1
    rounds_done: int = 0
    best_f: int | None = None
    problem: "T.Problem | None" = None
    footprint: int = 0
    # optional reference for reporting: ground-state f_q and logical size
    f_ref: int | None = None
    n_logical: int = 0
    # serving controls: a time limit in seconds after arrival (None: none),
    # and a flag the caller may set at any time to cancel the request
    deadline: float | None = None
    cancelled: bool = False
    # how the request ended: "hit", "cap", "timeout" or "cancelled"
    status: str | None = None


def _book(req: Request, rounds_done: int, first_hit: int, best_f: int, t0: float, t1: float,
          elapsed_base: float):
    """Book a chunk of rounds that ran from wall time t0 to t1, given the
    problem's status after it."""
    prev = req.rounds_done
    req.rounds_done = int(rounds_done)
    req.best_f = int(best_f)
    if req.hit_time is None and first_hit >= 0:
        mcs = req.cfg.mcs_per_swap
        hit_round = int(first_hit) // mcs
        frac = (hit_round - prev) / max(req.rounds_done - prev, 1)
        req.hit_sweep = int(first_hit)
        req.hit_time = (t0 - elapsed_base) + frac * (t1 - t0) - req.arrival


def _advance(req: Request, rounds: int, t0: float, t1: float, elapsed_base: float):
    """Book a chunk of `rounds` rounds of one problem (its own status read)."""
    q = req.problem.query()
    _book(req, q["rounds_done"], q["first_hit_sweep"], q["best_f_q"], t0, t1, elapsed_base)


def _advance_all(batch, reqs, t0: float, t1: float, elapsed_base: float):
    """Book a chunk for every member of the batch from one status poll
    (members in set_members order)."""
    words = batch.query()
    for r, w in zip(reqs, words):
        _book(r, w[0], w[1], w[2], t0, t1, elapsed_base)


def _done(req: Request) -> bool:
    return req.hit_time is not None or req.rounds_done >= req.max_rounds


def _finish_status(req: Request) -> str:
    return "hit" if req.hit_time is not None else "cap"


def _dropped(req: Request, now: float) -> str | None:
    """"cancelled" or "timeout" if the request is to be dropped at time now
    (seconds after the job's start), else None."""
    if req.cancelled:
        return "cancelled"
    if req.deadline is not None and now - req.arrival >= req.deadline:
        return "timeout"
    return None


def run_plain(requests, chunk: int, device="cuda"):
    """Each request alone, one after another (all present at t = 0)."""
    import torch
    base = time.perf_counter()
    for req in requests:
        req.problem = T.Problem(req.instance, req.cfg, device=device)
        torch.cuda.synchronize()
        req.start = time.perf_counter() - base
        while not _done(req):
            n = min(chunk, req.max_rounds - req.rounds_done)
            t0 = time.perf_counter()
            req.problem.run(n)
            torch.cuda.synchronize()
            _advance(req, n, t0, time.perf_counter(), base)
        req.end = time.perf_counter() - base
        req.status = _finish_status(req)
        req.problem.close()
        req.problem = None
    return time.perf_counter() - base


def run_batched(requests, chunk: int, device="cuda"):
    """All requests in one batch from t = 0; solved or capped ones retire."""
    import torch
    batch = T.Batch(len(requests), device=device)
    for req in requests:
        req.problem = T.Problem(req.instance, req.cfg, device=device)
    torch.cuda.synchronize()
    base = time.perf_counter()
    active = list(requests)
    for req in active:
        req.start = 0.0
    batch.set_members([r.problem for r in active])
    while active:
        n = min(chunk, min(r.max_rounds - r.rounds_done for r in active))
        t0 = time.perf_counter()
        batch.run(n)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _advance_all(batch, active, t0, t1, base)
        still = []
        for r in active:
            if _done(r):
                r.end = t1 - base
                r.status = _finish_status(r)
            else:
                still.append(r)
        if len(still) != len(active) and still:
            batch.set_members([r.problem for r in still])
        active = still
    total = time.perf_counter() - base
    batch.close()
    for req in requests:
        req.problem.close()
        req.problem = None
    return total


def serve(requests, chunk: int, budget_bytes: int, max_members: int = 4096, device="cuda",
          max_work: int | None = None, on_chunk=None):
    """Continuous batching: requests (sorted by arrival) join the running
    batch at round boundaries when their workspace fits the budget and, if
    max_work is given, while the spin updates per sweep of the running batch
    (replicas x spins, summed) stay within it (a request is always admitted
    into an empty batch).  Capping the running work lets requests finish in
    arrival order instead of all sharing the GPU until the end.

    A request whose `cancelled` flag is set, or whose `deadline` (seconds
    after its arrival) has passed, is dropped at the next round boundary
    (or before admission): its problem is released and its status set to
    "cancelled" or "timeout"; its counters keep the rounds it ran.
    on_chunk(now, active, pending), if given, is called after every chunk
    (the caller may set flags there)."""
    import torch
    pending = sorted(requests, key=lambda r: r.arrival)
    for r in pending:
        r.footprint = T.workspace_bytes(r.instance, r.cfg)
        if r.footprint > budget_bytes:
            raise ValueError(f"request {r.name} needs {r.footprint} bytes, budget {budget_bytes}")
    batch = T.Batch(max_members, device=device)
    active = []
    used = 0
    work = 0

    def work_of(r):
        return r.cfg.replicas * r.instance.n

    base = time.perf_counter()
    while pending or active:
        now = time.perf_counter() - base
        changed = False
        # requests dropped before they ran
        keep = []
        for r in pending:
            why = _dropped(r, now) if r.arrival <= now or r.cancelled else None
            if why:
                r.status = why
                r.end = now
            else:
                keep.append(r)
        pending = keep
        # requests dropped while running
        if active:
            still = []
            for r in active:
                why = _dropped(r, now)
                if why:
                    r.status = why
                    r.end = now
                    used -= r.footprint
                    work -= work_of(r)
                    r.problem.close()
                    r.problem = None
                    changed = True
                else:
                    still.append(r)
            active = still
        if not pending and not active:
            break
        while (pending and pending[0].arrival <= now and used + pending[0].footprint <= budget_bytes
               and len(active) < max_members
               and (max_work is None or not active or work + work_of(pending[0]) <= max_work)):
            r = pending.pop(0)
            r.problem = T.Problem(r.instance, r.cfg, device=device)
            r.start = time.perf_counter() - base
            used += r.footprint
            work += work_of(r)
            active.append(r)
            changed = True
        if not active:
            if changed:
                batch.set_members([])
            # idle until the next arrival
            time.sleep(max(0.0, min(pending[0].arrival - now, 0.01)))
            continue
        if changed:
            batch.set_members([r.problem for r in active])
        n = min(chunk, min(r.max_rounds - r.rounds_done for r in active))
        t0 = time.perf_counter()
        batch.run(n)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _advance_all(batch, active, t0, t1, base)
        still = []
        for r in active:
            if _done(r):
                r.end = t1 - base
                r.status = _finish_status(r)
                used -= r.footprint
                work -= work_of(r)
                r.problem.close()
                r.problem = None
            else:
                still.append(r)
        if len(still) != len(active):
            active = still
            batch.set_members([r.problem for r in active])
        if on_chunk is not None:
            on_chunk(t1 - base, list(active), list(pending))
    total = time.perf_counter() - base
    batch.close()
    return total


def summarize(requests, total_seconds: float):
    """p50/p99 of time to the target (censored requests count as not hit),
    sweeps to hit, success fraction and spin updates."""
    hit = [r for r in requests if r.hit_time is not None]
    times = np.array([r.hit_time for r in hit]) if hit else np.array([])
    sweeps = np.array([r.hit_sweep for r in hit]) if hit else np.array([])
    updates = sum(r.rounds_done * r.cfg.mcs_per_swap * r.cfg.replicas * r.instance.n
                  for r in requests)
    out = {
        "requests": len(requests),
        "hit_fraction": len(hit) / max(len(requests), 1),
        "dropped": {k: sum(1 for r in requests if r.status == k) for k in ("timeout", "cancelled")},
        "tts_p50_s": float(np.percentile(times, 50)) if len(times) else None,
        "tts_p99_s": float(np.percentile(times, 99)) if len(times) else None,
        "sweeps_to_hit_p50": float(np.percentile(sweeps, 50)) if len(sweeps) else None,
        "sweeps_to_hit_p99": float(np.percentile(sweeps, 99)) if len(sweeps) else None,
        "makespan_s": total_seconds,
        "spin_updates": int(updates),
        "spin_updates_per_s": updates / total_seconds if total_seconds > 0 else None,
    }
    lat = [r.end - r.arrival for r in requests if r.end is not None]
    if lat:
        out["latency_p50_s"] = float(np.percentile(lat, 50))
        out["latency_p99_s"] = float(np.percentile(lat, 99))
    # best feasible bottom-right energy reached, as residual energy per
    # logical spin above the reference (rho_E), where a reference is known
    feasible = [r for r in requests if r.best_f is not None and r.best_f < (1 << 62)]
    out["feasible_fraction"] = len(feasible) / max(len(requests), 1)
    rho = [(r.best_f - r.f_ref) / (4096.0 * r.n_logical) for r in feasible
           if r.f_ref is not None and r.n_logical > 0]
    if rho:
        out["best_rho_E_p50"] = float(np.percentile(rho, 50))
        out["best_rho_E_max"] = float(np.max(rho))
    return out
