"""Long GPU runs against the exact stationary distribution of the grid.

The stationary distribution of 2D-PT is the product over grid positions of
the Boltzmann distributions at (beta_i, P_j) (Appendix A), so on the
enumerable 10-spin instance every position's mean f and g and every
adjacent pair's swap acceptance (Eq. 2, Eq. 3) are known exactly.  One long
chain of 10^5 rounds runs on the GPU, sampled every 4 rounds (one period of
Algorithm 1's schedule) into device buffers with the library's _async
reads; its estimates must lie within 3 standard errors of the exact values,
the errors from 40 batch means after 10 % burn-in.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

from tests.tiny import batch_means_check, exact_grid_expectations, tiny_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2506_14781_amd as T
    return T


GRIDS = {
    "2x2": (np.array([0.4, 1.0]), np.array([2048, 6144], dtype=np.int32)),
    "4x4": (np.geomspace(0.1, 5.0, 4), np.array([0, 5461, 10923, 16384], dtype=np.int32)),
}


def gpu_long_run(T, inst, beta, p_q, chunks, mcs, seed, n_batches=40, burn=0.1):
    """One GPU chain of 4 * chunks rounds; f and g of every position after
    every 4 rounds (device buffers, read once at the end), swap counters
    read at the burn-in point and at every batch boundary.  Returns what
    batch_means_check takes: samples [chunks, I, J] and per-sample counter
    increments, each batch's increments booked on its first sample."""
    import torch
    I, J = len(beta), len(p_q)
    R = I * J
    P = T.Problem(T.Instance.from_synth(inst), T.RunConfig(beta, p_q, mcs_per_swap=mcs, seed=seed))
    fbuf = torch.zeros((chunks, R), dtype=torch.int64, device="cuda")
    gbuf = torch.zeros((chunks, R), dtype=torch.int64, device="cuda")
    t0 = int(chunks * burn)
    L = (chunks - t0) // n_batches
    marks = [t0 + k * L for k in range(n_batches + 1)]
    reads = {}

    def counters():
        pa, pc, ba, bc = P.counters()
        return pc.copy(), bc.copy(), pa.copy(), ba.copy()
    if t0 == 0:
        reads[0] = counters()
    for c in range(chunks):
        P.run(4)
        P.energies_async(fbuf[c], gbuf[c])
        if c + 1 in marks:
            reads[c + 1] = counters()
    driver = P.query()["driver"]
    fs = fbuf.cpu().numpy().reshape(chunks, I, J)
    gs = gbuf.cpu().numpy().reshape(chunks, I, J)
    P.close()
    pa = np.zeros((chunks, I, max(J - 1, 0)), np.int64)
    pt = np.zeros_like(pa)
    ba = np.zeros((chunks, J, max(I - 1, 0)), np.int64)
    bt = np.zeros_like(ba)
    for k in range(n_batches):
        a, b = reads[marks[k]], reads[marks[k + 1]]
        row = marks[k]
        pa[row], ba[row], pt[row], bt[row] = (b[0] - a[0], b[1] - a[1], b[2] - a[2], b[3] - a[3])
    return fs, gs, (pa, ba), (pt, bt), driver


@pytest.mark.parametrize("grid,driver", [("2x2", "1"), ("4x4", "1"), ("4x4", "0")])
def test_gpu_long_run_batch_means_within_3_se(T, grid, driver):
    inst = tiny_instance()
    beta, p_q = GRIDS[grid]
    print(f"[stats] {grid} driver {driver}: 1e5 rounds", file=sys.stderr, flush=True)
    old = os.environ.get("TDPT_PERSISTENT")
    os.environ["TDPT_PERSISTENT"] = driver
    try:
        fs, gs, acc, att, used = gpu_long_run(T, inst, beta, p_q, chunks=25000, mcs=2, seed=17)
    finally:
        if old is None:
            del os.environ["TDPT_PERSISTENT"]
        else:
            os.environ["TDPT_PERSISTENT"] = old
    assert used == int(driver)
    fails = batch_means_check(fs, gs, acc, att, exact_grid_expectations(inst, beta, p_q))
    assert not fails, "\n".join(fails)
