"""Fig. 2 on the GPU: with P-swaps the last replica samples the logical
Boltzmann distribution about as well as independent draws; without them
the hardest-penalty replica stays far from it."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from synth.configs import fig2_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2506_14781_amd as T
    return T


def test_p_swaps_reach_the_independent_sample_level(T):
    from paper_2506_14781_amd import sampling as S
    w = fig2_workload()
    inst = T.Instance.from_synth(w.instance, logical=True)
    target = S.boltzmann_logical(w.instance.J_logical_q, w.instance.b_logical_q, 1.0)
    fc = S.first_copies(w.instance.logical_of)
    t = 400
    kl = {}
    for label, flags in [("swaps", 0), ("none", T.NO_PSWAP)]:
        print(f"[sampling] {label}", file=sys.stderr, flush=True)
        vals = []
        for seed in range(3):
            P = T.Problem(inst, T.RunConfig(w.beta, w.p_q, mcs_per_swap=w.mcs_per_swap, seed=seed,
                                            flags=flags, hist_logical=True))
            counts, _ = S.sample_bottom_right(P, t, fc)
            vals.append(S.kl_divergence(counts, target))
        kl[label] = float(np.mean(vals))
    iid = (len(target) - 1) / (2.0 * t)
    assert kl["swaps"] < 4.0 * iid
    assert kl["none"] > 5.0 * kl["swaps"]
