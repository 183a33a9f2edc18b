"""Algorithm 2 on the GPU sampler equals the oracle's Algorithm 2."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import adaptive as OA
from synth.configs import wishart_small
from tests.tiny import tiny_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2506_14781_amd as T
    return T


@pytest.mark.parametrize("which,sigma_min,i_max,j_max", [("tiny", 0.0, 6, 6), ("wishart-N12", 0.3, 10, 5)])
def test_adaptive_schedule_equals_the_oracle(T, which, sigma_min, i_max, j_max):
    from paper_2506_14781_amd.adaptive import adaptive_schedule
    inst = tiny_instance() if which == "tiny" else wishart_small().instance
    print(f"[adaptive] {which}", file=sys.stderr, flush=True)
    s = adaptive_schedule(T.Instance.from_synth(inst), beta0=0.1, p0=0.0, i_max=i_max, j_max=j_max,
                          sigma_min=sigma_min, alpha_beta=0.5, alpha_p=0.5, n_chain=64, mcs=10, seed=3)
    ob, op, ok = OA.adaptive_schedule(inst, 0.1, 0.0, I=i_max, J=j_max, sigma_min=sigma_min, alpha_beta=0.5,
                                      alpha_P=0.5, N_chain=64, MCS=10, seed=3)
    assert s.populations == ok
    np.testing.assert_allclose(s.beta, ob, rtol=1e-12, atol=0)
    assert s.p_q.tolist() == op.tolist()
