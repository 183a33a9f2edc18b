"""J-column PT configuration (host logic, no GPU)."""
import numpy as np
import pytest

from paper_2506_14781_amd import jcolumn as JC
from synth.configs import jcolumn_member
from synth.instances import linear_penalties_q, q12


def test_mean_penalty_is_the_rounded_mean():
    assert JC.mean_penalty_q(linear_penalties_q(0, 6, 8)) == q12([3.0])[0]
    assert JC.mean_penalty_q([1, 2]) == 2          # 1.5 rounds away from zero
    assert JC.mean_penalty_q([0, 0, 1]) == 0


def test_column_configs_share_beta_and_penalty_but_not_streams():
    w = jcolumn_member(16, 20000)
    cfgs = JC.column_configs(w.beta, w.p_q, mcs_per_swap=50, seed=3, trace_cap=10)
    assert len(cfgs) == w.n_p
    assert all(np.array_equal(c.beta, w.beta) for c in cfgs)
    assert all(c.p_q.tolist() == [JC.mean_penalty_q(w.p_q)] for c in cfgs)
    seeds = {c.seed for c in cfgs} | {3}
    assert len(seeds) == w.n_p + 1


def test_three_copy_instances_fit_the_kernels():
    w = jcolumn_member(48, 20000)
    assert w.instance.n == 144
    deg = np.diff(w.instance.row_ptr)
    assert deg.max() <= 16
