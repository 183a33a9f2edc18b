"""Algorithm 2 (adaptive schedule): the oracle's version against closed forms
and its own structure (CPU).  The library's version is compared with it in
the GPU tests."""
import numpy as np
import pytest

from oracle import adaptive as OA
from synth.instances import Instance
from tests.tiny import tiny_instance


def _free_spins(b_q):
    """Isolated spins with fields (no couplings, no copies, one colour)."""
    n = len(b_q)
    return Instance(n=n, row_ptr=np.zeros(n + 1, np.int32), col=np.zeros(0, np.int32),
                    J_q=np.zeros(0, np.int32), b_q=np.asarray(b_q, np.int32),
                    copy_a=np.zeros(0, np.int32), copy_b=np.zeros(0, np.int32),
                    color=np.zeros(n, np.int32), logical_of=np.arange(n, dtype=np.int32), N=n)


def _copy_pair():
    """Two copies of one node, no couplings: g = (s_a - s_b)^2."""
    return Instance(n=2, row_ptr=np.zeros(3, np.int32), col=np.zeros(0, np.int32),
                    J_q=np.zeros(0, np.int32), b_q=np.zeros(2, np.int32),
                    copy_a=np.array([0], np.int32), copy_b=np.array([1], np.int32),
                    color=np.array([0, 1], np.int32), logical_of=np.zeros(2, np.int32), N=1)


def test_population_energy_spread_of_free_spins():
    """Independent spins with fields b: Var E = sum b^2 (1 - tanh^2(beta b))."""
    b = np.array([0.5, -1.0, 2.0, 0.25, -0.75])
    inst = _free_spins(np.round(b * 4096).astype(np.int32))
    beta = 0.8
    sig_e, sig_g, mean_g = OA.population(inst, beta, 0.0, N_chain=4096, MCS=3, seed=11)
    exact = np.sqrt(np.sum(b ** 2 * (1.0 - np.tanh(beta * b) ** 2)))
    assert sig_e == pytest.approx(exact, rel=0.05)
    assert sig_g == 0.0 and mean_g == 0.0


def test_population_constraint_statistics_of_a_copy_pair():
    """g = 4 with probability p = e^{-4 beta P} / (1 + e^{-4 beta P}), so
    mean g = 4p and sigma_g = 4 sqrt(p (1 - p)); with no couplings E = P g."""
    inst = _copy_pair()
    beta, P = 1.0, 0.3
    sig_e, sig_g, mean_g = OA.population(inst, beta, P, N_chain=4096, MCS=3, seed=5)
    Pq = OA._q12(P)
    w = np.exp(-4.0 * beta * Pq / 4096.0)
    p = w / (1.0 + w)
    assert mean_g == pytest.approx(4.0 * p, rel=0.06)
    assert sig_g == pytest.approx(4.0 * np.sqrt(p * (1.0 - p)), rel=0.05)
    assert sig_e == pytest.approx(Pq / 4096.0 * sig_g, rel=1e-12)


def test_no_constraints_means_one_column():
    inst = _free_spins([4096, -2048, 1024])
    beta, P, k = OA.adaptive_schedule(inst, 0.1, 0.5, I=5, J=4, sigma_min=0.0, alpha_beta=1.0,
                                      alpha_P=1.0, N_chain=64, MCS=5, seed=0)
    assert len(P) == 1 and P[0] == OA._q12(0.5)
    assert len(beta) == 5 and np.all(np.diff(beta) > 0)
    assert k == 5


def test_rows_stop_at_sigma_min_and_columns_grow_until_feasible():
    inst = tiny_instance()
    beta, P, k = OA.adaptive_schedule(inst, 0.1, 0.0, I=6, J=6, sigma_min=1e9, alpha_beta=1.0,
                                      alpha_P=1.0, N_chain=64, MCS=5, seed=0)
    assert beta.tolist() == [0.1] and k == 1 and len(P) == 1
    beta, P, k = OA.adaptive_schedule(inst, 0.1, 0.0, I=6, J=6, sigma_min=0.0, alpha_beta=0.5,
                                      alpha_P=0.5, N_chain=64, MCS=5, seed=0)
    assert len(beta) == 6 and np.all(np.diff(beta) > 0)
    assert 2 <= len(P) <= 6 and np.all(np.diff(P) > 0)
    assert k == 6 + 6 * (len(P) - 1)
