"""Fig. 2 measurement helpers (host, no GPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_14781_amd import sampling as S
from synth.configs import fig2_workload


def test_exact_distribution_matches_the_oracle_energies():
    """pi(x) from the logical couplings equals exp(-beta f) of the oracle's
    energy of the chain-consistent physical state (g = 0 there)."""
    w = fig2_workload()
    inst = w.instance
    pi = S.boltzmann_logical(inst.J_logical_q, inst.b_logical_q, 1.0)
    fs = []
    for k in range(32):
        x = np.array([1 if (k >> j) & 1 else -1 for j in range(5)], dtype=np.int8)
        f, g = O.energy(inst, inst.physical_state(x))
        assert g == 0
        fs.append(f / 4096.0)
    fs = np.array(fs)
    ref = np.exp(-(fs - fs.min()))
    np.testing.assert_allclose(pi, ref / ref.sum(), rtol=1e-9)


def test_logical_index_reads_the_state_back():
    w = fig2_workload()
    fc = S.first_copies(w.instance.logical_of)
    for k in [0, 5, 17, 31]:
        x = np.array([1 if (k >> j) & 1 else -1 for j in range(5)], dtype=np.int8)
        assert S.logical_index(w.instance.physical_state(x), fc) == k


def test_kl_divergence():
    p = np.array([0.5, 0.25, 0.25])
    assert S.kl_divergence(p * 8, p) == pytest.approx(0.0, abs=1e-15)
    assert S.kl_divergence([1, 0], [0.25, 0.75]) == pytest.approx(np.log(4.0))
    assert S.kl_divergence([3, 1], [0.5, 0.5]) == pytest.approx(0.75 * np.log(1.5) + 0.25 * np.log(0.5))
