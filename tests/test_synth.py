"""Host-side input builders: sparsification and colouring invariants."""
import numpy as np
import pytest

from synth.configs import batched_sizes, serving_grid, wishart_n200, wishart_small
from synth.instances import (_adjacency, build_instance, chain_length_for_degree,
                             mirror_chain_length, q12)


def _check(inst, cap=None):
    n = inst.n
    rp, col = inst.row_ptr, inst.col
    rows = np.repeat(np.arange(n), np.diff(rp))
    # symmetric, no self loops, no duplicates
    assert not np.any(rows == col)
    pairs = set(zip(rows.tolist(), col.tolist()))
    assert len(pairs) == len(col)
    assert all((b, a) in pairs for a, b in pairs)
    Jd = dict(zip(zip(rows.tolist(), col.tolist()), inst.J_q.tolist()))
    assert all(Jd[(a, b)] == Jd[(b, a)] for a, b in pairs)
    # copy edges join consecutive copies of one logical node, disjoint from problem edges
    assert np.all(inst.logical_of[inst.copy_a] == inst.logical_of[inst.copy_b])
    assert not any((a, b) in pairs for a, b in zip(inst.copy_a, inst.copy_b))
    ptr, adj = _adjacency(n, rp, col, inst.copy_a, inst.copy_b)
    deg = np.diff(ptr)
    if cap is not None:
        assert deg.max() <= cap
    # proper colouring
    src = np.repeat(np.arange(n), deg)
    assert not np.any(inst.color[src] == inst.color[adj])
    # every logical coupling appears exactly once between the two chains
    Jl = inst.J_logical_q
    lr, lc = inst.logical_of[rows], inst.logical_of[col]
    cnt = np.zeros_like(Jl, dtype=np.int64)
    np.add.at(cnt, (lr, lc), 1)
    assert np.array_equal(cnt, (Jl != 0).astype(np.int64))


def test_chain_lengths_for_the_workload_caps():
    assert chain_length_for_degree(11, 4) == 5
    assert chain_length_for_degree(199, 8) == 33
    assert chain_length_for_degree(999, 6) == 250
    assert chain_length_for_degree(3, 3) == 1
    # mirror embedding: even chains
    assert mirror_chain_length(12, 4) == 6
    assert mirror_chain_length(200, 8) == 34
    assert mirror_chain_length(1000, 6) == 250
    assert mirror_chain_length(64, 6) == 16
    assert mirror_chain_length(4, 3) == 1


@pytest.mark.parametrize("N,D", [(12, 4), (13, 4), (40, 5), (64, 6), (101, 6), (200, 8)])
def test_mirror_embedding_is_bipartite(N, D):
    """Every coupling joins copies of opposite parity, so two colour classes."""
    inst = build_instance(N, 0.75, 1, degree_cap=D)
    _check(inst, cap=D)
    assert inst.n_colors == 2
    sizes = np.bincount(inst.color)
    assert abs(int(sizes[0]) - int(sizes[1])) <= N


def test_small_and_n200_instances():
    a = wishart_small().instance
    assert a.n == 72
    _check(a, cap=4)
    b = wishart_n200().instance
    assert b.n == 6800
    _check(b, cap=8)
    assert b.n_colors == 2


def test_batched_member_shapes():
    sizes = batched_sizes(8)
    for N, alpha, seed in sizes[:3]:
        inst = build_instance(N, alpha, seed, degree_cap=6)
        _check(inst, cap=6)


def test_copies_per_node_mode():
    inst = build_instance(20, 0.75, 1, copies=3)
    assert inst.n == 60 and len(inst.copy_a) == 40
    _check(inst)


@pytest.mark.parametrize("order", ["circular", "ascending"])
def test_other_distribution_orders(order):
    inst = build_instance(30, 0.75, 2, degree_cap=6, order=order)
    _check(inst, cap=6)


def test_q12_rounding_half_away_from_zero():
    assert q12([0.5 / 4096, -0.5 / 4096, 1.49 / 4096, -2.5 / 4096]).tolist() == [1, -1, 1, -3]
    with pytest.raises(OverflowError):
        q12([2.0**20])


def test_serving_grid():
    assert serving_grid(64) == (8, 4)
    assert serving_grid(1024) == (64, 32)
