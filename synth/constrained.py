"""Seeded constrained problems whose penalty g is a sum of squared linear
forms, g = sum_t (sum_{i in t} a_ti s_i + d_t)^2, for the general-constraint
path of 2D-PT.

Like the rest of this package it builds inputs only (couplings, fields,
constraint terms, a proper colouring, a planted answer) and none of the
method's arithmetic.

The paper's energy E = f + P g (Eq. 1) needs only g >= 0 with g = 0 exactly
on feasible states; its introduction names knapsack-type limits handled with
slack variables, sequencing constraints, and the copy constraints of graph
sparsification.  An equality constraint sum_i w_i x_i = c on bits
x = (1 + s) / 2 becomes the term a = w, d = sum_i w_i - 2c, whose square is
4 (w.x - c)^2; a copy edge is a = (1, -1), d = 0, so copy chains are a
special case.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .instances import Instance, balanced_coloring


def _term_pairs(term_ptr, term_idx):
    """Every pair of spins that share a term (for the colouring)."""
    a, b = [], []
    for t in range(len(term_ptr) - 1):
        members = term_idx[term_ptr[t]:term_ptr[t + 1]]
        for x in range(len(members)):
            for y in range(x + 1, len(members)):
                a.append(members[x])
                b.append(members[y])
    return np.asarray(a, dtype=np.int32), np.asarray(b, dtype=np.int32)


def _csr(n, rows, cols, vals):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.int32)
    o = np.lexsort((cols, rows))
    rows, cols, vals = rows[o], cols[o], vals[o]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr).astype(np.int32), cols.astype(np.int32), vals


def with_terms(inst: Instance, term_ptr, term_idx, term_coef, term_const, *, recolor=True) -> Instance:
    """The instance's couplings and fields with the given constraint terms in
    place of its copy edges; recoloured over couplings and term pairs unless
    recolor is False (then the caller's colouring must already be proper)."""
    term_ptr = np.asarray(term_ptr, dtype=np.int32)
    term_idx = np.asarray(term_idx, dtype=np.int32)
    color = inst.color
    if recolor:
        pa, pb = _term_pairs(term_ptr, term_idx)
        color = balanced_coloring(inst.n, inst.row_ptr, inst.col, pa, pb)
    return dataclasses.replace(
        inst, copy_a=np.zeros(0, np.int32), copy_b=np.zeros(0, np.int32), color=color,
        term_ptr=term_ptr, term_idx=term_idx,
        term_coef=np.asarray(term_coef, dtype=np.int32),
        term_const=np.asarray(term_const, dtype=np.int32))


def terms_from_copies(inst: Instance) -> Instance:
    """The same problem with each copy edge (a, b) written as the general term
    (s_a - s_b)^2, keeping the colouring (already proper over copy edges)."""
    m = len(inst.copy_a)
    term_ptr = np.arange(0, 2 * m + 1, 2, dtype=np.int32)
    term_idx = np.stack([inst.copy_a, inst.copy_b], axis=1).reshape(-1)
    term_coef = np.tile(np.array([1, -1], dtype=np.int32), m)
    return with_terms(inst, term_ptr, term_idx, term_coef, np.zeros(m, np.int32), recolor=False)


@dataclasses.dataclass
class Planted:
    instance: Instance
    state: np.ndarray     # int8[n], a feasible optimum
    f_target_q: int       # its f (Q12)


def planted_coloring(V: int, k: int, degree: int, seed: int, *, weight_q: int = 4096) -> Planted:
    """Graph k-colouring as a constrained Ising problem (one-hot encoding).

    A random graph on V nodes with a planted proper k-colouring (colour of
    node u drawn uniformly, balanced), each node joined to at most `degree`
    others of different planted colours.  Spin u*k + c is the bit x_uc
    "node u has colour c".  Cost: weight times the number of monochromatic
    edges, sum_(u,v) sum_c x_uc x_vc, in Ising form J = -weight/4 between
    (u,c) and (v,c), field -weight deg(u)/4 on (u,c) (f is the cost minus
    the constant weight k |E| / 4).  Constraint: one colour per node, the
    term sum_c s_uc + (k - 2) per node (g = 4 (sum_c x_uc - 1)^2).  The
    planted colouring is feasible with cost 0, so it is an optimum with
    f = -weight k |E| / 4.  Without the constraint the all-zero assignment
    also has cost 0; the penalty is what makes the problem a colouring.
    """
    if k < 2 or V < 2 or weight_q % 4:
        raise ValueError("need k >= 2, V >= 2 and a weight divisible by 4")
    rng = np.random.default_rng(seed)
    col_of = rng.permutation(np.arange(V) % k)
    deg = np.zeros(V, dtype=np.int64)
    nbrs = [set() for _ in range(V)]
    order = rng.permutation(V)
    for u in order:
        tries = 0
        while deg[u] < degree and tries < 8 * degree:
            tries += 1
            v = int(rng.integers(V))
            if v == u or col_of[v] == col_of[u] or deg[v] >= degree or v in nbrs[u]:
                continue
            nbrs[u].add(v)
            nbrs[v].add(u)
            deg[u] += 1
            deg[v] += 1
    n = V * k
    rows, cols, vals = [], [], []
    jq = -weight_q // 4
    for u in range(V):
        for v in nbrs[u]:
            for c in range(k):
                rows.append(u * k + c)
                cols.append(v * k + c)
                vals.append(jq)
    row_ptr, col, J_q = _csr(n, rows, cols, vals)
    b_q = np.repeat(-(weight_q // 4) * deg, k).astype(np.int32)
    term_ptr = np.arange(0, n + 1, k, dtype=np.int32)
    term_idx = np.arange(n, dtype=np.int32)
    term_coef = np.ones(n, dtype=np.int32)
    term_const = np.full(V, k - 2, dtype=np.int32)
    base = Instance(n=n, row_ptr=row_ptr, col=col, J_q=J_q, b_q=b_q,
                    copy_a=np.zeros(0, np.int32), copy_b=np.zeros(0, np.int32),
                    color=np.zeros(n, np.int32), logical_of=np.arange(n, dtype=np.int32), N=n)
    inst = with_terms(base, term_ptr, term_idx, term_coef, term_const)
    state = -np.ones(n, dtype=np.int8)
    state[np.arange(V) * k + col_of] = 1
    n_edges = int(deg.sum()) // 2
    inst.planted = state
    return Planted(inst, state, -(weight_q // 4) * k * n_edges)


def slack_knapsack(n_items: int, seed: int) -> Instance:
    """Quadratic knapsack with one capacity limit written with slack spins.

    Items i = 0..n_items-1 with weights w_i in 1..7, values v_i in 1..9 and
    pair values v_ij in 0..3; capacity C = floor(sum w / 2).  Maximise
    sum v_i x_i + sum_{i<j} v_ij x_i x_j subject to sum w_i x_i <= C, as the
    equality sum w_i x_i + sum_l 2^l y_l = C over L slack bits y with
    2^L - 1 >= C: one term over all items and slack spins, coefficients
    (w, 1, 2, .., 2^(L-1)), constant sum of them - 2C.  f = -value in Ising
    form (J_ij = v_ij / 4, b_i = v_i / 2 + sum_j v_ij / 4), Q12.
    """
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 8, size=n_items)
    v = rng.integers(1, 10, size=n_items)
    vp = np.triu(rng.integers(0, 4, size=(n_items, n_items)), 1)
    vp = vp + vp.T
    C = int(w.sum()) // 2
    L = max(1, int(C).bit_length())
    n = n_items + L
    rows, cols, vals = [], [], []
    for i in range(n_items):
        for j in range(n_items):
            if i != j and vp[i, j]:
                rows.append(i)
                cols.append(j)
                vals.append(int(vp[i, j]) * 1024)
    row_ptr, col, J_q = _csr(n, rows, cols, vals)
    b_q = np.zeros(n, dtype=np.int32)
    b_q[:n_items] = v * 2048 + vp.sum(axis=1) * 1024
    coef = np.concatenate([w, 1 << np.arange(L)]).astype(np.int32)
    base = Instance(n=n, row_ptr=row_ptr, col=col, J_q=J_q, b_q=b_q,
                    copy_a=np.zeros(0, np.int32), copy_b=np.zeros(0, np.int32),
                    color=np.zeros(n, np.int32), logical_of=np.arange(n, dtype=np.int32), N=n)
    return with_terms(base, [0, n], np.arange(n, dtype=np.int32), coef, [int(coef.sum()) - 2 * C])
