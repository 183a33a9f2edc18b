"""Seeded synthetic inputs for two-dimensional parallel tempering (2D-PT).

This module builds the *inputs* of the method and nothing else: planted
Wishart couplings, their int32 fixed-point form, the copy-chain
sparsification that turns a dense logical problem into a bounded-degree
physical one, a proper colouring of the physical graph, and the beta / P
schedules.  It holds none of the method's arithmetic (no sweeps, energies,
swap rules or random streams); both the CPU oracle and the GPU library take
what it returns as plain arrays.

Passages of the paper these inputs follow:
  * planted Wishart instances with density alpha (section "Ground-state
    optimization under constraints"); the construction itself (t uniform
    +-1, z ~ N(0, I), w = z - (z.t/N) t, J = -(1/N) sum w w^T, zero
    diagonal) is the one the workload definitions state, since the paper's
    bibliography is not part of its text;
  * sparsification by copy chains: each logical node becomes a chain of
    physical copies that share its neighbours, consecutive copies joined by
    a copy constraint (S_a - S_b)^2 (section "Graph sparsification with copy
    constraints", Fig. 2a);
  * ordered beta and P vectors (Algorithm 1 inputs).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

Q_SHIFT = 12
Q_SCALE = 1 << Q_SHIFT


def q12(x) -> np.ndarray:
    """Round real values to int32 Q12 fixed point, half away from zero."""
    x = np.asarray(x, dtype=np.float64) * Q_SCALE
    r = np.where(x >= 0, np.floor(x + 0.5), np.ceil(x - 0.5))
    if np.any(np.abs(r) >= 2**31):
        raise OverflowError("value does not fit int32 Q12")
    return r.astype(np.int32)


def planted_wishart(N: int, alpha: float, seed: int):
    """Planted Wishart couplings (dense, float64) and the planted state t.

    M = floor(alpha*N + 0.5) random vectors are drawn, each projected so it
    is orthogonal to t; J = -(1/N) sum_mu w_mu w_mu^T has zero diagonal.
    With the energy convention f(s) = -sum_{i<j} J_ij s_i s_j, +-t are
    ground states.
    """
    rng = np.random.default_rng(seed)
    M = int(math.floor(alpha * N + 0.5))
    t = rng.choice(np.array([-1, 1], dtype=np.int64), N)
    Z = rng.standard_normal((M, N))
    W = Z - np.outer(Z @ t / N, t)
    J = -(W.T @ W) / N
    np.fill_diagonal(J, 0.0)
    return J, t.astype(np.int8)


@dataclasses.dataclass
class Instance:
    """A sparsified Ising instance in the form the library boundary takes.

    row_ptr/col/J_q: symmetric CSR of the problem couplings (Q12 int32) over
    the n physical spins, both directions present, rows sorted.
    b_q: Q12 fields (int32[n]).
    copy_a/copy_b: copy-constraint edges (int32[m]); g = sum (s_a - s_b)^2.
    term_*: general constraints instead (see below), None with copy edges.
    color: proper colouring over problem and copy edges (int32[n]).
    logical_of: logical node of each physical spin (int32[n]).
    N: logical size; planted: planted logical state (int8[N]) or None.
    """
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    J_q: np.ndarray
    b_q: np.ndarray
    copy_a: np.ndarray
    copy_b: np.ndarray
    color: np.ndarray
    logical_of: np.ndarray
    N: int
    planted: np.ndarray | None = None
    J_logical_q: np.ndarray | None = None
    b_logical_q: np.ndarray | None = None
    # General constraints in place of copy edges (copy_a / copy_b empty):
    # g = sum_t (sum_{e in t} term_coef[e] s[term_idx[e]] + term_const[t])^2,
    # term t holding entries term_ptr[t] .. term_ptr[t+1]-1.
    term_ptr: np.ndarray | None = None
    term_idx: np.ndarray | None = None
    term_coef: np.ndarray | None = None
    term_const: np.ndarray | None = None

    @property
    def n_colors(self) -> int:
        return int(self.color.max()) + 1 if self.n else 0

    def physical_state(self, logical_state) -> np.ndarray:
        """Copy a logical state onto every copy of its chain."""
        return np.asarray(logical_state, dtype=np.int8)[self.logical_of]


def chain_length_for_degree(deg: int, D: int) -> int:
    """Shortest chain whose copies can hold `deg` problem neighbours.

    End copies have one chain neighbour (D-1 problem slots), interior copies
    two (D-2 slots); a single copy holds D.
    """
    if deg <= D:
        return 1
    if D < 3:
        raise ValueError("degree cap must be >= 3 to build chains")
    L = 2
    while 2 * (D - 1) + (L - 2) * (D - 2) < deg:
        L += 1
    return L


def mirror_chain_length(N: int, D: int) -> int:
    """Even chain length of the mirror embedding under degree cap D.

    The first half of the chain holds the circular offsets d = 1 .. N/2 (the
    exact middle offset only for half of the nodes), so it needs
    (D-1) + (L/2 - 1)(D-2) >= ceil((N-1)/2) + (1 if N is even).
    """
    if N - 1 <= D:
        return 1
    if D < 3:
        raise ValueError("degree cap must be >= 3 to build chains")
    h = (N - 1) // 2 + (1 if N % 2 == 0 else 0)
    half = 1
    while (D - 1) + (half - 1) * (D - 2) < h:
        half += 1
    return 2 * half


def _mirror_holders(N: int, D: int, L: int, i: int):
    """Copy index of node i that holds circular offset d, for d = 1..N-1.

    Offsets of the first half fill copies 0, 1, .. L/2-1 in increasing d
    (copy 0 takes D-1, later ones D-2); offset d of the second half goes to
    copy L-1-c(N-d), the mirror of the copy holding N-d.  For even N the
    middle offset N/2 belongs to the first half of nodes i < N/2 and to the
    second half of the others.
    """
    half = []
    for d in range(1, N):
        if 2 * d < N or (2 * d == N and i < N // 2):
            half.append(d)
    first_n = (N - 1) // 2 + (1 if N % 2 == 0 else 0)
    cap = [D - 1] + [D - 2] * (L // 2 - 1)
    cfirst = {}
    c, used = 0, 0
    for d in range(1, first_n + 1):
        while used >= cap[c]:
            c += 1
            used = 0
        cfirst[d] = c
        used += 1
    out = np.zeros(N, dtype=np.int64)
    for d in range(1, N):
        if 2 * d < N or (2 * d == N and i < N // 2):
            out[d] = cfirst[d]
        else:
            out[d] = L - 1 - cfirst[N - d]
    return out


def sparsify(Jq_logical: np.ndarray, *, degree_cap: int | None = None,
             copies: int | None = None, order: str = "mirror", numbering: str = "copy"):
    """Copy-chain sparsification of a dense symmetric logical coupling matrix.

    Exactly one of degree_cap / copies is given.  The paper leaves open how a
    node's neighbours are distributed among its copies; three rules exist:

      "mirror" (degree_cap only): even chains; neighbour i+d (circular
          offset d) of node i sits on copy c(d) and offset N-d on copy
          L-1-c(d), so every coupling joins copies of opposite parity and
          the physical graph is bipartite (two colour classes);
      "circular": neighbours in circular order i+1, i+2, .. fill copy 0,
          then copy 1, .. (shortest chain under the cap);
      "ascending": the same with neighbours in index order 0, 1, ..

    copies: every chain has that many copies and the neighbours (circular
    order) are split into near-equal contiguous groups.  Couplings that are
    zero are not edges.

    numbering: how physical spins are numbered.  "copy" (copy-major): all
    copies 0 in logical order, then all copies 1, ..; with the mirror
    embedding the k-th neighbour of copy c of node i is then node i + d_k
    on one fixed copy, so spins with consecutive numbers have neighbours
    with consecutive numbers.  "logical": the copies of node 0, then of
    node 1, ..  Returns (row_ptr, col, Jq, copy_a, copy_b, logical_of,
    copy_index).
    """
    if numbering not in ("copy", "logical"):
        raise ValueError("numbering must be 'copy' or 'logical'")
    Jq_logical = np.asarray(Jq_logical)
    N = Jq_logical.shape[0]
    if (degree_cap is None) == (copies is None):
        raise ValueError("give exactly one of degree_cap / copies")
    if order == "mirror" and degree_cap is None:
        order = "circular"
    L = np.zeros(N, dtype=np.int64)
    holder = []  # holder[i][j] = copy index of node i that holds neighbour j (-1: none)
    for i in range(N):
        nb = np.flatnonzero(Jq_logical[i])
        nb = nb[nb != i]
        h = np.full(N, -1, dtype=np.int64)
        if order == "mirror":
            Li = mirror_chain_length(N, degree_cap)
            if Li == 1:
                h[nb] = 0
            else:
                cd = _mirror_holders(N, degree_cap, Li, i)
                h[nb] = cd[(nb - i) % N]
        else:
            if order == "circular":
                nb = nb[np.argsort((nb - i - 1) % N, kind="stable")]
            elif order != "ascending":
                raise ValueError("order must be 'mirror', 'circular' or 'ascending'")
            d = len(nb)
            if degree_cap is not None:
                Li = chain_length_for_degree(d, degree_cap)
                if Li == 1:
                    cap = np.array([degree_cap])
                else:
                    cap = np.full(Li, degree_cap - 2)
                    cap[0] = cap[-1] = degree_cap - 1
                h[nb] = np.repeat(np.arange(Li), cap)[:d]
            else:
                Li = copies
                h[nb] = (np.arange(d) * Li) // max(d, 1)
        L[i] = Li
        holder.append(h)
    off = np.concatenate([[0], np.cumsum(L)])
    n = int(off[-1])
    logical_of = np.repeat(np.arange(N), L).astype(np.int32)
    copy_index = (np.arange(n) - off[logical_of]).astype(np.int32)
    # number of each (node, copy) spin: logical-major first, then renumbered
    if numbering == "copy":
        old_of_new = np.lexsort((logical_of, copy_index))
    else:
        old_of_new = np.arange(n)
    new_of_old = np.empty(n, dtype=np.int64)
    new_of_old[old_of_new] = np.arange(n)
    rows, cols, vals = [], [], []
    for i in range(N):
        for j in np.flatnonzero(holder[i] >= 0):
            rows.append(off[i] + holder[i][j])
            cols.append(off[j] + holder[j][i])
            vals.append(Jq_logical[i, j])
    rows = new_of_old[np.asarray(rows, dtype=np.int64)]
    cols = new_of_old[np.asarray(cols, dtype=np.int64)]
    vals = np.asarray(vals, dtype=np.int32)
    # within a row, neighbours in increasing circular offset of their node
    # (for the mirror embedding the k-th neighbour of every copy c spin then
    # has the same offset), then by number
    lnew = logical_of[old_of_new]
    offset = (lnew[cols] - lnew[rows]) % N
    srt = np.lexsort((cols, offset, rows))
    rows, cols, vals = rows[srt], cols[srt], vals[srt]
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    ca, cb = [], []
    for i in range(N):
        for c in range(int(L[i]) - 1):
            ca.append(off[i] + c)
            cb.append(off[i] + c + 1)
    ca = new_of_old[np.asarray(ca, dtype=np.int64)]
    cb = new_of_old[np.asarray(cb, dtype=np.int64)]
    return (row_ptr, cols.astype(np.int32), vals, ca.astype(np.int32), cb.astype(np.int32),
            logical_of[old_of_new].astype(np.int32), copy_index[old_of_new].astype(np.int32))


def _adjacency(n, row_ptr, col, copy_a, copy_b):
    """Undirected adjacency (CSR) over problem and copy edges."""
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    a = np.concatenate([src, copy_a, copy_b]).astype(np.int64)
    b = np.concatenate([col, copy_b, copy_a]).astype(np.int64)
    order = np.lexsort((b, a))
    a, b = a[order], b[order]
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ptr, a + 1, 1)
    return np.cumsum(ptr), b


def parity_coloring_if_proper(n, row_ptr, col, copy_a, copy_b, copy_index):
    """Colour = copy index mod 2, if that is proper (bipartite embedding)."""
    color = (np.asarray(copy_index) % 2).astype(np.int32)
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    if np.any(color[src] == color[col]) or np.any(color[copy_a] == color[copy_b]):
        return None
    return color


def balanced_coloring(n, row_ptr, col, copy_a, copy_b, max_colors=None):
    """Proper colouring with few, near-equal classes.

    Vertices are taken in smallest-last order and each gets the admissible
    colour whose class is currently smallest among the first C colours, C
    growing only when no admissible colour exists.  Any proper colouring
    gives a valid chromatic sweep; fewer and evener classes only make the
    parallel sweep cheaper.
    """
    ptr, adj = _adjacency(n, row_ptr, col, copy_a, copy_b)
    deg = np.diff(ptr)
    # smallest-last ordering by repeated removal of a minimum-degree vertex
    maxd = int(deg.max()) if n else 0
    buckets = [set() for _ in range(maxd + 1)]
    cur = deg.copy()
    for v in range(n):
        buckets[cur[v]].add(v)
    removed = np.zeros(n, dtype=bool)
    order = []
    dmin = 0
    for _ in range(n):
        while not buckets[dmin]:
            dmin += 1
        v = min(buckets[dmin])
        buckets[dmin].discard(v)
        removed[v] = True
        order.append(v)
        for u in adj[ptr[v]:ptr[v + 1]]:
            if not removed[u]:
                buckets[cur[u]].discard(u)
                cur[u] -= 1
                buckets[cur[u]].add(u)
                if cur[u] < dmin:
                    dmin = cur[u]
    order.reverse()
    color = np.full(n, -1, dtype=np.int64)
    sizes = []
    for v in order:
        used = {int(color[u]) for u in adj[ptr[v]:ptr[v + 1]] if color[u] >= 0}
        best = -1
        for c in range(len(sizes)):
            if c not in used and (best < 0 or sizes[c] < sizes[best]):
                best = c
        if best < 0:
            best = len(sizes)
            sizes.append(0)
            if max_colors is not None and best >= max_colors:
                raise ValueError("colouring needs more than max_colors")
        color[v] = best
        sizes[best] += 1
    # rebalance: move vertices from the largest class to smaller admissible ones
    sizes = np.bincount(color, minlength=len(sizes))
    target = int(math.ceil(n / len(sizes)))
    for c in np.argsort(-sizes):
        for v in np.flatnonzero(color == c):
            if sizes[c] <= target:
                break
            used = {int(color[u]) for u in adj[ptr[v]:ptr[v + 1]]}
            cand = [k for k in range(len(sizes)) if k not in used and sizes[k] < target]
            if cand:
                k = min(cand, key=lambda k: sizes[k])
                color[v] = k
                sizes[c] -= 1
                sizes[k] += 1
    return color.astype(np.int32)


def build_instance(N: int, alpha: float, seed: int, *, degree_cap=None,
                   copies=None, order: str = "mirror") -> Instance:
    """Planted Wishart instance, Q12-quantised, sparsified and coloured."""
    J, t = planted_wishart(N, alpha, seed)
    Jq = q12(J)
    np.fill_diagonal(Jq, 0)
    row_ptr, col, vals, ca, cb, logical_of, cidx = sparsify(
        Jq, degree_cap=degree_cap, copies=copies, order=order)
    n = int(logical_of.shape[0])
    color = parity_coloring_if_proper(n, row_ptr, col, ca, cb, cidx)
    if color is None:
        color = balanced_coloring(n, row_ptr, col, ca, cb)
    return Instance(n=n, row_ptr=row_ptr, col=col, J_q=vals,
                    b_q=np.zeros(n, dtype=np.int32), copy_a=ca, copy_b=cb,
                    color=color, logical_of=logical_of, N=N, planted=t,
                    J_logical_q=Jq)


def instance_from_logical(Jq_logical, *, b_logical_q=None, degree_cap=None,
                          copies=None, planted=None, order: str = "mirror") -> Instance:
    """Sparsify and colour a caller-supplied dense logical Q12 problem."""
    Jq_logical = np.asarray(Jq_logical, dtype=np.int32)
    N = Jq_logical.shape[0]
    row_ptr, col, vals, ca, cb, logical_of, cidx = sparsify(
        Jq_logical, degree_cap=degree_cap, copies=copies, order=order)
    n = int(logical_of.shape[0])
    b = np.zeros(n, dtype=np.int32)
    if b_logical_q is not None:
        # the field of a logical node sits on its copy 0
        first = np.flatnonzero(cidx == 0)
        first = first[np.argsort(logical_of[first], kind="stable")]
        b[first] = np.asarray(b_logical_q, dtype=np.int32)
    color = parity_coloring_if_proper(n, row_ptr, col, ca, cb, cidx)
    if color is None:
        color = balanced_coloring(n, row_ptr, col, ca, cb)
    return Instance(n=n, row_ptr=row_ptr, col=col, J_q=vals, b_q=b,
                    copy_a=ca, copy_b=cb, color=color, logical_of=logical_of,
                    N=N, planted=planted, J_logical_q=Jq_logical,
                    b_logical_q=None if b_logical_q is None else np.asarray(b_logical_q, dtype=np.int32))


def geometric_betas(lo: float, hi: float, count: int) -> np.ndarray:
    return np.geomspace(lo, hi, count).astype(np.float64)


def linear_penalties_q(lo: float, hi: float, count: int) -> np.ndarray:
    return q12(np.linspace(lo, hi, count))


def random_spins(rng: np.random.Generator, count: int) -> np.ndarray:
    """Uniform +-1 int8 spins (caller-supplied initial states)."""
    return (rng.integers(0, 2, size=count, dtype=np.int8) * 2 - 1).astype(np.int8)
