"""The C-ABI library loads on any host and validates instances host-side.

No GPU is needed: instance creation, validation and workspace sizing run on
the host; nothing here launches a kernel.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2506_14781_amd as T
from paper_2506_14781_amd import tdpt as B
from synth.configs import wishart_n200, wishart_small
from tests.tiny import tiny_instance

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "tdpt.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tdpt_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = T.load_library()
    names = header_functions()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(B.EXPORTED)


def _mk(inst, **over):
    d = dict(n=inst.n, row_ptr=inst.row_ptr, col=inst.col, J_q=inst.J_q, b_q=inst.b_q,
             copy_a=inst.copy_a, copy_b=inst.copy_b, color=inst.color)
    d.update(over)
    return T.Instance(**d)


def test_info_of_the_workloads():
    a = T.Instance.from_synth(wishart_small().instance).info()
    assert (a["n"], a["n_colors"], a["max_degree"], a["narrow"]) == (72, 2, 3, 1)
    assert a["n_pad"] % 4 == 0 and a["n_pad"] >= 72
    b = T.Instance.from_synth(wishart_n200().instance).info()
    assert b["n"] == 6800 and b["max_degree"] == 7 and b["max_copy_degree"] == 2
    assert b["m"] == 6600 and b["nnz"] == wishart_n200().instance.row_ptr[-1]


def test_rejects_asymmetric_couplings():
    inst = tiny_instance()
    J = inst.J_q.copy()
    J[0] += 1
    with pytest.raises(T.TdptError, match="symmetric"):
        _mk(inst, J_q=J)


def test_rejects_improper_colouring():
    inst = tiny_instance()
    color = inst.color.copy()
    a, b = inst.copy_a[0], inst.copy_b[0]
    color[b] = color[a]
    with pytest.raises(T.TdptError, match="proper"):
        _mk(inst, color=color)


def test_rejects_self_loop_and_bad_index():
    inst = tiny_instance()
    col = inst.col.copy()
    col[0] = 0
    with pytest.raises(T.TdptError, match="self loop|symmetric"):
        _mk(inst, col=col)
    col = inst.col.copy()
    col[0] = inst.n + 3
    with pytest.raises(T.TdptError, match="range"):
        _mk(inst, col=col)


def test_rejects_copy_edge_that_is_also_a_coupling():
    inst = tiny_instance()
    rows = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
    a, b = int(rows[0]), int(inst.col[0])
    ca = np.concatenate([inst.copy_a, [a]]).astype(np.int32)
    cb = np.concatenate([inst.copy_b, [b]]).astype(np.int32)
    with pytest.raises(T.TdptError, match="coupling"):
        _mk(inst, copy_a=ca, copy_b=cb)


def test_rejects_copy_graph_that_is_not_chains():
    # a star of copy edges around spin 0
    n = 4
    rp = np.zeros(n + 1, dtype=np.int32)
    with pytest.raises(T.TdptError, match="chains"):
        T.Instance(n, rp, np.zeros(0, np.int32), np.zeros(0, np.int32), None,
                   np.array([0, 0, 0], np.int32), np.array([1, 2, 3], np.int32),
                   np.array([0, 1, 1, 1], np.int32))


def test_rejects_bad_schedules():
    inst = T.Instance.from_synth(tiny_instance())
    for beta, pq, mcs in [([1.0, 0.5], [0], 1), ([0.0, 1.0], [0], 1), ([1.0], [10, 5], 1),
                          ([1.0], [-1], 1), ([1.0], [0], 0)]:
        with pytest.raises(T.TdptError):
            T.workspace_bytes(inst, T.RunConfig(beta, pq, mcs_per_swap=mcs, seed=0))


def test_workspace_grows_with_grid_and_trace():
    inst = T.Instance.from_synth(wishart_small().instance)
    a = T.workspace_bytes(inst, T.RunConfig([1.0], [0], mcs_per_swap=1, seed=0))
    b = T.workspace_bytes(inst, T.RunConfig(np.arange(1, 33), np.arange(16), mcs_per_swap=1,
                                            seed=0))
    c = T.workspace_bytes(inst, T.RunConfig(np.arange(1, 33), np.arange(16), mcs_per_swap=1,
                                            seed=0, trace_cap=10000))
    assert a < b < c


def test_error_message_is_thread_local_text():
    inst = tiny_instance()
    J = inst.J_q.copy()
    J[1] += 5
    try:
        _mk(inst, J_q=J)
    except T.TdptError as e:
        assert "symmetric" in str(e) and e.code == B.E_INVALID
    assert "symmetric" in T.load_library().tdpt_last_error().decode()


# ------------------------------------------------------ general constraints

def _terms(inst):
    return (inst.term_ptr, inst.term_idx, inst.term_coef, inst.term_const)


def test_terms_instance_info():
    from synth.constrained import planted_coloring
    pc = planted_coloring(50, 4, degree=5, seed=0)
    info = T.Instance.from_synth(pc.instance).info()
    assert info["n"] == 200 and info["n_terms"] == 50 and info["m"] == 0
    # problem rows (colouring edges, J = -1024) fit the packed layout;
    # constraint rows stay 32-bit in either layout
    assert info["max_constraint_degree"] == 3 and info["narrow"] == 1


def test_terms_rejects_malformed_terms():
    from synth.constrained import slack_knapsack
    inst = slack_knapsack(5, seed=2)
    tp, ti, tc, td = _terms(inst)
    base = dict(n=inst.n, row_ptr=inst.row_ptr, col=inst.col, J_q=inst.J_q, b_q=inst.b_q,
                copy_a=None, copy_b=None, color=inst.color)
    T.Instance(**base, terms=(tp, ti, tc, td))
    ti2 = ti.copy()
    ti2[1] = ti2[0]
    with pytest.raises(T.TdptError, match="repeated"):
        T.Instance(**base, terms=(tp, ti2, tc, td))
    ti3 = ti.copy()
    ti3[0] = inst.n
    with pytest.raises(T.TdptError, match="range"):
        T.Instance(**base, terms=(tp, ti3, tc, td))
    color = inst.color.copy()
    color[ti[1]] = color[ti[0]]
    with pytest.raises(T.TdptError, match="constraint pair|coupling"):
        T.Instance(**{**base, "color": color}, terms=(tp, ti, tc, td))
    big = tc.copy()
    big[0] = 1 << 30
    with pytest.raises(T.TdptError, match="int32|2\\^"):
        T.Instance(**base, terms=(tp, ti, big, td))


def test_terms_pair_with_zero_net_weight_may_share_a_colour():
    """Two terms whose products a_ti a_tj cancel leave i and j uncoupled:
    they may share a colour class."""
    n = 3
    rp = np.zeros(n + 1, np.int32)
    # (s0 + s1 + s2)^2 and (s0 - s1)^2: weights 0-1 pair: -(1) - (-1) = 0
    tp = np.array([0, 3, 5], np.int32)
    ti = np.array([0, 1, 2, 0, 1], np.int32)
    tc = np.array([1, 1, 1, 1, -1], np.int32)
    td = np.array([-1, 0], np.int32)
    color = np.array([0, 0, 1], np.int32)
    e = np.zeros(0, np.int32)
    inst = T.Instance(n, rp, e, e, None, None, None, color, terms=(tp, ti, tc, td))
    assert inst.info()["max_constraint_degree"] == 2  # spin 2 pairs with 0 and 1
    with pytest.raises(T.TdptError, match="constraint pair"):
        T.Instance(n, rp, e, e, None, None, None, np.array([0, 1, 0], np.int32),
                   terms=(tp, ti, tc, td))


def test_terms_workspace_and_range_checks():
    from synth.constrained import slack_knapsack
    inst = T.Instance.from_synth(slack_knapsack(5, seed=2))
    cfg = T.RunConfig([0.5, 1.0], [0, 4096], mcs_per_swap=1, seed=0)
    assert T.workspace_bytes(inst, cfg) > 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library every entry point raises instead of
    falling back to anything else."""
    import paper_2506_14781_amd.tdpt as TD
    monkeypatch.setattr(TD, "_lib", None)
    monkeypatch.setattr(TD, "LIB_PATH", str(tmp_path / "libtdpt.so"))
    with pytest.raises(RuntimeError, match="missing"):
        TD.load_library()
    from synth.configs import wishart_small
    with pytest.raises(RuntimeError, match="missing"):
        TD.Instance.from_synth(wishart_small().instance)


def test_logical_of_is_validated_and_reported():
    w = wishart_small().instance
    a = T.Instance.from_synth(w, logical=True).info()
    assert a["n_logical"] == 12
    assert T.Instance.from_synth(w).info()["n_logical"] == 0
    bad = w.logical_of.copy()
    bad[3] = w.n  # out of range
    with pytest.raises(T.TdptError, match="logical_of"):
        _mk(w, logical_of=bad)
    gap = w.logical_of.copy()
    gap[gap == 5] = 6  # variable 5 has no spin left
    with pytest.raises(T.TdptError, match="logical variable 5"):
        _mk(w, logical_of=gap)


def test_histogram_needs_a_small_logical_map():
    w = wishart_small()
    cfg = T.RunConfig(w.beta, w.p_q, mcs_per_swap=1, seed=0, hist_logical=True)
    with pytest.raises(T.TdptError, match="logical_of"):
        T.workspace_bytes(T.Instance.from_synth(w.instance), cfg)
    with_map = T.Instance.from_synth(w.instance, logical=True)
    plain = T.RunConfig(w.beta, w.p_q, mcs_per_swap=1, seed=0)
    # 2^12 four-byte bins in place of an 8-byte stub (both rounded to 256 bytes)
    assert T.workspace_bytes(with_map, cfg) == T.workspace_bytes(with_map, plain) + 4 * 4096 - 256
    big = wishart_n200().instance
    with pytest.raises(T.TdptError, match="at most 20"):
        T.workspace_bytes(T.Instance.from_synth(big, logical=True),
                          T.RunConfig([1.0], [0], mcs_per_swap=1, seed=0, hist_logical=True))


def test_layout_group_keys(monkeypatch):
    """The structure layout that selects a problem's sweep kernel instance,
    and the batch group key built from it: packed copy-edge problems of one
    ELL width share a key; general constraints on the packed layout, a wider
    row, the 32-bit layout and the bit-packed layout each get their own."""
    from synth.constrained import planted_coloring, slack_knapsack
    w = wishart_small()
    cfg = T.RunConfig(w.beta, w.p_q, mcs_per_swap=1, seed=0)
    a = T.Instance.from_synth(w.instance).layout(cfg)
    assert (a["bits"], a["narrow"], a["general"]) == (0, 1, 0)
    assert a["ell_width"] % 2 == 0 and a["ell_width"] >= 3
    assert a["group_key"] == a["bits"] | a["narrow"] << 1 | a["ell_width"] << 3
    # the same instance with another seed and grid: same key
    b = T.Instance.from_synth(w.instance).layout(T.RunConfig([1.0, 2.0], [0, 4096], mcs_per_swap=3, seed=9))
    assert b["group_key"] == a["group_key"]
    # general constraints on the packed layout
    pc = planted_coloring(40, 3, degree=4, seed=1).instance
    c = T.Instance.from_synth(pc).layout(T.RunConfig([1.0], [0, 4096], mcs_per_swap=1, seed=0))
    assert (c["narrow"], c["general"]) == (1, 1) and c["group_key"] & 4
    assert c["group_key"] != a["group_key"]
    # a penalty large enough to leave the packed layout's 22-bit fields
    d = T.Instance.from_synth(w.instance).layout(T.RunConfig([1.0], [0, 1 << 21], mcs_per_swap=1, seed=0))
    assert d["narrow"] == 0 and d["group_key"] != a["group_key"]
    # wide constraint rows (a knapsack term over 30 spins)
    k = T.Instance.from_synth(slack_knapsack(24, seed=1)).layout(T.RunConfig([1.0], [64], mcs_per_swap=1, seed=0))
    assert k["general"] == 1
    # the bit-packed layout (forced; chosen by itself above 48 KiB per replica)
    monkeypatch.setenv("TDPT_LAYOUT", "bits")
    e = T.Instance.from_synth(w.instance).layout(cfg)
    assert (e["bits"], e["narrow"]) == (1, 0) and e["group_key"] & 1
    assert len({a["group_key"], c["group_key"], d["group_key"], e["group_key"]}) == 4
    # its two forms run different kernels, so they group apart
    assert e["pair16"] == 1 and e["group_key"] == 1 | e["ell_width"] << 3 | 1 << 12
    monkeypatch.setenv("TDPT_PAIR16", "0")
    f = T.Instance.from_synth(w.instance).layout(cfg)
    assert f["pair16"] == 0 and f["group_key"] == e["group_key"] & ~(1 << 12)


def test_layout_default_packing(monkeypatch):
    """The per-round sweep's default launch shape.  While the problem's round
    fits within 2048 waves (latency-bound), small packed copy-edge replicas
    take one spin per lane, 2^s lanes covering the largest colour class's
    spins, 64 / 2^s replicas per 64-thread workgroup below 64 lanes; beyond
    that, replicas whose largest class takes under 64 quads share a
    workgroup at one quad per lane.  Two colour classes let the lanes hold
    their structure in registers, and then rounds of 16 sweeps or more run
    per-round launches; large replicas and the bit-packed layout keep one
    replica per workgroup."""
    from synth.configs import wishart_n200
    from tests.test_gpu_parity import _unequal_classes
    from tests.tiny import tiny_instance

    def shape(lay):
        return lay["spin"], lay["slots"], lay["lanes"], lay["held"], lay["per_round"]
    w = wishart_small()   # 72 spins, 2 classes of 9 quads, no fields; 8 x 4 grid
    inst = T.Instance.from_synth(w.instance)
    assert shape(inst.layout(T.RunConfig(w.beta, w.p_q, mcs_per_swap=50, seed=0))) == (1, 1, 64, 1, 1)
    assert shape(inst.layout(T.RunConfig(w.beta, w.p_q, mcs_per_swap=15, seed=0))) == (1, 1, 64, 1, 0)
    # 3072 replicas are 3072 waves: one quad per lane, 4 replicas per wave
    big = T.RunConfig(np.geomspace(0.1, 5, 64), np.arange(48, dtype=np.int32) * 64, mcs_per_swap=50, seed=0)
    assert shape(inst.layout(big)) == (0, 4, 16, 1, 1)
    # 10 spins with fields, 2 quads per class: 8 lanes, 8 replicas per wave
    tiny = T.Instance.from_synth(tiny_instance())
    assert shape(tiny.layout(T.RunConfig([1.0], [0, 4096], mcs_per_swap=50, seed=0))) == (1, 8, 8, 1, 1)
    # 20480 replicas (2560 waves) of it: one quad per lane, structure re-read (fields)
    many = T.RunConfig(np.geomspace(0.1, 5, 64), np.arange(320, dtype=np.int32) * 16, mcs_per_swap=50, seed=0)
    assert shape(tiny.layout(many)) == (0, 16, 4, 0, 0)
    # classes of 1 and 3 quads, no fields
    u = T.Instance.from_synth(_unequal_classes()).layout(T.RunConfig([1.0], [0, 4096], mcs_per_swap=20, seed=0))
    assert shape(u) == (1, 4, 16, 1, 1)
    # four colour classes (the three-copy N=16 J-column member, 48 spins,
    # ELL width 6): held at one spin per lane only
    from synth.configs import jcolumn_member
    jc = jcolumn_member(16, 20000)
    jl = T.Instance.from_synth(jc.instance).layout(T.RunConfig(jc.beta, jc.p_q, mcs_per_swap=20, seed=0))
    assert shape(jl) == (1, 4, 16, 1, 1)
    # 6800 spins, 850 quads per class: one replica per workgroup
    n2 = wishart_n200()
    c = T.Instance.from_synth(n2.instance).layout(T.RunConfig(n2.beta, n2.p_q, mcs_per_swap=1, seed=0))
    assert shape(c) == (0, 1, 0, 0, 0)
    monkeypatch.setenv("TDPT_LAYOUT", "bits")
    e = inst.layout(T.RunConfig(w.beta, w.p_q, mcs_per_swap=50, seed=0))
    assert e["bits"] == 1 and shape(e) == (0, 1, 0, 0, 0)


def test_layout_pair_form(monkeypatch):
    """The bit-packed layout's pair form (two replicas per word, coupling
    sums in 16-bit halves) is chosen exactly when every spin's sum of 2 |J|
    over its problem neighbours is below 2^15: the N=1000 workload (largest
    row sum 1007) takes it, an instance whose row sum reaches 2^14 does not,
    one just below does; TDPT_PAIR16=0 turns it off, and byte-layout
    problems never report it."""
    from synth.configs import wishart_n1000
    w = wishart_n1000()
    cfg = T.RunConfig(w.beta, w.p_q, mcs_per_swap=50, seed=0)
    lay = T.Instance.from_synth(w.instance).layout(cfg)
    assert lay["bits"] == 1 and lay["pair16"] == 1
    small = wishart_small()
    assert T.Instance.from_synth(small.instance).layout(
        T.RunConfig(small.beta, small.p_q, mcs_per_swap=5, seed=0))["pair16"] == 0

    def ring(j):
        # 8 spins on a ring, each with two neighbours of coupling j (row sum 2 j)
        n = 8
        rows = [sorted(((i - 1) % n, (i + 1) % n)) for i in range(n)]
        row_ptr = np.arange(0, 2 * n + 1, 2, dtype=np.int32)
        col = np.array([c for r in rows for c in r], dtype=np.int32)
        Jq = np.full(2 * n, j, dtype=np.int32)
        return T.Instance(n, row_ptr, col, Jq, np.zeros(n, np.int32),
                          np.zeros(0, np.int32), np.zeros(0, np.int32), (np.arange(n) % 2).astype(np.int32))
    rc = T.RunConfig([1.0], [0], mcs_per_swap=5, seed=0)
    monkeypatch.setenv("TDPT_LAYOUT", "bits")
    assert ring(8191).layout(rc)["pair16"] == 1     # 2 * 16382 < 2^15
    assert ring(8192).layout(rc)["pair16"] == 0     # 2 * 16384 = 2^15
    monkeypatch.setenv("TDPT_PAIR16", "0")
    assert ring(8191).layout(rc)["pair16"] == 0
