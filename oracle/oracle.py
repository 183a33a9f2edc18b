"""ctypes wrapper around the CPU oracle (tdpt_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  The GPU library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tdpt_oracle.c")
# TDPT_ORACLE_LIB names another build of the same source (the sanitizer test
# loads an AddressSanitizer / UBSan build this way)
_LIB = os.environ.get("TDPT_ORACLE_LIB") or os.path.join(_HERE, "_build", "libtdpt_oracle.so")

NO_PSWAP = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle: plain C, -O2, no FMA contraction, no fast-math;
    OpenMP only to split a round's sweeps over positions when asked
    (set_threads)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.environ.get("TDPT_ORACLE_LIB") and (
                not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        _lib.oracle_philox4x32_10.argtypes = [P, P, P]
        _lib.oracle_color_rank.argtypes = [ctypes.c_int32, P, P, P]
        _lib.oracle_energy.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int32, P, P, P, P, P]
        _lib.oracle_pswap_exponent.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_int64, ctypes.c_int64]
        _lib.oracle_pswap_exponent.restype = ctypes.c_double
        _lib.oracle_bswap_exponent.argtypes = [ctypes.c_double, ctypes.c_double,
                                               ctypes.c_int64, ctypes.c_int64]
        _lib.oracle_bswap_exponent.restype = ctypes.c_double
        _lib.oracle_swap_accept.argtypes = [ctypes.c_double, ctypes.c_double]
        _lib.oracle_heat_bath.argtypes = [ctypes.c_double, ctypes.c_int64, ctypes.c_uint32]
        _lib.oracle_schedule.argtypes = [ctypes.c_int64, ctypes.c_uint32, P, P]
        _lib.oracle_set_threads.argtypes = [ctypes.c_int32]
        _lib.oracle_set_threads.restype = None
        _lib.oracle_run.argtypes = (
            [ctypes.c_int32, P, P, P, P, ctypes.c_int32, P, P, P,
             ctypes.c_int32, P, ctypes.c_int32, P,
             ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
             P, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32]
            + [P] * 3 + [P] * 4 + [P] * 4 + [P, P, ctypes.c_int64])
        _lib.oracle_run.restype = ctypes.c_int
        _lib.oracle_energy_terms.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int32, P, P, P, P,
                                             P, P, P]
        _lib.oracle_run_terms.argtypes = (
            [ctypes.c_int32, P, P, P, P, ctypes.c_int32, P, P, P, P, P,
             ctypes.c_int32, P, ctypes.c_int32, P,
             ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
             P, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32]
            + [P] * 3 + [P] * 4 + [P] * 4 + [P, P, ctypes.c_int64])
        _lib.oracle_run_terms.restype = ctypes.c_int
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def philox(ctr, key):
    lib = _load()
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def color_rank(color):
    lib = _load()
    color = _c(color, np.int32)
    rank = np.zeros(color.shape[0], dtype=np.int32)
    n_pad = np.zeros(1, dtype=np.int32)
    rc = lib.oracle_color_rank(color.shape[0], _p(color), _p(rank), _p(n_pad))
    if rc:
        raise ValueError("bad colouring")
    return rank, int(n_pad[0])


def _terms(inst):
    """The instance's general constraint terms as contiguous arrays, or None
    when its constraint is copy edges."""
    if getattr(inst, "term_ptr", None) is None:
        return None
    return (_c(inst.term_ptr, np.int32), _c(inst.term_idx, np.int32),
            _c(inst.term_coef, np.int32), _c(inst.term_const, np.int32))


def energy(inst, s):
    """(f_q, g) of one physical state under the instance's couplings and
    constraint."""
    lib = _load()
    s = _c(s, np.int8)
    f = np.zeros(1, dtype=np.int64)
    g = np.zeros(1, dtype=np.int64)
    rp, col, J, b = (_c(inst.row_ptr, np.int32), _c(inst.col, np.int32),
                     _c(inst.J_q, np.int32), _c(inst.b_q, np.int32))
    T = _terms(inst)
    if T is not None:
        tp, ti, tc, td = T
        lib.oracle_energy_terms(inst.n, _p(rp), _p(col), _p(J), _p(b), tp.shape[0] - 1, _p(tp), _p(ti),
                                _p(tc), _p(td), _p(s), _p(f), _p(g))
        return int(f[0]), int(g[0])
    ca, cb = _c(inst.copy_a, np.int32), _c(inst.copy_b, np.int32)
    lib.oracle_energy(inst.n, _p(rp), _p(col), _p(J), _p(b), ca.shape[0], _p(ca), _p(cb),
                      _p(s), _p(f), _p(g))
    return int(f[0]), int(g[0])


def pswap_exponent(beta, pq_a, pq_b, g_a, g_b):
    return _load().oracle_pswap_exponent(beta, int(pq_a), int(pq_b), int(g_a), int(g_b))


def bswap_exponent(beta_a, beta_b, e_a, e_b):
    return _load().oracle_bswap_exponent(beta_a, beta_b, int(e_a), int(e_b))


def swap_accept(x, u):
    return bool(_load().oracle_swap_accept(float(x), float(u)))


def heat_bath(beta, h_q, u):
    return int(_load().oracle_heat_bath(float(beta), int(h_q), int(u)))


def schedule(n, flags=0):
    d = np.zeros(1, dtype=np.int32)
    f = np.zeros(1, dtype=np.int32)
    _load().oracle_schedule(int(n), flags, _p(d), _p(f))
    return ("beta" if d[0] else "P"), int(f[0])


def run(inst, beta, p_q, *, mcs_per_swap, n_rounds, seed, s0=None, f_target=None,
        flags=0, trace=False, threads=1):
    """Run 2D-PT for n_rounds rounds; every output is in grid-position order.
    threads > 1 splits each round's sweeps over positions (same result)."""
    lib = _load()
    beta = _c(beta, np.float64)
    p_q = _c(p_q, np.int32)
    I, Jn = beta.shape[0], p_q.shape[0]
    R, n = I * Jn, inst.n
    rp, col, J, b = (_c(inst.row_ptr, np.int32), _c(inst.col, np.int32),
                     _c(inst.J_q, np.int32), _c(inst.b_q, np.int32))
    ca, cb = _c(inst.copy_a, np.int32), _c(inst.copy_b, np.int32)
    color = _c(inst.color, np.int32)
    s0a = None if s0 is None else _c(s0, np.int8).reshape(-1)
    if s0a is not None and s0a.shape[0] != R * n:
        raise ValueError("s0 must hold R*n spins")
    states = np.zeros(R * n, dtype=np.int8)
    f = np.zeros(R, dtype=np.int64)
    g = np.zeros(R, dtype=np.int64)
    best = np.zeros(n, dtype=np.int8)
    scal = np.zeros(3, dtype=np.int64)
    p_att = np.zeros(max(I * (Jn - 1), 1), dtype=np.int64)
    p_acc = np.zeros_like(p_att)
    b_att = np.zeros(max(Jn * (I - 1), 1), dtype=np.int64)
    b_acc = np.zeros_like(b_att)
    tcap = int(n_rounds) if trace else 0
    tf = np.zeros(max(tcap, 1), dtype=np.int64)
    tg = np.zeros(max(tcap, 1), dtype=np.int64)
    sc = [scal[i:i + 1] for i in range(3)]
    tail = (_p(color),
            I, _p(beta), Jn, _p(p_q), int(mcs_per_swap), int(n_rounds), int(seed) & (2**64 - 1),
            _p(s0a), 0 if f_target is None else 1, 0 if f_target is None else int(f_target), flags,
            _p(states), _p(f), _p(g), _p(best), _p(sc[0]), _p(sc[1]), _p(sc[2]),
            _p(p_att), _p(p_acc), _p(b_att), _p(b_acc), _p(tf), _p(tg), tcap)
    T = _terms(inst)
    lib.oracle_set_threads(int(threads))
    try:
        if T is not None:
            tp, ti, tc, td = T
            rc = lib.oracle_run_terms(n, _p(rp), _p(col), _p(J), _p(b), tp.shape[0] - 1, _p(tp),
                                      _p(ti), _p(tc), _p(td), *tail)
        else:
            rc = lib.oracle_run(n, _p(rp), _p(col), _p(J), _p(b), ca.shape[0], _p(ca), _p(cb), *tail)
    finally:
        lib.oracle_set_threads(1)
    if rc:
        raise RuntimeError("oracle_run failed with code %d" % rc)
    return {
        "states": states.reshape(R, n), "f": f, "g": g, "best_state": best,
        "best_f": int(scal[0]), "best_sweep": int(scal[1]), "first_hit": int(scal[2]),
        "p_att": p_att[:I * (Jn - 1)].reshape(I, max(Jn - 1, 0)),
        "p_acc": p_acc[:I * (Jn - 1)].reshape(I, max(Jn - 1, 0)),
        "b_att": b_att[:Jn * (I - 1)].reshape(Jn, max(I - 1, 0)),
        "b_acc": b_acc[:Jn * (I - 1)].reshape(Jn, max(I - 1, 0)),
        "trace_f": tf[:tcap], "trace_g": tg[:tcap],
    }
