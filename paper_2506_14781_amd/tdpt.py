"""Python binding of libtdpt.so (the C ABI declared in include/tdpt.h).

Argument marshalling only: every step of 2D parallel tempering runs in the
library's gfx950 kernels.  PyTorch supplies the device workspace (a uint8
tensor) and the HIP stream.  There is no fallback: if the library is not
built, or no GPU is present, the calls that need it raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TDPT_LIB names another build of the same sources (the host-sanitizer test
# loads an AddressSanitizer / UBSan build of the host code this way)
LIB_PATH = os.environ.get("TDPT_LIB") or os.path.join(_HERE, "_build", "libtdpt.so")

OK, E_INVALID, E_RANGE, E_NOMEM, E_DEVICE, E_STATE, E_BUSY = range(7)
NO_PSWAP = 1

EXPORTED = [
    "tdpt_instance_create", "tdpt_instance_create_terms", "tdpt_instance_info_get",
    "tdpt_instance_destroy",
    "tdpt_workspace_bytes", "tdpt_problem_create", "tdpt_problem_run", "tdpt_problem_query",
    "tdpt_problem_read_energies", "tdpt_problem_read_states", "tdpt_problem_read_perm",
    "tdpt_problem_read_best", "tdpt_problem_read_counters", "tdpt_problem_read_trace",
    "tdpt_problem_save", "tdpt_problem_load", "tdpt_problem_destroy", "tdpt_last_error",
    "tdpt_problem_set_timing", "tdpt_problem_read_timing",
    "tdpt_batch_workspace_bytes", "tdpt_batch_create", "tdpt_batch_set_members",
    "tdpt_batch_run", "tdpt_batch_destroy", "tdpt_problem_autotune", "tdpt_batch_autotune",
    "tdpt_batch_set_graph", "tdpt_batch_set_driver", "tdpt_batch_query_driver",
    "tdpt_layout_get", "tdpt_problem_query_async", "tdpt_problem_read_energies_async",
    "tdpt_problem_read_states_async", "tdpt_problem_read_best_async", "tdpt_problem_read_best_logical",
    "tdpt_problem_read_histogram", "tdpt_problem_create_static", "tdpt_problem_set_stage_trace",
    "tdpt_batch_query", "tdpt_batch_query_async",
]

STATIC_WORKSPACE_BYTES = 64 << 20


class TdptError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tdpt error {code}: {msg}")
        self.code = code


class _RunCfg(ctypes.Structure):
    _fields_ = [
        ("n_beta", ctypes.c_int32), ("beta", ctypes.c_void_p),
        ("n_p", ctypes.c_int32), ("p_q", ctypes.c_void_p),
        ("mcs_per_swap", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("s0", ctypes.c_void_p), ("has_target", ctypes.c_int32),
        ("f_target_q", ctypes.c_int64), ("flags", ctypes.c_uint32),
        ("trace_cap", ctypes.c_int64), ("hist_logical", ctypes.c_int32),
    ]


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_pad", ctypes.c_int32), ("n_colors", ctypes.c_int32),
                ("max_degree", ctypes.c_int32), ("max_copy_degree", ctypes.c_int32),
                ("narrow", ctypes.c_int32), ("nnz", ctypes.c_int64), ("m", ctypes.c_int32),
                ("n_terms", ctypes.c_int32), ("max_constraint_degree", ctypes.c_int32),
                ("n_logical", ctypes.c_int32)]


class _Layout(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_int32), ("narrow", ctypes.c_int32), ("general", ctypes.c_int32),
                ("ell_width", ctypes.c_int32), ("group_key", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("held", ctypes.c_int32), ("per_round", ctypes.c_int32),
                ("spin", ctypes.c_int32), ("pair16", ctypes.c_int32)]


class _TuneReport(ctypes.Structure):
    _fields_ = [("driver", ctypes.c_int32), ("block", ctypes.c_int32), ("ms_per_round", ctypes.c_double),
                ("n_trials", ctypes.c_int32), ("trial_driver", ctypes.c_int32 * 32),
                ("trial_block", ctypes.c_int32 * 32), ("trial_ms_per_round", ctypes.c_double * 32),
                ("slots", ctypes.c_int32), ("trial_slots", ctypes.c_int32 * 32), ("spin", ctypes.c_int32),
                ("trial_spin", ctypes.c_int32 * 32)]


class _BatchTuneReport(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int32), ("n_groups", ctypes.c_int32), ("group_block", ctypes.c_int32 * 32),
                ("group_ms_per_round", ctypes.c_double * 32), ("n_trials", ctypes.c_int32),
                ("trial_group", ctypes.c_int32 * 128), ("trial_block", ctypes.c_int32 * 128),
                ("trial_ms_per_round", ctypes.c_double * 128), ("group_slots", ctypes.c_int32 * 32),
                ("trial_slots", ctypes.c_int32 * 128), ("group_spin", ctypes.c_int32 * 32),
                ("trial_spin", ctypes.c_int32 * 128)]


class _Status(ctypes.Structure):
    _fields_ = [("rounds_done", ctypes.c_int64), ("sweeps_done", ctypes.c_int64),
                ("first_hit_sweep", ctypes.c_int64), ("best_f_q", ctypes.c_int64),
                ("best_sweep", ctypes.c_int64), ("driver", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("spin", ctypes.c_int32)]


_lib = None


def load_library():
    """Load libtdpt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2506_14781_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "tdpt_instance_create": [I32, P, P, P, P, I32, P, P, P, P, P],
        "tdpt_instance_create_terms": [I32, P, P, P, P, I32, P, P, P, P, P, P, P],
        "tdpt_layout_get": [P, P, P],
        "tdpt_problem_query_async": [P, P],
        "tdpt_problem_read_energies_async": [P, P, P],
        "tdpt_problem_read_states_async": [P, P],
        "tdpt_problem_read_best_async": [P, P, P],
        "tdpt_problem_read_best_logical": [P, P, P, P],
        "tdpt_problem_read_histogram": [P, P, P],
        "tdpt_problem_create_static": [P, P, P, P],
        "tdpt_problem_set_stage_trace": [P, P, I32],
        "tdpt_batch_query": [P, P],
        "tdpt_batch_query_async": [P, P],
        "tdpt_instance_info_get": [P, P],
        "tdpt_workspace_bytes": [P, P, P],
        "tdpt_problem_create": [P, P, P, SZ, P, P],
        "tdpt_problem_run": [P, I64],
        "tdpt_problem_query": [P, P],
        "tdpt_problem_read_energies": [P, P, P],
        "tdpt_problem_read_states": [P, P],
        "tdpt_problem_read_perm": [P, P],
        "tdpt_problem_read_best": [P, P, P, P],
        "tdpt_problem_read_counters": [P, P, P, P, P],
        "tdpt_problem_read_trace": [P, P, P, P],
        "tdpt_problem_save": [P, P, P],
        "tdpt_problem_load": [P, P, SZ],
        "tdpt_problem_set_timing": [P, I32],
        "tdpt_problem_read_timing": [P, P, P, P],
        "tdpt_batch_workspace_bytes": [I32, P],
        "tdpt_batch_create": [I32, P, SZ, P, P],
        "tdpt_batch_set_members": [P, P, I32],
        "tdpt_batch_run": [P, I64],
        "tdpt_problem_autotune": [P, I32, P],
        "tdpt_batch_autotune": [P, I32, P],
        "tdpt_batch_set_graph": [P, I32],
        "tdpt_batch_set_driver": [P, I32],
        "tdpt_batch_query_driver": [P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.tdpt_instance_destroy.argtypes = [P]
    lib.tdpt_instance_destroy.restype = None
    lib.tdpt_problem_destroy.argtypes = [P]
    lib.tdpt_problem_destroy.restype = None
    lib.tdpt_batch_destroy.argtypes = [P]
    lib.tdpt_batch_destroy.restype = None
    lib.tdpt_last_error.argtypes = []
    lib.tdpt_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        raise TdptError(rc, load_library().tdpt_last_error().decode())


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _dptr(t):
    """Device address of a torch tensor (None stays NULL)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _arr(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


class Instance:
    """A validated, colour-major re-laid-out instance (host memory).

    The constraint is either copy edges (copy_a, copy_b) or general terms
    (terms = (term_ptr, term_idx, term_coef, term_const)); see
    tdpt_instance_create_terms."""

    def __init__(self, n, row_ptr, col, J_q, b_q, copy_a, copy_b, color, terms=None, logical_of=None):
        lib = load_library()
        self._keep = [_arr(row_ptr, np.int32), _arr(col, np.int32), _arr(J_q, np.int32),
                      _arr(b_q, np.int32), _arr(copy_a, np.int32), _arr(copy_b, np.int32),
                      _arr(color, np.int32), _arr(logical_of, np.int32)]
        rp, cl, jq, bq, ca, cb, co, lo = self._keep
        h = ctypes.c_void_p()
        if terms is not None:
            tp, ti, tc, td = (_arr(x, np.int32) for x in terms)
            self._keep += [tp, ti, tc, td]
            _check(lib.tdpt_instance_create_terms(int(n), _ptr(rp), _ptr(cl), _ptr(jq), _ptr(bq),
                                                  int(tp.shape[0]) - 1, _ptr(tp), _ptr(ti), _ptr(tc),
                                                  _ptr(td), _ptr(co), _ptr(lo), ctypes.byref(h)))
        else:
            m = 0 if ca is None else int(ca.shape[0])
            _check(lib.tdpt_instance_create(int(n), _ptr(rp), _ptr(cl), _ptr(jq), _ptr(bq), m,
                                            _ptr(ca), _ptr(cb), _ptr(co), _ptr(lo), ctypes.byref(h)))
        self._h = h
        self.n = int(n)

    @classmethod
    def from_synth(cls, inst, logical=False):
        """From a synth Instance; logical=True also passes its logical_of."""
        terms = None
        if getattr(inst, "term_ptr", None) is not None:
            terms = (inst.term_ptr, inst.term_idx, inst.term_coef, inst.term_const)
        return cls(inst.n, inst.row_ptr, inst.col, inst.J_q, inst.b_q, inst.copy_a,
                   inst.copy_b, inst.color, terms=terms,
                   logical_of=inst.logical_of if logical else None)

    def info(self) -> dict:
        out = _Info()
        _check(load_library().tdpt_instance_info_get(self._h, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in _Info._fields_}

    def layout(self, cfg: "RunConfig") -> dict:
        """The structure layout (and batch group key) a problem would run with."""
        out = _Layout()
        c = cfg._c()
        _check(load_library().tdpt_layout_get(self._h, ctypes.byref(c), ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in _Layout._fields_}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.tdpt_instance_destroy(h)
            self._h = None


class RunConfig:
    def __init__(self, beta, p_q, *, mcs_per_swap, seed, s0=None, f_target=None, flags=0,
                 trace_cap=0, hist_logical=False):
        self.beta = _arr(beta, np.float64)
        self.p_q = _arr(p_q, np.int32)
        self.s0 = None if s0 is None else _arr(s0, np.int8).reshape(-1)
        self.mcs_per_swap = int(mcs_per_swap)
        self.seed = int(seed) & (2**64 - 1)
        self.f_target = f_target
        self.flags = int(flags)
        self.trace_cap = int(trace_cap)
        self.hist_logical = bool(hist_logical)

    def _c(self):
        c = _RunCfg()
        c.n_beta = self.beta.shape[0]
        c.beta = self.beta.ctypes.data
        c.n_p = self.p_q.shape[0]
        c.p_q = self.p_q.ctypes.data
        c.mcs_per_swap = self.mcs_per_swap
        c.seed = self.seed
        c.s0 = None if self.s0 is None else self.s0.ctypes.data
        c.has_target = 0 if self.f_target is None else 1
        c.f_target_q = 0 if self.f_target is None else int(self.f_target)
        c.flags = self.flags
        c.trace_cap = self.trace_cap
        c.hist_logical = 1 if self.hist_logical else 0
        return c

    @property
    def replicas(self):
        return self.beta.shape[0] * self.p_q.shape[0]


def workspace_bytes(instance: Instance, cfg: RunConfig) -> int:
    out = ctypes.c_size_t()
    c = cfg._c()
    _check(load_library().tdpt_workspace_bytes(instance._h, ctypes.byref(c), ctypes.byref(out)))
    return out.value


class Problem:
    """One 2D-PT run resident on the GPU; outputs are per grid position."""

    def __init__(self, instance: Instance, cfg: RunConfig, device="cuda", stream=None, static=False):
        """static=True: the workspace is the library's static device array
        (tdpt_problem_create_static; nothing is allocated, one such problem
        per GPU at a time)."""
        import torch
        lib = load_library()
        self.cfg = cfg
        self.n = instance.n
        self.I, self.J = cfg.beta.shape[0], cfg.p_q.shape[0]
        self.R = self.I * self.J
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        c = cfg._c()
        if static:
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(lib.tdpt_problem_create_static(instance._h, ctypes.byref(c),
                                                      ctypes.c_void_p(self.stream.cuda_stream),
                                                      ctypes.byref(h)))
        else:
            nbytes = workspace_bytes(instance, cfg)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            _check(lib.tdpt_problem_create(instance._h, ctypes.byref(c),
                                           ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.n_logical = instance.info()["n_logical"]

    def run(self, n_rounds: int):
        _check(_lib.tdpt_problem_run(self._h, int(n_rounds)))

    def query(self) -> dict:
        s = _Status()
        _check(_lib.tdpt_problem_query(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _Status._fields_}

    def energies(self):
        f = np.zeros(self.R, dtype=np.int64)
        g = np.zeros(self.R, dtype=np.int64)
        _check(_lib.tdpt_problem_read_energies(self._h, _ptr(f), _ptr(g)))
        return f, g

    def states(self):
        s = np.zeros((self.R, self.n), dtype=np.int8)
        _check(_lib.tdpt_problem_read_states(self._h, _ptr(s)))
        return s

    def perm(self):
        p = np.zeros(self.R, dtype=np.int32)
        _check(_lib.tdpt_problem_read_perm(self._h, _ptr(p)))
        return p

    def best(self):
        s = np.zeros(self.n, dtype=np.int8)
        f = np.zeros(1, dtype=np.int64)
        w = np.zeros(1, dtype=np.int64)
        _check(_lib.tdpt_problem_read_best(self._h, _ptr(s), _ptr(f), _ptr(w)))
        return s, int(f[0]), int(w[0])

    def best_logical(self):
        """The best feasible bottom-right state decoded to its logical
        variables (each read from its lowest-numbered copy), its f_q, sweep."""
        x = np.zeros(max(self.n_logical, 1), dtype=np.int8)
        f = np.zeros(1, dtype=np.int64)
        w = np.zeros(1, dtype=np.int64)
        _check(_lib.tdpt_problem_read_best_logical(self._h, _ptr(x), _ptr(f), _ptr(w)))
        return x[:self.n_logical], int(f[0]), int(w[0])

    def histogram(self):
        """(counts[2^N], samples) of the bottom-right replica's logical state,
        one sample per round (RunConfig(hist_logical=True))."""
        counts = np.zeros(1 << self.n_logical, dtype=np.uint32)
        k = np.zeros(1, dtype=np.int64)
        _check(_lib.tdpt_problem_read_histogram(self._h, _ptr(counts), _ptr(k)))
        return counts, int(k[0])

    def energies_async(self, f, g):
        """Enqueue f, g per position into device tensors (int64[R]) on the
        problem's stream."""
        _check(_lib.tdpt_problem_read_energies_async(self._h, _dptr(f), _dptr(g)))

    def states_async(self, s):
        """Enqueue the states per position into a device tensor (int8[R, n])."""
        _check(_lib.tdpt_problem_read_states_async(self._h, _dptr(s)))

    def best_async(self, s, f_sweep):
        """Enqueue the best state (int8[n]) and (best_f_q, best_sweep) (int64[2])."""
        _check(_lib.tdpt_problem_read_best_async(self._h, _dptr(s), _dptr(f_sweep)))

    def query_async(self, words):
        """Enqueue rounds_done, first_hit_sweep, best_f_q, best_sweep (int64[4])."""
        _check(_lib.tdpt_problem_query_async(self._h, _dptr(words)))

    def counters(self):
        I, J = self.I, self.J
        pa = np.zeros(max(I * (J - 1), 1), dtype=np.int64)
        pc = np.zeros_like(pa)
        ba = np.zeros(max(J * (I - 1), 1), dtype=np.int64)
        bc = np.zeros_like(ba)
        _check(_lib.tdpt_problem_read_counters(self._h, _ptr(pa), _ptr(pc), _ptr(ba), _ptr(bc)))
        return (pa[:I * (J - 1)].reshape(I, J - 1), pc[:I * (J - 1)].reshape(I, J - 1),
                ba[:J * (I - 1)].reshape(J, I - 1), bc[:J * (I - 1)].reshape(J, I - 1))

    def trace(self):
        cap = max(self.cfg.trace_cap, 1)
        f = np.zeros(cap, dtype=np.int64)
        g = np.zeros(cap, dtype=np.int64)
        c = np.zeros(1, dtype=np.int64)
        _check(_lib.tdpt_problem_read_trace(self._h, _ptr(f), _ptr(g), _ptr(c)))
        k = int(c[0])
        return f[:k], g[:k]

    def save(self) -> bytes:
        size = ctypes.c_size_t()
        _check(_lib.tdpt_problem_save(self._h, None, ctypes.byref(size)))
        buf = (ctypes.c_uint8 * size.value)()
        _check(_lib.tdpt_problem_save(self._h, buf, ctypes.byref(size)))
        return bytes(buf)

    def load(self, blob: bytes):
        buf = (ctypes.c_uint8 * len(blob)).from_buffer_copy(blob)
        _check(_lib.tdpt_problem_load(self._h, buf, len(blob)))

    def autotune(self, rounds_per_trial: int = 10) -> dict:
        """Time the admissible launch shapes (driver, workgroup size, replicas
        per workgroup) on this problem and keep the fastest; the problem's
        state is left as it was.  Trials are (driver, threads, replicas per
        workgroup, ms per round)."""
        r = _TuneReport()
        _check(_lib.tdpt_problem_autotune(self._h, int(rounds_per_trial), ctypes.byref(r)))
        k = r.n_trials
        return {"driver": r.driver, "block": r.block, "slots": r.slots, "spin": r.spin,
                "ms_per_round": r.ms_per_round,
                "trials": [(r.trial_driver[i], r.trial_block[i], r.trial_slots[i], r.trial_ms_per_round[i])
                           for i in range(k)],
                "trial_spin": [r.trial_spin[i] for i in range(k)]}

    def set_stage_trace(self, buf, rounds: int):
        """Persistent driver: per-round, per-slot stage timestamps (100 MHz
        clock) into a device int64 tensor of rounds * R * 4 (None, 0: off)."""
        if rounds and (buf is None or buf.numel() < rounds * self.R * 4):
            raise ValueError("the buffer needs rounds * R * 4 entries")
        _check(_lib.tdpt_problem_set_stage_trace(self._h, _dptr(buf), int(rounds)))

    def set_timing(self, every: int):
        """Time every `every`-th sweep-kernel launch with HIP events (0: off)."""
        _check(_lib.tdpt_problem_set_timing(self._h, int(every)))

    def timing(self):
        """(total ms of the timed launches, launches timed, rounds they covered)."""
        ms = ctypes.c_double()
        k = ctypes.c_int64()
        r = ctypes.c_int64()
        _check(_lib.tdpt_problem_read_timing(self._h, ctypes.byref(ms), ctypes.byref(k),
                                             ctypes.byref(r)))
        return ms.value, k.value, r.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.tdpt_problem_destroy(h)
        self._h = None

    def __del__(self):
        self.close()


class Batch:
    """Advance many problems together: one sweep launch and one swap launch
    per round for all members."""

    def __init__(self, max_members: int, device="cuda", stream=None):
        import torch
        lib = load_library()
        size = ctypes.c_size_t()
        _check(lib.tdpt_batch_workspace_bytes(int(max_members), ctypes.byref(size)))
        self.device = torch.device(device)
        self.workspace = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib.tdpt_batch_create(int(max_members), ctypes.c_void_p(self.workspace.data_ptr()),
                                     size.value, ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(h)))
        self._h = h
        self.members = []

    def set_members(self, problems):
        self.members = list(problems)
        arr = (ctypes.c_void_p * max(len(self.members), 1))(*[p._h.value for p in self.members])
        _check(_lib.tdpt_batch_set_members(self._h, arr, len(self.members)))

    def run(self, n_rounds: int):
        _check(_lib.tdpt_batch_run(self._h, int(n_rounds)))

    def query(self):
        """Status of every member at once, in set_members order: int64
        [count, 4] = rounds_done, first_hit_sweep, best_f_q, best_sweep."""
        out = np.zeros((max(len(self.members), 1), 4), dtype=np.int64)
        _check(_lib.tdpt_batch_query(self._h, _ptr(out)))
        return out[:len(self.members)]

    def query_async(self, words):
        """Enqueue the same status words into a device int64 tensor [count, 4]."""
        _check(_lib.tdpt_batch_query_async(self._h, _dptr(words)))

    def set_driver(self, driver: int):
        """-1: persistent driver when it fits (default); 0: per-round launches."""
        _check(_lib.tdpt_batch_set_driver(self._h, int(driver)))

    def driver(self) -> int:
        """1 if runs use the persistent driver, else 0."""
        d = ctypes.c_int32()
        _check(_lib.tdpt_batch_query_driver(self._h, ctypes.byref(d)))
        return d.value

    def set_graph(self, rounds_per_graph: int):
        """Replay runs from a HIP graph of this many rounds (0: direct launches)."""
        _check(_lib.tdpt_batch_set_graph(self._h, int(rounds_per_graph)))

    def autotune(self, rounds_per_trial: int = 3) -> dict:
        """Pick each layout group's workgroup size and replicas per workgroup
        by timing batch rounds; every member's state is left as it was.
        Trials are (group, threads, replicas per workgroup, ms per round)."""
        r = _BatchTuneReport()
        _check(_lib.tdpt_batch_autotune(self._h, int(rounds_per_trial), ctypes.byref(r)))
        g, k = r.n_groups, r.n_trials
        return {"persistent": r.persistent, "group_block": list(r.group_block[:g]),
                "group_slots": list(r.group_slots[:g]), "group_spin": list(r.group_spin[:g]),
                "group_ms_per_round": list(r.group_ms_per_round[:g]),
                "trials": [(r.trial_group[i], r.trial_block[i], r.trial_slots[i], r.trial_ms_per_round[i])
                           for i in range(k)],
                "trial_spin": [r.trial_spin[i] for i in range(k)]}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.tdpt_batch_destroy(h)
        self._h = None

    def __del__(self):
        self.close()
