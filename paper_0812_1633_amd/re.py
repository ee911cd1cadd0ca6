"""Python binding of the replica-exchange LJ engine (``include/re.h``).

Argument marshalling only: every step of the method runs in the HIP library
``libre_hip.so``.  Loading fails loudly when the library has not been built;
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libre_hip.so")

RE_OK, RE_EINVAL, RE_ENOMEM, RE_EDEVICE, RE_ETIMEOUT, RE_ESTATE, RE_EOVERFLOW = 0, -1, -2, -3, -4, -5, -6
RE_LANGEVIN, RE_SVR = 0, 1
RE_MIXED, RE_FP64 = 0, 1
RE_BATCHED, RE_PLAIN = 0, 1
RE_LOCKSTEP, RE_PERSISTENT = 0, 1
RE_SYNC, RE_ASYNC = 0, 1
RE_BARRIER_AUTO, RE_BARRIER_AGENT = 0, 1

_ERRNAMES = {RE_EINVAL: "RE_EINVAL", RE_ENOMEM: "RE_ENOMEM", RE_EDEVICE: "RE_EDEVICE",
             RE_ETIMEOUT: "RE_ETIMEOUT", RE_ESTATE: "RE_ESTATE", RE_EOVERFLOW: "RE_EOVERFLOW"}


class ReError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "?"), code, msg))
        self.code = code


class Options(C.Structure):
    _fields_ = [("thermostat", C.c_int), ("gamma", C.c_double), ("gamma_set", C.c_int),
                ("precision", C.c_int), ("form", C.c_int), ("batched_engine", C.c_int),
                ("exchange_mode", C.c_int), ("rho_per_replica", C.POINTER(C.c_double)),
                ("stream", C.c_void_p), ("watchdog_seconds", C.c_double),
                ("log_capacity", C.c_int64), ("threads_per_atom", C.c_int), ("block_size", C.c_int),
                ("team_size", C.c_int), ("tune_cache", C.c_char_p), ("autotune", C.c_int),
                ("team_barrier", C.c_int), ("svr_tau", C.c_double), ("exchange_max_distance", C.c_int),
                ("debug_delay_us", C.c_int), ("threads_per_atom_per_replica", C.POINTER(C.c_int32)),
                ("team_balance", C.c_int)]


class XLogRec(C.Structure):
    _fields_ = [("attempt", C.c_int64), ("master", C.c_int32), ("slot_lo", C.c_int32),
                ("rep_a", C.c_int32), ("rep_b", C.c_int32), ("step_a", C.c_int64),
                ("step_b", C.c_int64), ("U_a", C.c_double), ("U_b", C.c_double),
                ("T_a", C.c_double), ("T_b", C.c_double), ("u", C.c_double),
                ("accepted", C.c_int32), ("slot_hi", C.c_int32)]


_lib = None


def lib():
    """Load libre_hip.so (built by ``paper_0812_1633_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libre_hip.so is not built: run `python -m paper_0812_1633_amd.build` "
                              "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        L.re_create.argtypes = [C.POINTER(vp), C.c_int, vp, vp, dbl, dbl, dbl, dbl, C.c_int, u64,
                                C.POINTER(Options)]
        L.re_step.argtypes = [vp, i64]
        L.re_exchange.argtypes = [vp]
        for f in ("re_query_energies", "re_query_temps", "re_query_slots", "re_query_box"):
            getattr(L, f).argtypes = [vp, vp]
        L.re_query_acceptance.argtypes = [vp, vp, vp]
        L.re_query_steps.argtypes = [vp, vp, vp]
        L.re_query_attempt_count.argtypes = [vp, C.POINTER(i64)]
        L.re_query_exchange_log.argtypes = [vp, vp, i64, C.POINTER(i64), C.POINTER(i64)]
        L.re_get_state.argtypes = [vp, C.c_int, vp, vp]
        L.re_set_state.argtypes = [vp, C.c_int, vp, vp]
        L.re_compute_forces.argtypes = [vp, C.c_int, vp, vp]
        L.re_query_forces.argtypes = [vp, C.c_int, vp]
        L.re_set_schedule.argtypes = [vp, vp, i64]
        L.re_test_exchange.argtypes = [vp, vp, vp, C.c_int, u64, i64, C.c_int, vp]
        L.re_test_exchange_noalloc.argtypes = [vp, vp, vp, C.c_int, u64, i64, C.c_int, vp]
        L.re_test_philox.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_int, vp]
        L.re_test_normals.argtypes = [C.c_int, u64, vp, C.c_int, vp]
        L.re_profile.argtypes = [vp, C.c_int]
        L.re_query_config.argtypes = [vp, vp, vp, vp]
        L.re_query_lanes.argtypes = [vp, vp]
        L.re_query_teams.argtypes = [vp, vp]
        L.re_query_kernel_time.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64)]
        L.re_destroy.argtypes = [vp]
        L.re_destroy.restype = None
        L.re_last_error.argtypes = [vp]
        L.re_last_error.restype = C.c_char_p
        for f in ("re_create", "re_step", "re_exchange", "re_query_energies", "re_query_temps",
                  "re_query_slots", "re_query_box", "re_query_acceptance", "re_query_steps",
                  "re_query_exchange_log", "re_get_state", "re_set_state", "re_compute_forces",
                  "re_set_schedule", "re_test_exchange", "re_test_philox", "re_test_normals",
                  "re_profile", "re_query_kernel_time", "re_query_config", "re_query_attempt_count",
                  "re_query_forces", "re_test_exchange_noalloc", "re_query_lanes", "re_query_teams"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _check(rc, ctx=None):
    if rc != RE_OK:
        msg = lib().re_last_error(ctx)
        raise ReError(rc, msg.decode() if msg else "")


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # a torch.cuda.Stream


class Engine:
    """A replica-exchange run (``re_create`` .. ``re_destroy``).

    N: atoms per replica (sequence of R ints); T_ladder: ascending ladder.
    precision: "mixed" | "fp64"; form: "batched" | "plain";
    engine: "persistent" | "lockstep"; exchange: "sync" | "async".
    thermostat: "langevin" (friction gamma) | "svr" (stochastic velocity
    rescaling, relaxation time svr_tau; 0 = 0.5).
    exchange_max_distance: largest ladder distance of an exchange pair (1:
    alternating nearest neighbours).
    debug_delay_us: test hook (persistent engine): workgroups pause for up to
    this many microseconds after team barriers (0: off).
    threads_per_atom_per_replica: R force lane counts (1, 2, 4, 8), one per
    replica (None: threads_per_atom for all).
    team_balance: persistent engine, automatic team sizes: re-plan the teams
    from the measured list-update rates (off by default: teams proportional
    to N).
    """

    def __init__(self, N, T_ladder, rho, r_c, skin, dt, N_x, seed, *, gamma=None, precision="mixed",
                 form="batched", engine="persistent", exchange="sync", rho_per_replica=None, stream=None,
                 watchdog_seconds=0.0, log_capacity=0, threads_per_atom=0, block_size=0, team_size=0,
                 tune_cache=None, autotune=False, team_barrier="auto", thermostat="langevin", svr_tau=0.0,
                 exchange_max_distance=1, debug_delay_us=0, threads_per_atom_per_replica=None,
                 team_balance=False):
        self._ctx = None
        N = np.ascontiguousarray(N, np.int32)
        T = np.ascontiguousarray(T_ladder, np.float64)
        self.R = int(N.size)
        self.N = N.copy()
        o = Options()
        if gamma is not None:
            o.gamma, o.gamma_set = float(gamma), 1
        o.precision = {"mixed": RE_MIXED, "fp64": RE_FP64}[precision]
        o.form = {"batched": RE_BATCHED, "plain": RE_PLAIN}[form]
        o.batched_engine = {"persistent": RE_PERSISTENT, "lockstep": RE_LOCKSTEP}[engine]
        o.exchange_mode = {"sync": RE_SYNC, "async": RE_ASYNC}[exchange]
        self._rho = None
        if rho_per_replica is not None:
            self._rho = np.ascontiguousarray(rho_per_replica, np.float64)
            o.rho_per_replica = self._rho.ctypes.data_as(C.POINTER(C.c_double))
        o.stream = _stream_handle(stream)
        o.watchdog_seconds = float(watchdog_seconds)
        o.log_capacity = int(log_capacity)
        o.threads_per_atom = int(threads_per_atom)
        o.block_size = int(block_size)
        o.team_size = int(team_size)
        o.tune_cache = tune_cache.encode() if tune_cache else None
        o.autotune = 1 if autotune else 0
        o.team_barrier = {"auto": RE_BARRIER_AUTO, "agent": RE_BARRIER_AGENT}[team_barrier]
        o.thermostat = {"langevin": RE_LANGEVIN, "svr": RE_SVR}[thermostat]
        o.svr_tau = float(svr_tau)
        o.exchange_max_distance = int(exchange_max_distance)
        o.debug_delay_us = int(debug_delay_us)
        o.team_balance = 1 if team_balance else 0
        self._tpa_r = None
        if threads_per_atom_per_replica is not None:
            self._tpa_r = np.ascontiguousarray(threads_per_atom_per_replica, np.int32)
            o.threads_per_atom_per_replica = self._tpa_r.ctypes.data_as(C.POINTER(C.c_int32))
        ctx = C.c_void_p()
        rc = lib().re_create(C.byref(ctx), self.R, _ptr(N), _ptr(T), float(rho), float(r_c), float(skin),
                             float(dt), int(N_x), int(seed), C.byref(o))
        _check(rc, None)
        self._ctx = ctx
        self.T_ladder = T.copy()
        self.precision, self.form, self.engine, self.exchange_mode = precision, form, engine, exchange

    # lifetime
    def close(self):
        if self._ctx is not None:
            lib().re_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # stepping
    def step(self, n):
        _check(lib().re_step(self._ctx, int(n)), self._ctx)

    def exchange(self):
        _check(lib().re_exchange(self._ctx), self._ctx)

    def set_schedule(self, join):
        j = np.ascontiguousarray(join, np.int64)
        _check(lib().re_set_schedule(self._ctx, _ptr(j), int(j.shape[0])), self._ctx)

    # queries
    def query_energies(self):
        U = np.zeros(self.R)
        _check(lib().re_query_energies(self._ctx, _ptr(U)), self._ctx)
        return U

    def query_temps(self):
        T = np.zeros(self.R)
        _check(lib().re_query_temps(self._ctx, _ptr(T)), self._ctx)
        return T

    def query_slots(self):
        s = np.zeros(self.R, np.int32)
        _check(lib().re_query_slots(self._ctx, _ptr(s)), self._ctx)
        return s

    def query_box(self):
        L = np.zeros(self.R)
        _check(lib().re_query_box(self._ctx, _ptr(L)), self._ctx)
        return L

    def query_acceptance(self):
        n = max(1, self.R - 1)
        a = np.zeros(n, np.int64)
        b = np.zeros(n, np.int64)
        _check(lib().re_query_acceptance(self._ctx, _ptr(a), _ptr(b)), self._ctx)
        return a[: self.R - 1], b[: self.R - 1]

    def query_steps(self):
        s = np.zeros(self.R, np.int64)
        r = np.zeros(self.R, np.int64)
        _check(lib().re_query_steps(self._ctx, _ptr(s), _ptr(r)), self._ctx)
        return s, r

    def query_attempt_count(self):
        """Exchange attempts made so far (the next attempt's index)."""
        n = C.c_int64()
        _check(lib().re_query_attempt_count(self._ctx, C.byref(n)), self._ctx)
        return n.value

    def query_exchange_log(self, cap=1 << 20):
        buf = (XLogRec * max(1, cap))()
        n = C.c_int64()
        tot = C.c_int64()
        _check(lib().re_query_exchange_log(self._ctx, C.cast(buf, C.c_void_p), int(cap), C.byref(n),
                                           C.byref(tot)), self._ctx)
        return [buf[i] for i in range(n.value)], tot.value

    def _n(self, r):
        # out-of-range replicas reach the library, which rejects them
        return int(self.N[r]) if 0 <= r < self.R else 0

    def query_config(self):
        """(engine, threads_per_atom, team_size) the context runs with."""
        e = np.zeros(1, np.int32)
        t = np.zeros(1, np.int32)
        m = np.zeros(1, np.int32)
        _check(lib().re_query_config(self._ctx, _ptr(e), _ptr(t), _ptr(m)), self._ctx)
        return ("persistent" if e[0] == RE_PERSISTENT else "lockstep"), int(t[0]), int(m[0])

    def query_lanes(self):
        """Force lanes per atom of each replica."""
        t = np.zeros(self.R, np.int32)
        _check(lib().re_query_lanes(self._ctx, _ptr(t)), self._ctx)
        return t

    def query_teams(self):
        """Persistent engine: workgroups serving each replica."""
        t = np.zeros(self.R, np.int32)
        _check(lib().re_query_teams(self._ctx, _ptr(t)), self._ctx)
        return t

    def profile(self, enable):
        _check(lib().re_profile(self._ctx, int(enable)), self._ctx)

    def query_kernel_time(self):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().re_query_kernel_time(self._ctx, C.byref(ms), C.byref(n)), self._ctx)
        return ms.value, n.value

    def get_state(self, r):
        n = self._n(r)
        x = np.zeros((n, 3))
        v = np.zeros((n, 3))
        _check(lib().re_get_state(self._ctx, int(r), _ptr(x), _ptr(v)), self._ctx)
        return x, v

    def set_state(self, r, x, v):
        x = np.ascontiguousarray(x, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        if x.size != 3 * self._n(r) or v.size != 3 * self._n(r):
            raise ReError(RE_EINVAL, "x and v need 3 N values for replica %d" % r)
        _check(lib().re_set_state(self._ctx, int(r), _ptr(x), _ptr(v)), self._ctx)

    def query_forces(self, r):
        """Forces at the current boundary as the last engine pass computed
        them (atom-id order)."""
        n = self._n(r)
        F = np.zeros((n, 3))
        _check(lib().re_query_forces(self._ctx, int(r), _ptr(F)), self._ctx)
        return F

    def compute_forces(self, r):
        n = self._n(r)
        F = np.zeros((n, 3))
        U = np.zeros(1)
        _check(lib().re_compute_forces(self._ctx, int(r), _ptr(F), _ptr(U)), self._ctx)
        return F, float(U[0])


# --------------------------------------------------------------------------
# context-free test hooks

def re_test_exchange(U, T, slot, seed, attempt, max_distance=1):
    """Device exchange rule on given energies/ladder/slots: decisions per
    pair by its lower slot (255 = not the lower slot of a pair in this
    attempt's pattern)."""
    U = np.ascontiguousarray(U, np.float64)
    T = np.ascontiguousarray(T, np.float64)
    slot = np.ascontiguousarray(slot, np.int32)
    R = U.size
    dec = np.zeros(max(1, R - 1), np.uint8)
    _check(lib().re_test_exchange(_ptr(U), _ptr(T), _ptr(slot), R, int(seed), int(attempt),
                                  int(max_distance), _ptr(dec)))
    return dec[: R - 1]


def re_test_exchange_noalloc(U, T, slot, seed, attempt, max_distance=1):
    """re_test_exchange without any device allocation (the staging lives in
    a fixed array inside the library; at most 4096 replicas)."""
    U = np.ascontiguousarray(U, np.float64)
    T = np.ascontiguousarray(T, np.float64)
    slot = np.ascontiguousarray(slot, np.int32)
    R = U.size
    dec = np.zeros(max(1, R - 1), np.uint8)
    _check(lib().re_test_exchange_noalloc(_ptr(U), _ptr(T), _ptr(slot), R, int(seed), int(attempt),
                                          int(max_distance), _ptr(dec)))
    return dec[: R - 1]


def re_test_philox(ctr, key0, key1):
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    out = np.zeros_like(ctr)
    _check(lib().re_test_philox(_ptr(ctr), int(key0), int(key1), ctr.shape[0], _ptr(out)))
    return out


def re_test_normals(fp64, seed, ctr):
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    out = np.zeros((ctr.shape[0], 3))
    _check(lib().re_test_normals(int(fp64), int(seed), _ptr(ctr), ctr.shape[0], _ptr(out)))
    return out
