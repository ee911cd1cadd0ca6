"""FP64 CPU oracle for replica-exchange Lennard-Jones MD.

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only users.  The GPU library never
imports, links or calls anything here, and this package imports nothing from
the GPU library.

``re_oracle.c`` holds the arithmetic (plain C, double precision); this module
compiles it with gcc into ``libre_oracle.so`` next to the source and exposes
thin numpy wrappers.  Each wrapper names the paper passage its C function
follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "re_oracle.c")
_LIB = os.path.join(_HERE, "libre_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over replicas)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class XRec(C.Structure):
    """One exchange record (attempt, ladder pair, replicas, join steps,
    energies, temperatures, uniform, decision)."""
    _fields_ = [("attempt", C.c_int64), ("slot_lo", C.c_int32), ("rep_a", C.c_int32),
                ("rep_b", C.c_int32), ("accepted", C.c_int32), ("step_a", C.c_int64),
                ("step_b", C.c_int64), ("U_a", C.c_double), ("U_b", C.c_double),
                ("T_a", C.c_double), ("T_b", C.c_double), ("u", C.c_double), ("slot_hi", C.c_int32),
                ("pad", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_normals3.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, dp]
        L.oracle_normals3.restype = None
        L.oracle_uniform53.argtypes = [C.c_uint64, C.c_int64, C.c_int32]
        L.oracle_uniform53.restype = C.c_double
        L.oracle_box_length.argtypes = [C.c_int32, C.c_double]
        L.oracle_box_length.restype = C.c_double
        L.oracle_fcc_cells.argtypes = [C.c_int32]
        L.oracle_fcc_cells.restype = C.c_int
        L.oracle_init.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_uint64, C.c_int32, dp, dp]
        L.oracle_init.restype = C.c_int
        L.oracle_lj_shift.argtypes = [C.c_double]
        L.oracle_lj_shift.restype = C.c_double
        L.oracle_forces.argtypes = [C.c_int32, C.c_double, C.c_double, dp, dp,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_forces.restype = C.c_int
        L.oracle_force_on.argtypes = [C.c_int32, C.c_double, C.c_double, dp, C.c_int32, dp,
                                      C.POINTER(C.c_double)]
        L.oracle_force_on.restype = C.c_int
        L.oracle_md.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                                C.c_double, C.c_double, C.c_uint64, C.c_int32, C.c_int64,
                                C.c_int64, dp, dp, dp, dp, C.POINTER(C.c_int64),
                                C.POINTER(C.c_double), C.c_int, C.c_int, C.c_double]
        L.oracle_svr_factor.argtypes = [C.c_double] * 6
        L.oracle_svr_factor.restype = C.c_double
        L.oracle_svr_noise.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int64,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_svr_noise.restype = None
        L.oracle_md.restype = C.c_int
        L.oracle_metropolis.argtypes = [C.c_double] * 5
        L.oracle_metropolis.restype = C.c_int
        L.oracle_exchange.argtypes = [C.c_int32, dp, i32p, dp, C.c_void_p, C.c_uint64, C.c_int64,
                                      C.c_int32, dp, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]
        L.oracle_pattern_distance.argtypes = [C.c_uint64, C.c_int64, C.c_int32]
        L.oracle_pattern_distance.restype = C.c_int
        L.oracle_exchange.restype = C.c_int
        L.oracle_run.argtypes = [C.c_int32, i32p, i64p, dp, dp, C.c_double, C.c_double, C.c_double,
                                 C.c_double, C.c_int, C.c_double, C.c_int32, C.c_uint64, C.c_int, dp, dp, dp,
                                 dp, i64p, dp, i64p,
                                 i32p, C.c_int64, C.c_int32, C.c_void_p, C.c_int64, C.c_int64,
                                 i64p, i64p, C.c_void_p, C.POINTER(C.c_int64)]
        L.oracle_run.restype = C.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = C.c_int
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# Thin wrappers

def philox4x32_10(ctr, key):
    """Philox4x32-10 block (Salmon et al., SC'11)."""
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(np.ascontiguousarray(ctr, np.uint32),
                               np.ascontiguousarray(key, np.uint32), out)
    return out


def normals3(seed, c0, c1, c2, purpose):
    z = np.zeros(3)
    lib().oracle_normals3(seed, c0, c1, c2, purpose, z)
    return z


def uniform53(seed, attempt, lower_id):
    """Uniform of an exchange attempt, drawn for the lower replica id
    (Implementation section)."""
    return lib().oracle_uniform53(seed, attempt, lower_id)


def box_length(N, rho):
    return lib().oracle_box_length(int(N), float(rho))


def lj_shift(rc):
    return lib().oracle_lj_shift(float(rc))


def init_replica(N, L, T, seed, replica):
    """FCC start with Maxwell-Boltzmann velocities (atom-id order)."""
    x = np.zeros(3 * N)
    v = np.zeros(3 * N)
    rc = lib().oracle_init(int(N), float(L), float(T), seed, int(replica), x, v)
    if rc:
        raise ValueError("oracle_init failed: %d" % rc)
    return x.reshape(N, 3), v.reshape(N, 3)


def forces(x, L, rc):
    """All-pairs truncated-shifted LJ forces, energy and virial (Example
    section: cutoff 2.5)."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1)
    N = x.size // 3
    F = np.zeros(3 * N)
    U = C.c_double()
    W = C.c_double()
    lib().oracle_forces(N, float(L), float(rc), x, F, C.byref(U), C.byref(W))
    return F.reshape(N, 3), U.value, W.value


def force_on(x, L, rc, i):
    """Force on atom i and its pair-energy sum, by the all-pairs definition."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1)
    F = np.zeros(3)
    e = C.c_double()
    lib().oracle_force_on(x.size // 3, float(L), float(rc), x, int(i), F, C.byref(e))
    return F, e.value


THERMOSTATS = {"langevin": 0, "svr": 1}
SVR_TAU = 0.5  # relaxation time of the velocity rescale (the paper gives none)


def svr_factor(K, Kbar, Nf, c, R1, S):
    """Velocity factor sqrt(K'/K) of one stochastic velocity rescale
    (Bussi, Donadio, Parrinello 2007; the Example section's thermostat):
    R1 standard normal, S chi-square with N_f - 1 degrees of freedom,
    c = exp(-dt/tau)."""
    return lib().oracle_svr_factor(float(K), float(Kbar), float(Nf), float(c), float(R1), float(S))


def svr_noise(seed, N, replica, step):
    """(R1, S) of the rescale of `replica` at step boundary `step`: Philox
    normals of counter (atom id, step, replica, purpose 4)."""
    R1 = C.c_double()
    S = C.c_double()
    lib().oracle_svr_noise(seed, int(N), int(replica), int(step), C.byref(R1), C.byref(S))
    return R1.value, S.value


def metropolis(Ua, Ub, Tj, Tj1, u):
    """Metropolis decision for swapping T_j (held by a) and T_{j+1} (held by
    b) (Implementation section)."""
    return lib().oracle_metropolis(float(Ua), float(Ub), float(Tj), float(Tj1), float(u))


class Replica:
    """One replica's MD state for :func:`md` (atom-id order)."""

    def __init__(self, x, v, L, rc):
        self.x = np.ascontiguousarray(x, np.float64).reshape(-1).copy()
        self.v = np.ascontiguousarray(v, np.float64).reshape(-1).copy()
        self.L = float(L)
        self.rc = float(rc)
        F, U, _ = forces(self.x, L, rc)
        self.F = F.reshape(-1).copy()
        self.U = U
        self.xref = self.x.copy()
        self.rebuilds = 1  # the list is built at step 0
        self.step = 0

    @property
    def N(self):
        return self.x.size // 3


def md(rep: Replica, nsteps, skin, dt, gamma, T, seed, replica_id, use_list=True, thermostat="langevin",
       tau=SVR_TAU):
    """Advance one replica ``nsteps`` steps (Example section: dt, thermostat;
    list update at half the skin): BAOAB Langevin with friction ``gamma``, or
    velocity Verlet with the stochastic velocity rescale of relaxation time
    ``tau`` (thermostat="svr")."""
    nreb = C.c_int64(rep.rebuilds)
    U = C.c_double(rep.U)
    rc = lib().oracle_md(rep.N, rep.L, rep.rc, float(skin), float(dt), float(gamma), float(T),
                         seed, int(replica_id), int(rep.step), int(nsteps), rep.x, rep.v,
                         rep.F, rep.xref, C.byref(nreb), C.byref(U), int(use_list),
                         THERMOSTATS[thermostat], float(tau))
    if rc:
        raise RuntimeError("oracle_md failed: %d" % rc)
    rep.rebuilds = nreb.value
    rep.U = U.value
    rep.step += int(nsteps)
    return rep


def pattern_distance(seed, k, max_distance):
    """Pairing distance of attempt k (1 for the nearest-neighbour pattern)."""
    return lib().oracle_pattern_distance(seed, int(k), int(max_distance))


def exchange(Tl, slot, U, seed, k, steps=None, max_distance=1):
    """One exchange attempt k over the ladder (Implementation section):
    ladder pairs at the attempt's distance (1: alternating nearest
    neighbours).  Returns (new slot, alpha per replica, list of XRec)."""
    R = len(slot)
    Tl = np.ascontiguousarray(Tl, np.float64)
    slot = np.ascontiguousarray(slot, np.int32).copy()
    U = np.ascontiguousarray(U, np.float64)
    alpha = np.ones(R)
    recs = (XRec * max(1, R))()
    n = C.c_int64(0)
    st = None if steps is None else np.ascontiguousarray(steps, np.int64)
    lib().oracle_exchange(R, Tl, slot, U, None if st is None else st.ctypes.data, seed, int(k),
                          int(max_distance), alpha,
                          None, None, C.cast(recs, C.c_void_p), C.byref(n))
    return slot, alpha, [recs[i] for i in range(n.value)]


class Ensemble:
    """All replicas of a replica-exchange run, concatenated in replica order
    (each replica's atoms in atom-id order)."""

    def __init__(self, N, L, Tl, rc, skin, dt, gamma, seed, x=None, v=None, use_list=True,
                 thermostat="langevin", tau=SVR_TAU, max_distance=1):
        self.N = np.ascontiguousarray(N, np.int32)
        self.R = len(self.N)
        self.off = np.zeros(self.R, np.int64)
        self.off[1:] = np.cumsum(3 * self.N.astype(np.int64))[:-1]
        self.L = np.ascontiguousarray(L, np.float64)
        self.Tl = np.ascontiguousarray(Tl, np.float64)
        self.rc, self.skin, self.dt, self.gamma = float(rc), float(skin), float(dt), float(gamma)
        self.seed = int(seed)
        self.use_list = int(use_list)
        self.thermostat, self.tau = THERMOSTATS[thermostat], float(tau)
        self.max_distance = int(max_distance)
        self.slot = np.arange(self.R, dtype=np.int32)
        tot = int(3 * self.N.astype(np.int64).sum())
        if x is None:
            xs, vs = [], []
            for r in range(self.R):
                xr, vr = init_replica(int(self.N[r]), self.L[r], self.Tl[self.slot[r]], seed, r)
                xs.append(xr.reshape(-1))
                vs.append(vr.reshape(-1))
            x = np.concatenate(xs)
            v = np.concatenate(vs)
        self.x = np.ascontiguousarray(x, np.float64).reshape(-1).copy()
        self.v = np.ascontiguousarray(v, np.float64).reshape(-1).copy()
        assert self.x.size == tot and self.v.size == tot
        self.F = np.zeros(tot)
        self.U = np.zeros(self.R)
        for r in range(self.R):
            a, b = self.off[r], self.off[r] + 3 * self.N[r]
            F, U, _ = forces(self.x[a:b], self.L[r], rc)
            self.F[a:b] = F.reshape(-1)
            self.U[r] = U
        self.xref = self.x.copy()
        self.steps = np.zeros(self.R, np.int64)
        self.rebuilds = np.ones(self.R, np.int64)
        self.attempts = np.zeros(max(1, self.R - 1), np.int64)
        self.accepts = np.zeros(max(1, self.R - 1), np.int64)
        self.log = []

    def replica_x(self, r):
        a = self.off[r]
        return self.x[a:a + 3 * self.N[r]].reshape(-1, 3)

    def replica_v(self, r):
        a = self.off[r]
        return self.v[a:a + 3 * self.N[r]].reshape(-1, 3)

    def _run(self, nsteps, Nx, sched, A, k0, cap):
        recs = (XRec * max(1, cap))()
        n = C.c_int64(0)
        rc = lib().oracle_run(self.R, self.N, self.off, self.L, self.Tl, self.rc, self.skin,
                              self.dt, self.gamma, self.thermostat, self.tau, self.max_distance, self.seed,
                              self.use_list, self.x, self.v,
                              self.F, self.xref, self.steps, self.U, self.rebuilds, self.slot,
                              int(nsteps), int(Nx),
                              None if sched is None else sched.ctypes.data, int(A), int(k0),
                              self.attempts, self.accepts, C.cast(recs, C.c_void_p), C.byref(n))
        if rc:
            raise RuntimeError("oracle_run failed: %d" % rc)
        self.log.extend(recs[i] for i in range(n.value))

    def run_sync(self, nsteps, Nx):
        """Synchronous variant: every replica attempts after each N_x of its
        steps (Implementation section, last paragraph)."""
        nattempts = (int(nsteps) // int(Nx)) + 1
        self._run(nsteps, Nx, None, 0, 0, nattempts * (self.R // 2 + 1))

    def run_schedule(self, join, k0):
        """Replay attempts k0 .. k0+A-1 with the given per-replica join steps
        (array A x R) (Implementation section, asynchronous iteration)."""
        join = np.ascontiguousarray(join, np.int64)
        A = join.shape[0]
        self._run(0, 1, join, A, k0, A * (self.R // 2 + 1))

    def temps(self):
        return self.Tl[self.slot]


def num_threads():
    return lib().oracle_num_threads()
