"""The Example section's measurements, on one GPU through the library.

* ``efficiency``: parallel efficiency lambda against the number of replicas
  (Scalability subsection, Fig. 1b): the total number of steps all replicas
  do per unit of wall-clock time with exchanges, divided by the same number
  without exchanges; synchronous exchanges with N_x = 5 against
  asynchronous ones with N_x = 1.
* ``diffusion``: diffusion coefficient D of log T against the observed
  exchange stride <N_x> (Diffusion subsection, Fig. 1a), for both forms at
  N_r = 48.
* ``acceptance``: the acceptance of each ladder pair against the estimate
  from the run's own energy distributions (Gaussian energies), and the
  configurational heat capacity along the ladder, which sets the acceptance
  the Example section reports for its ladder ratio.
* ``phases``: where the persistent kernel's time goes per step, without and
  with exchanges (a library built with the phase timers).

The workload is the paper's Lennard-Jones liquid: 4000 atoms per replica at
density 0.844, cutoff 2.5, neighbour list to 3.0 (skin 0.5) updated at half
the skin, time step 0.005, stochastic velocity rescaling, and temperatures
T_k = 0.7 * 1.0275^k.  <N_x> is the average number of steps a replica does
between two attempts (total steps of all replicas / (replicas x attempts)).

Command line: ``python -m paper_0812_1633_amd.experiments
efficiency|diffusion|acceptance|phases [--out FILE] [...]`` prints (and
writes) one JSON document.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

PAPER = dict(N=4000, rho=0.844, rc=2.5, skin=0.5, dt=0.005, Tmin=0.7, ratio=1.0275, thermostat="svr")


def paper_ladder(Nr, Tmin=PAPER["Tmin"], ratio=PAPER["ratio"]):
    """T_k = Tmin ratio^k, k = 0 .. Nr - 1 (Example section)."""
    return Tmin * ratio ** np.arange(Nr, dtype=np.float64)


def _engine(R, Nr, exchange, Nx, seed, N, **kw):
    return R.Engine([N] * Nr, paper_ladder(Nr), PAPER["rho"], PAPER["rc"], PAPER["skin"], PAPER["dt"], Nx, seed,
                    engine="persistent", exchange=exchange, thermostat=PAPER["thermostat"], watchdog_seconds=30,
                    **kw)


def _window(e, n0):
    """Exchange records written since the log held n0 records."""
    log, n1 = e.query_exchange_log()
    k = n1 - n0
    if k > len(log):
        raise RuntimeError("exchange log ring too small for the window")
    return log[len(log) - k:] if k > 0 else []


def timed_run(R, Nr, exchange, Nx, steps, warmup, seed=1, N=PAPER["N"], **kw):
    """Run `warmup` then `steps` steps; returns steps/s over all replicas,
    atom-steps/s, <N_x> in the timed window and the attempts there."""
    e = _engine(R, Nr, exchange, Nx, seed, N, log_capacity=1 << 20, **kw)
    try:
        e.step(warmup)
        s0, _ = e.query_steps()
        a0 = e.query_attempt_count()
        t0 = time.perf_counter()
        e.step(steps)
        e.query_energies()
        t1 = time.perf_counter()
        s1, _ = e.query_steps()
        att = e.query_attempt_count() - a0
        done = int((s1 - s0).sum())
        return dict(steps_per_s=done / (t1 - t0), atom_steps_per_s=done * N / (t1 - t0),
                    mean_Nx=(done / (Nr * att)) if att else None, attempts=att, seconds=t1 - t0,
                    steps_done=done)
    finally:
        e.close()


def efficiency(Nr_list=(2, 4, 8, 16, 32, 48, 64, 96, 128), steps=500, warmup=100, sync_Nx=5, async_Nx=(1, 3),
               N=PAPER["N"], seed=1):
    """lambda(N_r): steps/s of all replicas with exchanges divided by the
    same form's steps/s without exchanges (the paper's count of steps in a
    fixed wall-clock time).  The asynchronous base lets every replica step
    freely for the whole call; the synchronous base is the synchronous form
    with no boundary inside the call, so that each lambda measures what the
    exchanges cost that form.  Synchronous form at sync_Nx; asynchronous
    form at each of async_Nx (N_x = 1 is the paper's choice; a larger N_x
    brings <N_x> near the synchronous stride on one GPU, where a trigger
    reaches the other replicas within one step).  The ladder reaches
    0.7 * 1.0275^(N_r - 1): 22 at N_r = 128, too hot for dt = 0.005 much
    beyond that."""
    from . import re as R
    rows = []
    for Nr in Nr_list:
        base = timed_run(R, Nr, "async", 10**9, steps, warmup, seed, N)
        base_sync = timed_run(R, Nr, "sync", 10**9, steps, warmup, seed, N)
        row = dict(Nr=int(Nr), base_steps_per_s=base["steps_per_s"], base_sync_steps_per_s=base_sync["steps_per_s"])
        runs = [("sync", sync_Nx)] + [("async", nx) for nx in async_Nx]
        for mode, nx in runs:
            t = timed_run(R, Nr, mode, nx, steps, warmup, seed, N)
            b = base_sync if mode == "sync" else base
            row["%s_Nx%d" % (mode, nx)] = dict(mode=mode, Nx=nx, lam=t["steps_per_s"] / b["steps_per_s"],
                                               mean_Nx=t["mean_Nx"], attempts=t["attempts"])
        rows.append(row)
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return dict(experiment="efficiency", workload=dict(PAPER, N=N), steps=steps, warmup=warmup, rows=rows)


# ---------------------------------------------------------------------------
# Diffusion in log-temperature space

def logT_paths(log, T_ladder, slot0, t0):
    """Per replica, the (step, log T) points where its temperature changes:
    replica r holds slot0[r] from its step t0[r]; an accepted swap in the
    exchange records moves the two replicas to each other's slots at their
    join steps."""
    slot = np.array(slot0, dtype=np.int64)
    lt = np.log(np.asarray(T_ladder, np.float64))
    paths = [[(int(t0[r]), lt[slot[r]])] for r in range(len(slot))]
    for g in sorted(log, key=lambda g: (g.attempt, g.slot_lo)):
        if g.accepted:
            a, b = g.rep_a, g.rep_b
            slot[a], slot[b] = slot[b], slot[a]
            paths[a].append((int(g.step_a), lt[slot[a]]))
            paths[b].append((int(g.step_b), lt[slot[b]]))
    return paths


def _sample(path, t):
    """log T of a step-function path at steps t (the value set at the last
    change at or before t)."""
    s = np.array([p[0] for p in path])
    v = np.array([p[1] for p in path])
    return v[np.searchsorted(s, t, side="right") - 1]


def msd(paths, t_start, t_end, lags):
    """Mean squared displacement of log T at the given lags (steps),
    averaged over replicas r and over origins t in [t_start[r], t_end[r] - lag]
    (each replica on its own step count)."""
    out = []
    for lag in lags:
        acc, n = 0.0, 0
        for r, p in enumerate(paths):
            t = np.arange(int(t_start[r]), int(t_end[r]) - lag + 1, max(1, lag // 4))
            if t.size == 0:
                continue
            d = _sample(p, t + lag) - _sample(p, t)
            acc += float((d * d).sum())
            n += d.size
        out.append(acc / max(n, 1))
    return np.array(out)


def diffusion_coefficient(paths, t_start, t_end, dt, stride, nlags=6):
    """D of log T per unit of time: half the least-squares slope of the MSD
    over lags of 2, 4, ..., 2 nlags exchange strides (short enough to stay
    well below the saturation set by the ladder width), divided by dt.
    Returns (D, lags, msd)."""
    lags = np.array([max(1, int(round(2 * k * stride))) for k in range(1, nlags + 1)])
    m = msd(paths, t_start, t_end, lags)
    A = np.vstack([lags, np.ones_like(lags)]).T.astype(np.float64)
    slope, _ = np.linalg.lstsq(A, m, rcond=None)[0]
    return 0.5 * slope / dt, lags, m


def diffusion(Nr=48, sync_Nx=(2, 5, 10, 20, 50), async_Nx=(1, 2, 5, 10, 20), steps=20000, warmup=1000,
              N=PAPER["N"], seed=1):
    """D(<N_x>) for both forms at N_r replicas."""
    from . import re as R
    rows = []
    for mode, nxs in (("sync", sync_Nx), ("async", async_Nx)):
        for Nx in nxs:
            e = _engine(R, Nr, mode, Nx, seed, N, log_capacity=1 << 22)
            try:
                e.step(warmup)
                s0, _ = e.query_steps()
                slot0 = e.query_slots().copy()
                _, n0 = e.query_exchange_log(0)
                a0 = e.query_attempt_count()
                t0 = time.perf_counter()
                e.step(steps)
                t1 = time.perf_counter()
                s1, _ = e.query_steps()
                win = _window(e, n0)
                paths = logT_paths(win, paper_ladder(Nr), slot0, s0)
                att = e.query_attempt_count() - a0
                mean_Nx = float((s1 - s0).sum()) / (Nr * max(att, 1))
                D, lags, m = diffusion_coefficient(paths, s0, s1, PAPER["dt"], mean_Nx)
                rows.append(dict(mode=mode, Nx=int(Nx), mean_Nx=mean_Nx, D=D, attempts=att,
                                 accept=float(np.mean([g.accepted for g in win])) if win else None,
                                 msd=[float(x) for x in m], lags=[int(x) for x in lags], seconds=t1 - t0))
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            finally:
                e.close()
    return dict(experiment="diffusion", workload=dict(PAPER, N=N), Nr=Nr, steps=steps, warmup=warmup, rows=rows)


# ---------------------------------------------------------------------------
# Acceptance along the ladder against the Gaussian-energy estimate

def expected_min1_exp(m, v):
    """E[min(1, e^x)] for x ~ N(m, v): P(x >= 0) + E[e^x; x < 0]."""
    from math import erfc, exp, sqrt
    sd = sqrt(v)
    phi = lambda z: 0.5 * erfc(-z / sqrt(2.0))
    return phi(m / sd) + exp(m + 0.5 * v) * phi(-(m + v) / sd)


def ladder_acceptance(log, T_ladder, kmin=0):
    """Per ladder pair (j, j+1): the measured acceptance of the records of
    attempts >= kmin, and the estimate from the energies the log holds.
    Every record gives the energy of the replica at slot j (U_a, at T_a) and
    at slot j+1 (U_b, at T_b); with the mean and variance of U at each
    temperature, the Metropolis exponent (1/T_j - 1/T_{j+1})(U_a - U_b) of
    two independent replicas is Gaussian with mean dB (mean_j - mean_{j+1})
    and variance dB^2 (var_j + var_{j+1}), whose expected min(1, e^x) is the
    estimate.  Also the configurational heat capacity per replica var / T^2
    at each temperature."""
    T = np.asarray(T_ladder, np.float64)
    R = T.size
    samples = [[] for _ in range(R)]
    acc = [[] for _ in range(R - 1)]
    for g in log:
        if g.attempt < kmin:
            continue
        samples[g.slot_lo].append(g.U_a)
        samples[g.slot_hi].append(g.U_b)
        if g.slot_hi == g.slot_lo + 1:
            acc[g.slot_lo].append(g.accepted)
    mean = np.array([np.mean(x) if x else np.nan for x in samples])
    var = np.array([np.var(x, ddof=1) if len(x) > 1 else np.nan for x in samples])
    rows = []
    for j in range(R - 1):
        dB = 1.0 / T[j] - 1.0 / T[j + 1]
        m = dB * (mean[j] - mean[j + 1])
        v = dB * dB * (var[j] + var[j + 1])
        est = expected_min1_exp(m, v) if np.isfinite(m) and v > 0 else None
        rows.append(dict(j=j, T=float(T[j]), attempts=len(acc[j]),
                         measured=float(np.mean(acc[j])) if acc[j] else None, gaussian=est,
                         cv_conf=float(var[j] / T[j] ** 2) if np.isfinite(var[j]) else None))
    return rows


def acceptance(Nr=48, Nx=5, steps=20000, warmup=2000, N=PAPER["N"], seed=1):
    """The paper's workload at N_r replicas, synchronous exchanges every N_x
    steps: per ladder pair the measured acceptance against the
    Gaussian-energy estimate from the run's own energies, and the
    configurational heat capacity per atom along the ladder."""
    from . import re as R
    e = _engine(R, Nr, "sync", Nx, seed, N, log_capacity=1 << 22)
    try:
        e.step(warmup)
        k0 = e.query_attempt_count()
        e.step(steps)
        log, _ = e.query_exchange_log()
    finally:
        e.close()
    rows = ladder_acceptance(log, paper_ladder(Nr), k0)
    meas = [r["measured"] for r in rows if r["measured"] is not None]
    est = [r["gaussian"] for r in rows if r["gaussian"] is not None]
    cv = [r["cv_conf"] / N for r in rows if r["cv_conf"] is not None]
    return dict(experiment="acceptance", workload=dict(PAPER, N=N), Nr=Nr, Nx=Nx, steps=steps, warmup=warmup,
                mean_measured=float(np.mean(meas)), mean_gaussian=float(np.mean(est)),
                cv_conf_per_atom=dict(first=cv[0], last=cv[-1], mean=float(np.mean(cv))), rows=rows)


# ---------------------------------------------------------------------------
# Where the persistent kernel's time goes (instrumented build)

PHASES = ("boundary, exchange join, barrier", "first half of a step (with the rescale), barrier", "reorder, barrier",
          "list build", "force pass (the workgroup's first wave)", "team barrier after the forces",
          "rest of a stop", "rest of the workgroup after the force pass",
          "exchange join: wait at the gate", "exchange join: wait for the partner",
          "stop: the leader's potential energy", "stop: the leader's velocity rescale")


def _workload_engine(R, name, melt=500, equil=500, **kw):
    """A persistent-engine context of a named benchmark workload, prepared as
    the benchmark prepares it: every replica melted at T = 1.5 from the FCC
    start, then equilibrated at its ladder temperature."""
    from . import workloads as W
    cfg = W.expand(name)
    N, rho, T = cfg["N_list"], cfg["rho_list"], cfg["T_list"]
    common = dict(rho_per_replica=rho, gamma=cfg["gamma"])
    em = R.Engine(N, 1.5 * (1.0 + 1e-9 * np.arange(len(N))), 0.0, cfg["rc"], cfg["skin"], cfg["dt"], 10**9,
                  cfg["seed"] + 1000, **common)
    em.step(melt)
    states = [em.get_state(r) for r in range(len(N))]
    em.close()
    e = R.Engine(N, T, 0.0, cfg["rc"], cfg["skin"], cfg["dt"], cfg["Nx"], cfg["seed"], engine="persistent",
                 **common, **kw)
    for r, (x, v) in enumerate(states):
        e.set_state(r, x, v)
    e.step(equil)
    return e


def phases(lib_path, Nr=16, modes=(("async", None), ("async", 1), ("sync", 5)), steps=1000, warmup=300,
           N=PAPER["N"], seed=1, workload=None, threads_per_atom=2):
    """Microseconds per step (and per workgroup) in each phase of the
    persistent kernel, from a library built with RE_PHASE_TIMERS
    (``python -m paper_0812_1633_amd.build --phase-timers`` writes
    ``libre_hip_timers.so``): on the paper's workload at N_r replicas
    without exchanges and with the given (mode, N_x); or, with ``workload``,
    on that benchmark workload (its own exchange settings, melted start).
    The two join waits lie inside the first phase.  With exchanges, also the
    microseconds per attempt of the team leaders (the workgroups that time
    the stop reductions) and of the other members."""
    import ctypes as C
    from . import re as R
    R.LIB_PATH = lib_path
    L = R.lib()
    L.re_debug_phase_ticks.argtypes = [C.c_void_p, C.c_int]
    rows = []
    buf = np.zeros(1024 * 12, np.uint64)
    if workload:
        modes = (("workload", None),)
    for mode, nx in modes:
        if workload:
            e = _workload_engine(R, workload, threads_per_atom=threads_per_atom)
            Nr = e.R
        else:
            e = _engine(R, Nr, mode, nx or 10**9, seed, N, log_capacity=1 << 16)
        try:
            e.step(warmup)
            L.re_debug_phase_ticks(buf.ctypes.data, 1024)
            s0, _ = e.query_steps()
            a0 = e.query_attempt_count()
            t0 = time.perf_counter()
            e.step(steps)
            t1 = time.perf_counter()
            s1, _ = e.query_steps()
            a1 = e.query_attempt_count()
            L.re_debug_phase_ticks(buf.ctypes.data, 1024)
        finally:
            e.close()
        t = buf.reshape(1024, 12).astype(np.float64)
        act = t[:, :8].sum(1) > 0
        done = float((s1 - s0).sum())
        us = t[act].mean(0)[:len(PHASES)] / 100.0 / (done / Nr)  # 100 MHz ticks
        row = dict(mode=mode, Nx=nx, steps_per_s_per_replica=done / Nr / (t1 - t0),
                   mean_Nx=(done / (Nr * (a1 - a0))) if a1 > a0 else None,
                   us_per_step=dict(zip(PHASES, [float(x) for x in us])))
        lead = act & (t[:, 10] + t[:, 11] > 0)
        if a1 > a0 and lead.any() and (act & ~lead).any():
            # every replica joins every attempt (asynchronous and synchronous forms)
            per = lambda m: dict(zip(PHASES, [float(x) for x in t[m].mean(0)[:len(PHASES)] / 100.0 / (a1 - a0)]))
            row["us_per_attempt_leader"] = per(lead)
            row["us_per_attempt_member"] = per(act & ~lead)
        rows.append(row)
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return dict(experiment="phases", workload=workload or dict(PAPER, N=N), Nr=Nr, steps=steps, warmup=warmup,
                rows=rows)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("which", choices=["efficiency", "diffusion", "acceptance", "phases"])
    ap.add_argument("--lib", default=None, help="phases: a library built with RE_PHASE_TIMERS")
    ap.add_argument("--workload", default=None, help="phases: a benchmark workload instead of the paper's")
    ap.add_argument("--out", default=None)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--atoms", type=int, default=PAPER["N"])
    ap.add_argument("--replicas", type=str, default=None, help="comma-separated N_r values (efficiency)")
    args = ap.parse_args(argv)
    kw = dict(N=args.atoms)
    if args.steps:
        kw["steps"] = args.steps
    if args.warmup is not None:
        kw["warmup"] = args.warmup
    if args.which == "efficiency":
        if args.replicas:
            kw["Nr_list"] = tuple(int(x) for x in args.replicas.split(","))
        res = efficiency(**kw)
    elif args.which == "phases":
        if args.replicas:
            kw["Nr"] = int(args.replicas)
        if args.workload:
            kw["workload"] = args.workload
            kw.pop("N", None)
        res = phases(args.lib, **kw)
    elif args.which == "acceptance":
        if args.replicas:
            kw["Nr"] = int(args.replicas)
        res = acceptance(**kw)
    else:
        res = diffusion(**kw)
    txt = json.dumps(res, indent=1)
    print(txt)
    if args.out:
        with open(args.out, "w") as f:
            f.write(txt + "\n")


if __name__ == "__main__":
    main()
