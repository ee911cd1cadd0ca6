"""Benchmark: atom-steps/s of batched replica-exchange LJ MD on one MI355X.

One "step" is one MD step of every replica (list-update test, neighbour-list
rebuilds where triggered, LJ force, BAOAB integration) plus, every N_x steps,
the temperature-exchange attempt with velocity rescaling.  The default
workload is 32 replicas x 4000 LJ atoms (rho 0.8442, geometric ladder
T = 0.7 .. 2.0, r_c 2.5, skin 0.3, dt 0.005, N_x 50), batched mixed
precision; the plain per-replica FP64 form is timed beside it.

The input is prepared untimed: every replica is melted at T = 1.5 from the
FCC start, then equilibrated at its ladder temperature, so that the timed
window sees liquid-state list-update rates that differ along the ladder.
The timed window is placed so that an exchange attempt falls in its middle
(at the workload's N_x = 50 a 20-step window holds one attempt, a longer
one one per 50 steps); the cost of one attempt is measured apart, from
windows of N_x - 1 steps with and without one.

Prints one JSON line: the metric and its value, the configuration, the
dominant kernel's roofline figures, the CPU oracle's throughput, the
oracle-checked tolerance of the same configuration (on seeded injected
states), the plain per-replica FP64 form's throughput (the ratio's
baseline), the batched FP64 form's (the precision effect alone), and the
throughput under stochastic velocity rescaling.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "atom-steps/s over all replicas (batched mixed vs plain FP64) at stated tol"
PEAK_FP32_TFLOPS = 157.3  # MI355X published FP32 vector peak (packed FMA)
# the same unit counts without packed FP32 (the library is compiled with packed FP32
# instructions disabled): 256 CUs x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz
PEAK_FP32_UNPACKED_TFLOPS = 78.6

# HBM bytes per atom-step of the dominant kernel, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs of this benchmark with --copy-calibration,
# each scaled by what the counter reads for the 256 MiB device copy (FETCH_SIZE
# x 1.99975: it counts half the bytes the copy reads; WRITE_SIZE x 1.0), with
# the hash of the kernel sources they were taken with: a changed kernel
# reports traffic null until it is measured again.
TRAFFIC = {
    ("lj-32x4000", "persistent", 2): dict(fetch=72.61, write=66.68, src="885045b75436f1d8"),
}
KERNEL_SOURCES = ("re_persist.hip", "re_persist.hpp", "re_device.hpp", "re_internal.hpp", "re_kernels.hip")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_0812_1633_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pair_counts(x, L, rc, rl, max_exact=8192, sample=4096):
    """Unique pairs with r < rc and with rc <= r < rl (minimum image), for
    the algorithmic work: by brute force in blocks up to max_exact atoms;
    beyond, from the full neighbour counts of `sample` evenly spaced atoms
    (every pair is seen from both its atoms, so the unique pairs are N times
    half the mean count)."""
    n_c = n_s = 0
    N = len(x)
    if N <= max_exact:
        for a in range(0, N, 512):
            d = x[a:a + 512, None, :] - x[None, :, :]
            d -= L * np.round(d / L)
            r2 = (d * d).sum(-1)
            idx = np.arange(a, min(N, a + 512))[:, None]
            upper = np.arange(N)[None, :] > idx
            n_c += int(((r2 < rc * rc) & upper).sum())
            n_s += int(((r2 >= rc * rc) & (r2 < rl * rl) & upper).sum())
        return n_c, n_s
    pick = np.linspace(0, N - 1, sample).astype(np.int64)
    for a in range(0, sample, 64):
        ii = pick[a:a + 64]
        d = x[ii, None, :] - x[None, :, :]
        d -= L * np.round(d / L)
        r2 = (d * d).sum(-1)
        other = ii[:, None] != np.arange(N)[None, :]
        n_c += int(((r2 < rc * rc) & other).sum())
        n_s += int(((r2 >= rc * rc) & (r2 < rl * rl)).sum())
    return int(round(n_c * N / (2.0 * sample))), int(round(n_s * N / (2.0 * sample)))


def progress(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def melted_states(R, W, cfg, N, rho, T, melt_steps, kw):
    """Untimed input preparation: every replica melted at T = 1.5 (a flat
    ladder 1.5 (1 + 1e-9 k), so that all replicas are thermostatted at the
    melting temperature) from the FCC start; returns the states (x, v) in
    atom-id order."""
    Tm = 1.5 * (1.0 + 1e-9 * np.arange(len(N)))
    em = R.Engine(N, Tm, 0.0, cfg["rc"], cfg["skin"], cfg["dt"], 10**9, cfg["seed"] + 1000, **kw)
    em.step(melt_steps)
    st = [em.get_state(r) for r in range(len(N))]
    em.close()
    return st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--workload", default="lj-32x4000")
    ap.add_argument("--engine", default=None, help="persistent | lockstep (default: autotuned)")
    ap.add_argument("--tpa", type=int, default=0, help="force lanes per atom with --engine (default: 4)")
    ap.add_argument("--team-balance", action="store_true",
                    help="persistent engine: re-plan teams from measured list-update rates")
    ap.add_argument("--melt-steps", type=int, default=500,
                    help="input preparation: steps at T = 1.5 from the FCC start (0: start from FCC)")
    ap.add_argument("--equil-steps", type=int, default=500,
                    help="input preparation: steps at the ladder after melting")
    ap.add_argument("--plain-steps", type=int, default=100)
    ap.add_argument("--fp64-steps", type=int, default=1000,
                    help="steps of the batched FP64 form (the precision effect alone; 0: skip)")
    ap.add_argument("--svr-steps", type=int, default=1000,
                    help="steps of the same workload under stochastic velocity rescaling (0: skip)")
    ap.add_argument("--exchange", choices=["sync", "async"], default="sync",
                    help="exchange timing of the measured form (async: persistent engine; every step of every "
                         "replica counted, the call ending when all have done --steps)")
    ap.add_argument("--attempt-reps", type=int, default=10,
                    help="windows with and without an exchange attempt, for the per-attempt cost")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 256 MiB device-to-device (a kernel of known traffic for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs every replica on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0812_1633_amd import re as R
    from paper_0812_1633_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg = W.expand(args.workload)
    N, rho, T = cfg["N_list"], cfg["rho_list"], cfg["T_list"]
    rc, skin, dt, Nx, seed = cfg["rc"], cfg["skin"], cfg["dt"], cfg["Nx"], cfg["seed"]
    atoms = int(N.sum())
    Rn = len(N)
    kw = dict(rho_per_replica=rho, gamma=cfg["gamma"])
    tune = {"team_balance": True} if args.team_balance else {}
    if args.engine:
        tune["engine"] = args.engine
        tune["threads_per_atom"] = args.tpa
    else:
        tune["autotune"] = True
        import tempfile
        tune["tune_cache"] = os.environ.get("RE_TUNE_CACHE",
                                            os.path.join(tempfile.gettempdir(), "re_tune_cache.json"))
        os.makedirs(os.path.dirname(tune["tune_cache"]), exist_ok=True)

    # ---- batched mixed-precision form ------------------------------------
    progress("%s: %d replicas, %d atoms; creating the context" % (args.workload, Rn, atoms))
    xkw = {"exchange": "async"} if args.exchange == "async" else {}
    if xkw and tune.get("engine", "persistent") != "persistent":
        raise SystemExit("bench.py: asynchronous exchanges run in the persistent engine")
    eng = R.Engine(N, T, 0.0, rc, skin, dt, Nx, seed, precision="mixed", form="batched", **kw, **tune, **xkw)
    engine_used, tpa_used, team_used = eng.query_config()
    lanes = eng.query_lanes()
    lanes_used = (int(lanes[0]) if len(set(lanes.tolist())) == 1
                  else {"%d..%d atoms" % (2 ** k, 2 ** (k + 1) - 1): sorted(set(int(t) for t, n in zip(lanes, N)
                                                                               if int(np.log2(n)) == k))[0]
                        for k in sorted(set(int(np.log2(n)) for n in N))})
    start = "FCC lattice, Maxwell-Boltzmann velocities at the ladder"
    if args.melt_steps > 0:
        progress("input preparation: %d steps at T = 1.5, then %d at the ladder" % (args.melt_steps,
                                                                                  args.equil_steps))
        for r, (x, v) in enumerate(melted_states(R, W, cfg, N, rho, T, args.melt_steps, kw)):
            eng.set_state(r, x, v)
        start = "melted: %d steps at T = 1.5 from FCC, then %d at the ladder (untimed)" % (args.melt_steps,
                                                                                       args.equil_steps)
    eng.step(args.equil_steps if args.melt_steps > 0 else 0)
    prepared = [eng.get_state(r) for r in range(Rn)] if (args.plain_steps or args.fp64_steps) else None
    progress("engine %s, %d lanes per atom; %d warm-up steps" % (engine_used, tpa_used, args.warmup))
    eng.step(args.warmup)
    # the timed window holds an exchange attempt: its middle step is a
    # multiple of N_x (untimed padding steps before it)
    s_now = int(eng.query_steps()[0][0])
    pad = (-(s_now + (args.steps + 1) // 2)) % Nx if not xkw else 0
    eng.step(pad)
    steps0, reb0 = eng.query_steps()
    att0, acc0 = eng.query_acceptance()
    torch.cuda.synchronize()
    eng.profile(1)
    t0 = time.perf_counter()
    eng.step(args.steps)  # (returns after synchronising the library's stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    eng.profile(0)
    k_ms, k_n = eng.query_kernel_time()
    steps1, reb1 = eng.query_steps()
    att1, acc1 = eng.query_acceptance()
    done = int(((steps1 - steps0) * N).sum())
    value = done / (t1 - t0)
    # (asynchronous: per mean step of a replica, as replicas do different counts)
    ms_per_step = 1e3 * (t1 - t0) / (args.steps if not xkw else float((steps1 - steps0).mean()))
    win_att = int((att1 - att0).sum())
    win_acc = int((acc1 - acc0).sum())
    progress("%d timed steps: %.4f ms per step, %d exchange records in the window" % (args.steps, ms_per_step,
                                                                                   win_att))

    # ---- cost of one exchange attempt: windows of N_x - 1 steps with no
    # attempt (starting at a multiple of N_x) against the same windows with
    # one attempt in their middle (untimed steps realign between them)
    attempt = None
    if args.attempt_reps > 0 and Nx >= 3 and not xkw:
        tA, tB = [], []
        for rep in range(args.attempt_reps):
            for kind in ("A", "B"):
                s_now = int(eng.query_steps()[0][0])
                phase = 0 if kind == "A" else Nx // 2
                eng.step((phase - s_now) % Nx)
                torch.cuda.synchronize()
                a = time.perf_counter()
                eng.step(Nx - 1)
                torch.cuda.synchronize()
                (tA if kind == "A" else tB).append(time.perf_counter() - a)
        attempt = {"per_attempt_us": 1e6 * (np.mean(tB) - np.mean(tA)),
                   "window_steps": Nx - 1, "windows_each": args.attempt_reps,
                   "ms_per_step_no_attempt": 1e3 * np.mean(tA) / (Nx - 1),
                   "ms_per_step_one_attempt": 1e3 * np.mean(tB) / (Nx - 1)}

    progress("counting pairs")
    L = eng.query_box()
    # pair counts of two replicas at the states the run reached, for the
    # algorithmic flops (27 per unique in-cutoff pair, 9 per unique pair in
    # the skin shell); the persistent kernel does the whole timed run in
    # one launch, the lockstep engine's fused force kernel one step
    counts = []
    for r in (0, Rn - 1):
        x, _ = eng.get_state(r)
        counts.append(pair_counts(x, L[r], rc, rc + skin) + (int(N[r]),))
    flop_per_atom = np.mean([(27 * c + 9 * sk) / n for c, sk, n in counts])
    atom_steps_launch = atoms if engine_used == "lockstep" else done / max(1, k_n)
    flops_launch = flop_per_atom * atom_steps_launch
    achieved = flops_launch / (k_ms * 1e-3) / 1e12 if k_ms > 0 else None
    # the mixed form's list entries are 16-bit slots when every replica has at
    # most 65536 atoms (policy PMixed16), 32-bit byte offsets otherwise
    policy = "PMixed16" if int(N.max()) <= 65536 else "PMixed"
    tr = TRAFFIC.get((args.workload, engine_used, tpa_used))
    src = kernel_source_hash()
    traffic = None
    if tr and tr["src"] == src:
        traffic = (tr["fetch"] + tr["write"]) * atom_steps_launch
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": (achieved / PEAK_FP32_TFLOPS) if achieved else None, "traffic": traffic,
                "traffic_unit": "bytes per launch (HBM, counter-measured)",
                "hbm_GBps_at_traffic": (traffic / (k_ms * 1e-3) / 1e9) if traffic and k_ms > 0 else None,
                "peak_unpacked_fp32": PEAK_FP32_UNPACKED_TFLOPS,
                "frac_unpacked": (achieved / PEAK_FP32_UNPACKED_TFLOPS) if achieved else None,
                "kernel": ("k_force<%s,fused,%d>" % (policy, tpa_used)) if engine_used == "lockstep"
                else "k_persist<%s,%d,false>" % (policy, tpa_used),
                "kernel_ms": k_ms, "launches_timed": k_n, "atom_steps_per_launch": atom_steps_launch,
                "flop_per_atom_step": float(flop_per_atom), "kernel_src": src,
                "wall_over_kernel": ((t1 - t0) * 1e3 / (k_ms * k_n)) if (engine_used != "lockstep" and k_ms > 0)
                else None}

    # ---- tolerance of the same configuration against the oracle, on
    # seeded injected states (perturbed FCC on the position grid,
    # FP32-representable velocities): forces of every atom (or of 64 sampled
    # atoms of replicas too large for the all-pairs oracle) and the energy
    tol = None
    if not args.no_cpu:
        import oracle
        tol = {"force_normwise_max": 0.0, "energy_rel_max": 0.0, "input": "seeded perturbed FCC (amp 0.07)"}
        for r in (0, Rn - 1):
            x = W.perturbed_fcc(int(N[r]), L[r], 0.07, 7000 + r)
            eng.set_state(r, x, W.maxwell(int(N[r]), float(T[r]), 7100 + r))
            F, U = eng.compute_forces(r)
            if N[r] <= 20000:
                Fo, Uo, _ = oracle.forces(x, L[r], rc)
                tol["energy_rel_max"] = max(tol["energy_rel_max"], abs(U - Uo) / abs(Uo))
                rms = np.sqrt((Fo * Fo).sum(1).mean())
                tol["force_normwise_max"] = max(tol["force_normwise_max"], float(np.abs(F - Fo).max() / rms))
            else:
                g = np.random.default_rng(r)
                idx = g.choice(int(N[r]), size=64, replace=False)
                Fo = np.array([oracle.force_on(x, L[r], rc, int(i))[0] for i in idx])
                rms = np.sqrt((Fo * Fo).sum(1).mean())
                tol["force_normwise_max"] = max(tol["force_normwise_max"],
                                                float(np.abs(F[idx] - Fo).max() / rms))
                tol["energy"] = "not checked above 20000 atoms per replica (all-pairs oracle)"
        tol["passed"] = bool(tol["force_normwise_max"] <= 1e-5 and tol["energy_rel_max"] <= 1e-5)
    eng.close()

    def other_form(label, steps, **opts):
        """Throughput of another form of the same workload from the same
        prepared states (untimed warm-up of min(steps, 50) steps)."""
        e = R.Engine(N, T, 0.0, rc, skin, dt, Nx, seed, **kw, **opts)
        if prepared is not None:
            for r, (x, v) in enumerate(prepared):
                e.set_state(r, x, v)
        e.step(min(steps, 50))
        torch.cuda.synchronize()
        a = time.perf_counter()
        e.step(steps)
        torch.cuda.synchronize()
        b = time.perf_counter()
        out = {"value": atoms * steps / (b - a), "unit": "atom-steps/s", "steps": steps,
               "ms_per_step": 1e3 * (b - a) / steps, "config": e.query_config()}
        e.close()
        progress("%s: %.4f ms per step" % (label, out["ms_per_step"]))
        return out

    # ---- the precision effect alone: batched FP64 (autotuned the same way)
    fp64 = None
    if args.fp64_steps > 0:
        fp64 = other_form("batched fp64", args.fp64_steps, precision="fp64", form="batched", **tune)
        fp64["ratio_mixed_over_fp64"] = value / fp64["value"]
    # ---- plain per-replica FP64 form (the baseline the ratio is quoted on)
    plain = None
    if args.plain_steps > 0:
        plain = other_form("plain fp64", args.plain_steps, precision="fp64", form="plain")
        plain["ratio_mixed_over_plain"] = value / plain["value"]
    # ---- the paper's thermostat (stochastic velocity rescaling) ------------
    svr = None
    if args.svr_steps > 0:
        svr = other_form("mixed, velocity rescale", args.svr_steps, precision="mixed", form="batched",
                         thermostat="svr", engine=engine_used, threads_per_atom_per_replica=lanes)

    # ---- CPU leg: the oracle timed on a bounded sample of the workload ----
    cpu = None
    if not args.no_cpu:
        import oracle
        nthreads = oracle.num_threads()
        ens = oracle.Ensemble(N, L, T, rc, skin, dt, cfg["gamma"], seed)
        t0 = time.perf_counter()
        ens.run_sync(2, 10**9)
        t_probe = time.perf_counter() - t0
        n_more = max(1, int(args.cpu_seconds / max(t_probe / 2, 1e-6)))
        t0 = time.perf_counter()
        ens.run_sync(n_more, 10**9)
        t1c = time.perf_counter()
        cpu = {"value": atoms * n_more / (t1c - t0), "unit": "atom-steps/s", "cores": nthreads, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": "%d steps of all %d replicas of %s from the FCC start (Verlet-list oracle, "
                         "OpenMP over replicas, %d threads)" % (n_more, Rn, args.workload, nthreads)}

    out = {"metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": args.workload, "replicas": int(Rn), "atoms": atoms,
                      "atoms_per_replica": int(N[0]) if len(set(N.tolist())) == 1 else "uneven",
                      "rho": float(rho[0]) if len(set(rho.tolist())) == 1 else "uneven",
                      "T_ladder": [float(T[0]), float(T[-1])], "r_c": rc, "skin": skin, "dt": dt, "N_x": Nx,
                      "start": start, "exchange": "asynchronous" if xkw else "synchronous",
                      "precision": "FP32 pair arithmetic, 32-bit fixed-point positions, FP64 energies/exchange",
                      "engine": engine_used, "threads_per_atom": tpa_used, "team_size": team_used,
                      "lanes_per_replica": lanes_used,
                      "tuning": "explicit" if args.engine else "autotuned",
                      "parallelism": "replicas batched on 1 GPU"},
           "roofline": roofline, "cpu_baseline": cpu, "plain_fp64": plain, "batched_fp64": fp64,
           "thermostat_svr": svr, "tolerance": tol,
           "exchange": {"records_in_window": win_att, "accepted_in_window": win_acc, "attempt_cost": attempt},
           "rebuilds_per_replica_step": float((reb1 - reb0).sum() / max(1, (steps1 - steps0).sum()))}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
