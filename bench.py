"""Benchmark: atom-steps/s of batched replica-exchange LJ MD on one MI355X.

One "step" is one MD step of every replica (list-update test, neighbour-list
rebuilds where triggered, LJ force, BAOAB integration) plus, every N_x steps,
the temperature-exchange attempt with velocity rescaling.  The default
workload is 32 replicas x 4000 LJ atoms (rho 0.8442, geometric ladder
T = 0.7 .. 2.0, r_c 2.5, skin 0.3, dt 0.005, N_x 50), batched mixed
precision; the plain per-replica FP64 form is timed beside it.

Prints one JSON line: the metric and its value, the configuration, the
dominant kernel's roofline figures, the CPU oracle's throughput and the
oracle-checked tolerance of the same run, the plain FP64 form's throughput
and the throughput under stochastic velocity rescaling.
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
    ("lj-32x4000", "persistent", 2): dict(fetch=351.7, write=93.6, src="8426a61382a89720"),
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--workload", default="lj-32x4000")
    ap.add_argument("--engine", default=None, help="persistent | lockstep (default: autotuned)")
    ap.add_argument("--plain-steps", type=int, default=100)
    ap.add_argument("--svr-steps", type=int, default=1000,
                    help="steps of the same workload under stochastic velocity rescaling (0: skip)")
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
    kw = dict(rho_per_replica=rho, gamma=cfg["gamma"])
    tune = {}
    if args.engine:
        tune["engine"] = args.engine
    else:
        tune["autotune"] = True
        import tempfile
        tune["tune_cache"] = os.environ.get("RE_TUNE_CACHE",
                                            os.path.join(tempfile.gettempdir(), "re_tune_cache.json"))
        os.makedirs(os.path.dirname(tune["tune_cache"]), exist_ok=True)

    # ---- batched mixed-precision form ------------------------------------
    progress("%s: %d replicas, %d atoms; creating the context" % (args.workload, len(N), atoms))
    eng = R.Engine(N, T, 0.0, rc, skin, dt, Nx, seed, precision="mixed", form="batched", **kw, **tune)
    engine_used, tpa_used, team_used = eng.query_config()
    progress("engine %s, %d lanes per atom; %d warm-up steps" % (engine_used, tpa_used, args.warmup))
    eng.step(args.warmup)
    steps0, reb0 = eng.query_steps()
    torch.cuda.synchronize()
    eng.profile(1)
    t0 = time.perf_counter()
    eng.step(args.steps)
    eng.query_energies()  # synchronises the library stream
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    eng.profile(0)
    k_ms, k_n = eng.query_kernel_time()
    steps1, reb1 = eng.query_steps()
    done = int(((steps1 - steps0) * N).sum())
    value = done / (t1 - t0)
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    acc_att, acc_acc = eng.query_acceptance()

    progress("%d timed steps: %.4f ms per step; counting pairs" % (args.steps, ms_per_step))
    # state and forces of two replicas, for the tolerance check of the CPU
    # leg, and their pair counts (the algorithmic work)
    L = eng.query_box()
    snaps, counts = [], []
    for r in (0, len(N) - 1):
        x, _ = eng.get_state(r)
        F, U = eng.compute_forces(r)
        snaps.append((r, x, F, U))
        counts.append(pair_counts(x, L[r], rc, rc + skin) + (int(N[r]),))

    # algorithmic flops per atom-step: 27 per unique in-cutoff pair and 9 per
    # unique pair in the skin shell (measured pair counts of two replicas).
    # The lockstep engine's dominant kernel does one step of every replica
    # per launch; the persistent kernel does the whole timed run.
    flop_per_atom = np.mean([(27 * c + 9 * s) / n for c, s, n in counts])
    flops_launch = flop_per_atom * (atoms if engine_used == "lockstep" else done / max(1, k_n))
    achieved = flops_launch / (k_ms * 1e-3) / 1e12 if k_ms > 0 else None
    atom_steps_launch = atoms if engine_used == "lockstep" else done / max(1, k_n)
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
                "kernel": "k_force<PMixed,fused>" if engine_used == "lockstep" else "k_persist<PMixed,%d,false>" % tpa_used,
                "kernel_ms": k_ms, "launches_timed": k_n, "atom_steps_per_launch": atom_steps_launch,
                "flop_per_atom_step": float(flop_per_atom), "kernel_src": src}
    eng.close()

    # ---- plain per-replica FP64 form ---------------------------------------
    plain = None
    if args.plain_steps > 0:
        ep = R.Engine(N, T, 0.0, rc, skin, dt, Nx, seed, precision="fp64", form="plain", **kw)
        ep.step(min(args.plain_steps, 50))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ep.step(args.plain_steps)
        ep.query_energies()
        t1 = time.perf_counter()
        pv = atoms * args.plain_steps / (t1 - t0)
        plain = {"value": pv, "unit": "atom-steps/s", "ms_per_step": 1e3 * (t1 - t0) / args.plain_steps,
                 "steps": args.plain_steps, "ratio_mixed_over_plain": value / pv}
        ep.close()

    # ---- the paper's thermostat (stochastic velocity rescaling) ------------
    svr = None
    if args.svr_steps > 0:
        es = R.Engine(N, T, 0.0, rc, skin, dt, Nx, seed, precision="mixed", form="batched", thermostat="svr",
                      engine=engine_used, threads_per_atom=tpa_used, **kw)
        es.step(min(args.svr_steps, 100))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        es.step(args.svr_steps)
        es.query_energies()
        t1 = time.perf_counter()
        svr = {"value": atoms * args.svr_steps / (t1 - t0), "unit": "atom-steps/s", "steps": args.svr_steps,
               "ms_per_step": 1e3 * (t1 - t0) / args.svr_steps}
        es.close()

    # ---- CPU leg: the oracle, (1) checking the GPU's forces and energy on the
    # states taken above, (2) timed on a bounded sample of the workload ----
    cpu = None
    tol = None
    if not args.no_cpu:
        import oracle
        tol = {"force_normwise_max": 0.0, "energy_rel_max": 0.0}
        for r, x, F, U in snaps:
            g = np.random.default_rng(r)
            idx = g.choice(int(N[r]), size=min(64, int(N[r])), replace=False)
            Fo = np.array([oracle.force_on(x, L[r], rc, int(i))[0] for i in idx])
            rms = np.sqrt((Fo * Fo).sum(1).mean())
            tol["force_normwise_max"] = max(tol["force_normwise_max"], float(np.abs(F[idx] - Fo).max() / rms))
            if r == 0:
                _, Uo, _ = oracle.forces(x, L[r], rc)
                tol["energy_rel_max"] = abs(U - Uo) / abs(Uo)
        tol["passed"] = bool(tol["force_normwise_max"] <= 1e-5 and tol["energy_rel_max"] <= 1e-5)
        nthreads = oracle.num_threads()
        ens = oracle.Ensemble(N, L, T, rc, skin, dt, cfg["gamma"], seed)
        t0 = time.perf_counter()
        ens.run_sync(2, 10**9)
        t_probe = time.perf_counter() - t0
        n_more = max(1, int(args.cpu_seconds / max(t_probe / 2, 1e-6)))
        t0 = time.perf_counter()
        ens.run_sync(n_more, 10**9)
        t1 = time.perf_counter()
        cpu = {"value": atoms * n_more / (t1 - t0), "unit": "atom-steps/s", "cores": nthreads, "kind": "oracle",
               "sample": "%d steps of all %d replicas of %s from the FCC start (Verlet-list oracle, "
                         "OpenMP over replicas)" % (n_more, len(N), args.workload)}

    out = {"metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": args.workload, "replicas": int(len(N)), "atoms": atoms,
                      "atoms_per_replica": int(N[0]) if len(set(N.tolist())) == 1 else "uneven",
                      "rho": float(rho[0]) if len(set(rho.tolist())) == 1 else "uneven",
                      "T_ladder": [float(T[0]), float(T[-1])], "r_c": rc, "skin": skin, "dt": dt, "N_x": Nx,
                      "precision": "FP32 pair arithmetic, 32-bit fixed-point positions, FP64 energies/exchange",
                      "engine": engine_used, "threads_per_atom": tpa_used, "team_size": team_used,
                      "tuning": "explicit" if args.engine else "autotuned",
                      "parallelism": "replicas batched on 1 GPU"},
           "roofline": roofline, "cpu_baseline": cpu, "plain_fp64": plain, "thermostat_svr": svr,
           "tolerance": tol,
           "exchange": {"attempts": int(acc_att.sum()), "accepted": int(acc_acc.sum())},
           "rebuilds_per_replica_step": float((reb1 - reb0).sum() / max(1, (steps1 - steps0).sum()))}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
