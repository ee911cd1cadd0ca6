"""GPU tests of the Example-section experiments and of the long-run
exchange statistics.

* the efficiency and diffusion drivers run end to end at small sizes: the
  synchronous form's observed stride equals N_x exactly, the asynchronous
  one's is at least 1, lambda and D are finite and positive;
* acceptance rates of a long synchronous run (mixed precision on the GPU)
  agree with the FP64 oracle's within 3 sigma overall and per ladder pair,
  over more than 10^4 attempts per pair (block-averaged errors; the
  trajectories themselves diverge chaotically, so only statistics can
  agree), for both thermostats;
* asynchronous attempts accept at the same rates as synchronous ones.
"""
import numpy as np
import pytest

import oracle
from paper_0812_1633_amd import experiments as E
from paper_0812_1633_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def relib():
    from paper_0812_1633_amd import re as R
    R.lib()
    return R


def test_efficiency_driver(relib):
    res = E.efficiency(Nr_list=(2, 4), steps=100, warmup=20, N=500, async_Nx=(1,))
    assert [r["Nr"] for r in res["rows"]] == [2, 4]
    for row in res["rows"]:
        assert row["base_steps_per_s"] > 0 and row["base_sync_steps_per_s"] > 0
        assert row["sync_Nx5"]["mean_Nx"] == pytest.approx(5.0)
        assert row["async_Nx1"]["mean_Nx"] >= 1.0
        for k in ("sync_Nx5", "async_Nx1"):
            assert 0.05 < row[k]["lam"] < 1.5


def test_async_call_keeps_every_replica_busy(relib):
    """Asynchronous re_step(n): every replica does at least n steps; the
    ones that get there first keep stepping until the last does, so with a
    hot/cold ladder the step counts differ (FP64 decisions still follow the
    Metropolis rule in the log)."""
    R, N = 4, 500
    T = np.array([0.7, 1.5, 2.5, 4.0])
    e = relib.Engine([N] * R, T, 0.8442, 2.5, 0.3, 0.005, 5, 3, exchange="async", precision="fp64",
                     watchdog_seconds=10)
    e.step(300)
    s, _ = e.query_steps()
    assert s.min() >= 300
    log, tot = e.query_exchange_log()
    assert tot > 0
    import oracle
    for g in log:
        assert oracle.metropolis(g.U_a, g.U_b, g.T_a, g.T_b, g.u) == g.accepted
    e.step(0)
    assert np.array_equal(e.query_steps()[0], s)
    e.close()


def test_diffusion_driver(relib):
    res = E.diffusion(Nr=6, sync_Nx=(5,), async_Nx=(2,), steps=3000, warmup=100, N=500)
    rows = {r["mode"]: r for r in res["rows"]}
    assert rows["sync"]["mean_Nx"] == pytest.approx(5.0)
    assert rows["async"]["mean_Nx"] >= 1.0
    for r in rows.values():
        assert np.isfinite(r["D"]) and r["D"] > 0
        assert r["attempts"] > 100


def block_err(x, nblocks=40):
    x = np.asarray(x, np.float64)
    n = x.size // nblocks * nblocks
    b = x[:n].reshape(nblocks, -1).mean(1)
    return b.std(ddof=1) / np.sqrt(nblocks)


@pytest.mark.parametrize("thermostat", ["langevin", "svr"])
def test_acceptance_matches_oracle(relib, thermostat):
    """Long-run acceptance, per ladder pair and overall, within 3 sigma of
    the FP64 oracle's independent run (sigma from 40 block averages of
    each run's 0/1 decisions, combined in quadrature), over more than 10^4
    attempts per pair: 4 replicas x 256 atoms, attempts every step."""
    import threading
    R, N, Nx, steps, burn = 4, 256, 1, 23000, 1000
    T = W.ladder(0.8, 1.0, R)
    rc, skin, dt, rho, seed = 2.5, 0.3, 0.005, 0.8442, 17
    L = oracle.box_length(N, rho)
    ens = oracle.Ensemble([N] * R, [L] * R, T, rc, skin, dt, 1.0, seed + 1, thermostat=thermostat)
    # the oracle's run (C, outside the interpreter lock) beside the GPU's
    th = threading.Thread(target=ens.run_sync, args=(steps, Nx))
    th.start()
    try:
        e = relib.Engine([N] * R, T, rho, rc, skin, dt, Nx, seed, thermostat=thermostat, engine="persistent",
                         log_capacity=1 << 17, watchdog_seconds=10)
        assert e.query_box()[0] == L
        e.step(steps)
        glog, total = e.query_exchange_log(cap=1 << 17)
        assert total == len(glog)
        e.close()
    finally:
        th.join()
    kmin = burn // Nx

    def per_pair(log):
        d = {j: [] for j in range(R - 1)}
        for g in sorted(log, key=lambda g: (g.attempt, g.slot_lo)):
            if g.attempt >= kmin:
                d[g.slot_lo].append(g.accepted)
        return d

    pg, po = per_pair(glog), per_pair(ens.log)
    allg = np.concatenate([pg[j] for j in pg])
    allo = np.concatenate([po[j] for j in po])
    s = np.sqrt(block_err(allg) ** 2 + block_err(allo) ** 2)
    assert 0.05 < allo.mean() < 0.95  # the ladder gives informative acceptance
    assert abs(allg.mean() - allo.mean()) <= 3 * s, (allg.mean(), allo.mean(), s)
    for j in range(R - 1):
        assert len(pg[j]) >= 10**4 and len(po[j]) >= 10**4, (j, len(pg[j]), len(po[j]))
        sj = np.sqrt(block_err(pg[j]) ** 2 + block_err(po[j]) ** 2)
        assert abs(np.mean(pg[j]) - np.mean(po[j])) <= 3 * sj, (j, np.mean(pg[j]), np.mean(po[j]), sj)


def test_async_acceptance_matches_sync(relib):
    """Asynchronous attempts sample the same acceptance as synchronous ones
    (the rule keeps detailed balance whatever the join steps): per ladder
    pair, over more than 10^4 attempts each, within 3.5 sigma of a
    synchronous run of the same ladder (block-averaged errors combined in
    quadrature; 3.5 rather than 3 because the asynchronous run depends on
    timing, so the comparison is drawn afresh on every run)."""
    R, N, steps_sync, steps_async = 4, 256, 23000, 70000
    T = W.ladder(0.8, 1.0, R)
    rc, skin, dt, rho, seed = 2.5, 0.3, 0.005, 0.8442, 17
    logs = {}
    for mode, n in (("sync", steps_sync), ("async", steps_async)):
        e = relib.Engine([N] * R, T, rho, rc, skin, dt, 1, seed, exchange=mode, engine="persistent",
                         log_capacity=1 << 18, watchdog_seconds=10)
        e.step(1000)
        k0 = e.query_attempt_count()
        e.step(n)
        glog, total = e.query_exchange_log(cap=1 << 18)
        assert total <= 1 << 18
        logs[mode] = [g for g in glog if g.attempt >= k0]
        e.close()

    def per_pair(log):
        d = {j: [] for j in range(R - 1)}
        for g in sorted(log, key=lambda g: (g.attempt, g.slot_lo)):
            if g.slot_hi == g.slot_lo + 1:
                d[g.slot_lo].append(g.accepted)
        return {j: np.array(v, dtype=np.float64) for j, v in d.items()}

    ps, pa = per_pair(logs["sync"]), per_pair(logs["async"])
    for j in range(R - 1):
        assert len(ps[j]) >= 10**4 and len(pa[j]) >= 10**4, (j, len(ps[j]), len(pa[j]))
        sj = np.sqrt(block_err(ps[j]) ** 2 + block_err(pa[j]) ** 2)
        assert abs(np.mean(ps[j]) - np.mean(pa[j])) <= 3.5 * sj, (j, np.mean(ps[j]), np.mean(pa[j]), sj)
