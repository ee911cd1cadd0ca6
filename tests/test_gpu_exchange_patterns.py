"""GPU tests of non-nearest-neighbour exchange patterns (Implementation
section: the scheme extends to them): attempt k pairs ladder slots (j, j+d)
at a distance d drawn in 1..D.

* the device rule on given inputs makes the oracle's decisions bit for bit;
* a synchronous FP64 run (lockstep and persistent engines) makes the
  oracle's pairings and decisions;
* an injected asynchronous schedule (persistent engine, partners found by
  each replica from its own slot) matches the oracle's replay.
"""
import numpy as np
import pytest

import oracle
from paper_0812_1633_amd import workloads as W

pytestmark = pytest.mark.gpu

RC, SKIN, DT = 2.5, 0.3, 0.005


@pytest.fixture(scope="module")
def relib():
    from paper_0812_1633_amd import re as R
    R.lib()
    return R


def test_decisions_bit_exact(relib):
    g = np.random.default_rng(31)
    for trial in range(200):
        R = int(g.integers(2, 65))
        D = int(g.integers(1, 9))
        T = np.sort(g.uniform(0.5, 3.0, R)) + np.arange(R) * 1e-9
        slot = g.permutation(R).astype(np.int32)
        U = -2000.0 + g.normal(0, 1, R) * g.choice([0.01, 1.0, 30.0])
        k = int(g.integers(0, 2**40))
        seed = int(g.integers(0, 2**63))
        dec = relib.re_test_exchange(U, T, slot, seed, k, D)
        _, _, recs = oracle.exchange(T, slot, U, seed, k, max_distance=D)
        expect = np.full(R - 1, 255, np.uint8)
        for rec in recs:
            expect[rec.slot_lo] = rec.accepted
        assert np.array_equal(dec, expect), (trial, R, D)


def melted(N, rho, seed, T):
    L = oracle.box_length(N, rho)
    x = W.perturbed_fcc(N, L, 0.05, seed)
    v = W.maxwell(N, T, seed + 1)
    rep = oracle.Replica(x, v, L, RC)
    oracle.md(rep, 80, SKIN, DT, 1.0, T, seed, 0)
    return W.snap_to_grid(rep.x.reshape(-1, 3), L), W.round_f32(rep.v.reshape(-1, 3))


@pytest.mark.parametrize("engine", ["lockstep", "persistent"])
def test_sync_run_matches_oracle(relib, engine):
    R, N, Nx, steps, seed, D = 6, 256, 10, 150, 12, 3
    T = W.ladder(0.9, 1.2, R)
    e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, Nx, seed, precision="fp64", engine=engine,
                     exchange_max_distance=D, watchdog_seconds=5)
    L = e.query_box()[0]
    xs, vs = [], []
    for r in range(R):
        x, v = melted(N, 0.8442, 50 + r, T[r])
        e.set_state(r, x, v)
        xs.append(x)
        vs.append(v)
    ens = oracle.Ensemble([N] * R, [L] * R, T, RC, SKIN, DT, 1.0, seed,
                          x=np.concatenate([a.reshape(-1) for a in xs]),
                          v=np.concatenate([a.reshape(-1) for a in vs]), max_distance=D)
    e.step(steps)
    ens.run_sync(steps, Nx)
    log, total = e.query_exchange_log()
    glog = sorted(log, key=lambda g: (g.attempt, g.slot_lo))
    assert total == len(ens.log) > 0
    assert any(g.slot_hi - g.slot_lo > 1 for g in glog)
    for g, o in zip(glog, ens.log):
        assert (g.attempt, g.slot_lo, g.slot_hi, g.rep_a, g.rep_b) == (o.attempt, o.slot_lo, o.slot_hi, o.rep_a,
                                                                         o.rep_b)
        assert abs(g.U_a - o.U_a) <= 1e-9 * abs(o.U_a)
        assert g.u == o.u and g.accepted == o.accepted
    assert any(g.accepted for g in glog)
    assert np.array_equal(e.query_slots(), ens.slot)
    att, acc = e.query_acceptance()
    assert np.array_equal(att, ens.attempts) and np.array_equal(acc, ens.accepts)
    e.close()


def test_injected_schedule_matches_oracle(relib):
    R, N, seed, D = 5, 256, 14, 4
    T = np.array([0.9, 0.93, 0.96, 0.99, 1.02])
    e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, 10, seed, precision="fp64", exchange="async",
                     exchange_max_distance=D, watchdog_seconds=5)
    L = e.query_box()[0]
    xs, vs = [], []
    for r in range(R):
        x, v = melted(N, 0.8442, 80 + r, T[r])
        e.set_state(r, x, v)
        xs.append(x)
        vs.append(v)
    join = np.array([[6, 9, 7, 8, 10], [13, 12, 15, 14, 11], [20, 22, 19, 21, 18], [26, 25, 27, 29, 28],
                     [33, 31, 34, 32, 35]], np.int64)
    e.set_schedule(join)
    e.step(0)
    ens = oracle.Ensemble([N] * R, [L] * R, T, RC, SKIN, DT, 1.0, seed,
                          x=np.concatenate([a.reshape(-1) for a in xs]),
                          v=np.concatenate([a.reshape(-1) for a in vs]), max_distance=D)
    ens.run_schedule(join, 0)
    log, total = e.query_exchange_log()
    glog = sorted(log, key=lambda g: (g.attempt, g.slot_lo))
    assert total == len(ens.log)
    for g, o in zip(glog, ens.log):
        assert (g.attempt, g.slot_lo, g.slot_hi, g.rep_a, g.rep_b) == (o.attempt, o.slot_lo, o.slot_hi, o.rep_a,
                                                                         o.rep_b)
        assert (g.step_a, g.step_b) == (o.step_a, o.step_b)
        assert abs(g.U_a - o.U_a) <= 1e-9 * abs(o.U_a) and g.accepted == o.accepted
    assert np.array_equal(e.query_slots(), ens.slot)
    e.close()
