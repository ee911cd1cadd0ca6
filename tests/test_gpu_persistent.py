"""GPU tests of the persistent engine (one launch per re_step) and of the
asynchronous exchange protocol (Implementation section: rotating master,
partners wait for each other, replicas may take different numbers of steps
between attempts).

Synchronous mode must give bit-identical states to the lockstep engine (the
same kernels per atom, the same list-update decisions); an injected
asynchronous schedule must make the exchange decisions of the oracle's
replay of that schedule; a free-running asynchronous run must log decisions
that the oracle's rule reproduces, with a log whose schedule, replayed by the
oracle from the same start, gives the same decisions (FP64).
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


def states(eng, R):
    return [eng.get_state(r) for r in range(R)]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("team", [0, 1, 2])
def test_persistent_sync_equals_lockstep(relib, precision, team):
    R, N, Nx = 6, 700, 10
    T = W.ladder(0.7, 1.6, R)
    out = {}
    for eng in ("lockstep", "persistent"):
        e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, Nx, 4, precision=precision, engine=eng,
                         team_size=team if eng == "persistent" else 0, watchdog_seconds=5)
        e.step(37)
        e.step(83)  # calls that do not end on an exchange step
        out[eng] = (states(e, R), e.query_energies(), e.query_slots(), e.query_steps(), e.query_acceptance())
        log, tot = e.query_exchange_log()
        out[eng] += (sorted((g.attempt, g.slot_lo, g.accepted) for g in log),)
        e.close()
    a, b = out["lockstep"], out["persistent"]
    for r in range(R):
        assert np.array_equal(a[0][r][0], b[0][r][0]) and np.array_equal(a[0][r][1], b[0][r][1]), r
    assert np.allclose(a[1], b[1], rtol=1e-13, atol=0)
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[3][0], b[3][0]) and np.array_equal(a[3][1], b[3][1])
    assert np.array_equal(a[4][0], b[4][0]) and np.array_equal(a[4][1], b[4][1])
    assert a[5] == b[5]


def test_team_sizes_agree(relib):
    """Teams of 1, 3 and 8 workgroups per replica, with either team barrier
    (one-XCD release where the team shares an L2, or agent scope always),
    give the same run."""
    R, N = 4, 3000
    T = W.ladder(0.8, 1.4, R)
    ref = None
    for team, bar in ((1, "auto"), (3, "auto"), (8, "auto"), (8, "agent"), (3, "agent")):
        e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, 20, 2, team_size=team, watchdog_seconds=5,
                         team_barrier=bar)
        e.step(60)
        st = states(e, R)
        e.close()
        if ref is None:
            ref = st
        else:
            for r in range(R):
                assert np.array_equal(st[r][0], ref[r][0]) and np.array_equal(st[r][1], ref[r][1])


def melted(N, rho, seed, T):
    L = oracle.box_length(N, rho)
    x = W.perturbed_fcc(N, L, 0.05, seed)
    v = W.maxwell(N, T, seed + 1)
    rep = oracle.Replica(x, v, L, RC)
    oracle.md(rep, 80, SKIN, DT, 1.0, T, seed, 0)
    return W.snap_to_grid(rep.x.reshape(-1, 3), L), W.round_f32(rep.v.reshape(-1, 3))


def test_injected_schedule_matches_oracle(relib):
    """Asynchronous timing replaced by an injected schedule (replica r joins
    attempt a at join[a, r]): the GPU (FP64) and the oracle's replay make the
    same pairings and decisions on energies equal to 1e-9, and every
    replica ends at its last join step."""
    R, N, seed = 4, 256, 8
    T = np.array([0.9, 0.95, 1.0, 1.05])
    e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, 10, seed, precision="fp64", exchange="async",
                     watchdog_seconds=5)
    L = e.query_box()[0]
    xs, vs = [], []
    for r in range(R):
        x, v = melted(N, 0.8442, 70 + r, T[r])
        e.set_state(r, x, v)
        xs.append(x)
        vs.append(v)
    join = np.array([[8, 11, 9, 12], [15, 19, 16, 14], [23, 21, 30, 25], [31, 33, 35, 29]], np.int64)
    e.set_schedule(join)
    e.step(0)
    steps, _ = e.query_steps()
    assert list(steps) == list(join[-1])
    ens = oracle.Ensemble([N] * R, [L] * R, T, RC, SKIN, DT, 1.0, seed,
                          x=np.concatenate([a.reshape(-1) for a in xs]), v=np.concatenate([a.reshape(-1) for a in vs]))
    ens.run_schedule(join, 0)
    log, total = e.query_exchange_log()
    glog = sorted(log, key=lambda g: (g.attempt, g.slot_lo))
    assert total == len(ens.log)
    for g, o in zip(glog, ens.log):
        assert (g.attempt, g.slot_lo, g.rep_a, g.rep_b) == (o.attempt, o.slot_lo, o.rep_a, o.rep_b)
        assert (g.step_a, g.step_b) == (o.step_a, o.step_b)
        assert g.u == o.u
        assert abs(g.U_a - o.U_a) <= 1e-9 * abs(o.U_a) and abs(g.U_b - o.U_b) <= 1e-9 * abs(o.U_b)
        assert g.accepted == o.accepted
    assert any(g.accepted for g in glog)
    assert np.array_equal(e.query_slots(), ens.slot)
    for r in range(R):
        xg, vg = e.get_state(r)
        d = xg - ens.replica_x(r)
        d -= L * np.round(d / L)
        assert np.abs(d).max() < 1e-8
    e.close()


def test_async_free_run(relib):
    """Free-running asynchronous exchange: the rotating master of attempt k
    is k mod R and joins N_x of its own steps after its previous join; every
    other replica joins at a later boundary; decisions follow the oracle's
    rule; every replica does at least n steps; replaying the logged join
    steps in the oracle (FP64) reproduces every decision."""
    R, N, Nx, n, seed = 6, 400, 5, 120, 21
    T = W.ladder(0.8, 1.3, R)
    e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, Nx, seed, precision="fp64", exchange="async",
                     watchdog_seconds=5)
    L = e.query_box()[0]
    xs = [e.get_state(r) for r in range(R)]
    e.step(n)
    steps, _ = e.query_steps()
    assert steps.min() >= n
    log, total = e.query_exchange_log()
    assert total > 0
    byk = {}
    for g in log:
        assert g.master == g.attempt % R
        assert oracle.metropolis(g.U_a, g.U_b, g.T_a, g.T_b, g.u) == g.accepted
        assert g.u == oracle.uniform53(seed, g.attempt, min(g.rep_a, g.rep_b))
        byk.setdefault(g.attempt, []).append(g)
    ks = sorted(byk)
    assert ks == list(range(len(ks)))
    # join step of every replica in every attempt (paired ones from the log,
    # unpaired ones are not logged); the master joins N_x steps after its
    # previous join
    join = {}
    for k in ks:
        for g in byk[k]:
            join[(k, g.rep_a)] = g.step_a
            join[(k, g.rep_b)] = g.step_b
    # (a replica's previous join is known when it was paired then)
    prev = {r: (-1, 0) for r in range(R)}  # (attempt, step) of the last logged join
    checked = 0
    for k in ks:
        m = k % R
        if (k, m) in join and prev[m][0] == k - 1:
            assert join[(k, m)] == prev[m][1] + Nx
            checked += 1
        for r in range(R):
            if (k, r) in join:
                prev[r] = (k, join[(k, r)])
    assert checked > 0
    acc_att, acc_acc = e.query_acceptance()
    assert acc_att.sum() == total and acc_acc.sum() == sum(g.accepted for g in log)
    slots = e.query_slots()
    assert sorted(slots) == list(range(R))
    e.close()


def test_async_replay_in_oracle(relib):
    """The schedule of a free asynchronous run, recovered from the log and
    the step counts, replayed by the oracle from the same initial state,
    reproduces every logged decision (FP64; short run, so energies agree to
    1e-9)."""
    R, N, Nx, n, seed = 4, 256, 4, 60, 5
    T = np.array([0.9, 0.95, 1.0, 1.05])
    e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, Nx, seed, precision="fp64", exchange="async",
                     watchdog_seconds=5)
    L = e.query_box()[0]
    xs, vs = [], []
    for r in range(R):
        x, v = melted(N, 0.8442, 90 + r, T[r])
        e.set_state(r, x, v)
        xs.append(x)
        vs.append(v)
    e.step(n)
    log, total = e.query_exchange_log()
    byk = {}
    for g in log:
        byk.setdefault(g.attempt, []).append(g)
    ks = sorted(byk)
    # unpaired replicas join too but are not logged; a replica that does not
    # exchange only keeps stepping, so any join step not below its previous
    # one replays it: take the previous one
    join = np.zeros((len(ks), R), np.int64)
    prev = np.zeros(R, np.int64)
    for a, k in enumerate(ks):
        known = {}
        for g in byk[k]:
            known[g.rep_a] = g.step_a
            known[g.rep_b] = g.step_b
        for r in range(R):
            join[a, r] = known.get(r, prev[r])
        prev = join[a].copy()
    ens = oracle.Ensemble([N] * R, [L] * R, T, RC, SKIN, DT, 1.0, seed,
                          x=np.concatenate([q.reshape(-1) for q in xs]), v=np.concatenate([q.reshape(-1) for q in vs]))
    ens.run_schedule(join, 0)
    olog = {(o.attempt, o.slot_lo): o for o in ens.log}
    for g in log:
        o = olog[(g.attempt, g.slot_lo)]
        assert (o.rep_a, o.rep_b) == (g.rep_a, g.rep_b)
        assert abs(g.U_a - o.U_a) <= 1e-9 * abs(o.U_a)
        assert o.accepted == g.accepted
    e.close()


def test_watchdog_timeout_is_reported(relib):
    """A watchdog bound far below one step's duration makes every wait give
    up (the condition is forced from the host; every workgroup still exits
    normally): re_step reports RE_ETIMEOUT; a new context works."""
    R, N = 4, 2000
    T = W.ladder(0.8, 1.2, R)
    e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, 5, 1, team_size=4, watchdog_seconds=1e-7)
    with pytest.raises(relib.ReError) as err:
        e.step(50)
    assert err.value.code == relib.RE_ETIMEOUT
    e.close()
    e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, 5, 1, team_size=4, watchdog_seconds=5)
    e.step(20)
    assert list(e.query_steps()[0]) == [20] * R
    e.close()


@pytest.mark.parametrize("thermostat", ["langevin", "svr"])
def test_explicit_exchange_between_calls(relib, thermostat):
    """re_exchange() between two re_step calls: its velocity factors are
    applied by the next step in both engines (bit-identical runs), and
    get_state reports the rescaled velocities right after the exchange."""
    R, N = 4, 600
    T = np.array([1.0, 1.001, 1.002, 1.003])  # nearly equal: swaps are accepted
    out = {}
    for eng in ("lockstep", "persistent"):
        e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, 10**6, 6, precision="fp64", engine=eng,
                         thermostat=thermostat, watchdog_seconds=5)
        e.step(15)
        before = [e.get_state(r)[1] for r in range(R)]
        slots0 = e.query_slots().copy()
        e.exchange()
        slots1 = e.query_slots()
        assert not np.array_equal(slots0, slots1)
        for r in range(R):
            fac = np.sqrt(T[slots1[r]] / T[slots0[r]])
            assert np.allclose(e.get_state(r)[1], fac * before[r], rtol=1e-14, atol=0), r
        e.step(20)
        out[eng] = [e.get_state(r) for r in range(R)]
        e.close()
    for r in range(R):
        assert np.array_equal(out["lockstep"][r][0], out["persistent"][r][0]), r
        assert np.array_equal(out["lockstep"][r][1], out["persistent"][r][1]), r


def test_wide_reorder_equals_persistent(relib):
    """Replicas of 20000 atoms are reordered by grid-wide passes in the
    lockstep engine and by one workgroup in the persistent engine: the same
    canonical order, so the runs agree bitwise (with exchanges)."""
    R, N, Nx = 3, 20000, 15
    T = W.ladder(0.8, 1.2, R)
    out = {}
    for eng in ("lockstep", "persistent"):
        e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, Nx, 8, engine=eng, watchdog_seconds=10)
        e.step(45)
        out[eng] = ([e.get_state(r) for r in range(R)], e.query_steps()[1].copy(), e.query_slots().copy())
        e.close()
    a, b = out["lockstep"], out["persistent"]
    assert np.array_equal(a[1], b[1]) and a[1].min() >= 2
    assert np.array_equal(a[2], b[2])
    for r in range(R):
        assert np.array_equal(a[0][r][0], b[0][r][0]) and np.array_equal(a[0][r][1], b[0][r][1]), r


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_reorder_paths_agree(relib, precision):
    """One ladder of 20000-, 4000- and 1500-atom replicas: with a replica of
    16384 atoms or more the lockstep engine reorders every replica by
    grid-wide passes, while the persistent engine reorders the small ones
    with their atoms held in registers (and builds their lists and forces
    from LDS copies) and the large one through global scratch.  The same
    canonical order (cell, then atom id) makes the runs agree bitwise."""
    N = [20000, 4000, 1500]
    R, Nx = len(N), 10
    T = W.ladder(0.8, 1.3, R)
    out = {}
    for eng in ("lockstep", "persistent"):
        e = relib.Engine(N, T, 0.8442, RC, SKIN, DT, Nx, 12, precision=precision, engine=eng,
                         watchdog_seconds=10)
        e.step(17)
        e.step(33)
        out[eng] = ([e.get_state(r) for r in range(R)], e.query_steps()[1].copy(), e.query_slots().copy(),
                    e.query_energies().copy())
        e.close()
    a, b = out["lockstep"], out["persistent"]
    assert np.array_equal(a[1], b[1]) and a[1].min() >= 2
    assert np.array_equal(a[2], b[2])
    for r in range(R):
        assert np.array_equal(a[0][r][0], b[0][r][0]) and np.array_equal(a[0][r][1], b[0][r][1]), r
    assert np.array_equal(a[3], b[3])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_list_key_staging_paths_agree(relib, precision):
    """Replicas of 7000, 5000, 9000 and 2000 atoms: in the persistent engine
    (4 lanes per atom) the mixed form takes the list keys and the force sums'
    positions from LDS copies for all but the 9000-atom replica, which reads
    both from global memory; the FP64 form stages only the smallest.  The
    lockstep engine reads everything from global memory.  Synchronous runs
    with list updates and exchanges agree bitwise."""
    N = [7000, 5000, 9000, 2000]
    R, Nx = len(N), 10
    T = W.ladder(0.8, 1.3, R)
    out = {}
    for eng in ("lockstep", "persistent"):
        e = relib.Engine(N, T, 0.8442, RC, SKIN, DT, Nx, 21, precision=precision, engine=eng,
                         watchdog_seconds=10)
        e.step(17)
        e.step(33)
        out[eng] = ([e.get_state(r) for r in range(R)], e.query_steps()[1].copy(), e.query_slots().copy(),
                    e.query_energies().copy())
        e.close()
    a, b = out["lockstep"], out["persistent"]
    assert np.array_equal(a[1], b[1]) and a[1].min() >= 2
    assert np.array_equal(a[2], b[2])
    for r in range(R):
        assert np.array_equal(a[0][r][0], b[0][r][0]) and np.array_equal(a[0][r][1], b[0][r][1]), r
    assert np.array_equal(a[3], b[3])


@pytest.mark.parametrize("tpa,nfit,precision", [(1, 9216, "mixed"), (2, 8192, "mixed"), (4, 8704, "mixed"),
                                                 (8, 8960, "mixed"), (2, 2432, "fp64"), (8, 2432, "fp64")])
def test_position_copy_at_its_limit(relib, tpa, nfit, precision):
    """The mixed form's LDS copy of the positions (16 B per atom) and the
    stash of per-atom sums (32 B per atom of a pass: 1024 / tpa atoms) share
    the persistent workgroup's 144 KiB: replicas of nfit atoms fill it
    exactly, one atom more reads the positions from global memory, where the
    sums of tpa passes share one epilogue round (the FP64 form's copy sits
    above the list-build tables: 2432 atoms).  Both agree bitwise with the
    lockstep engine over list updates and exchanges."""
    N = [nfit, nfit + 1]
    R, Nx = len(N), 10
    T = W.ladder(0.8, 1.3, R)
    out = {}
    for eng in ("lockstep", "persistent"):
        e = relib.Engine(N, T, 0.8442, RC, SKIN, DT, Nx, 5, engine=eng, threads_per_atom=tpa,
                         precision=precision, watchdog_seconds=10)
        e.step(40)
        out[eng] = ([e.get_state(r) for r in range(R)], e.query_steps()[1].copy(), e.query_energies().copy())
        e.close()
    a, b = out["lockstep"], out["persistent"]
    assert np.array_equal(a[1], b[1]) and a[1].min() >= 2
    for r in range(R):
        assert np.array_equal(a[0][r][0], b[0][r][0]) and np.array_equal(a[0][r][1], b[0][r][1]), r
    assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("precision,team,thermostat", [("mixed", 8, "langevin"), ("fp64", 3, "langevin"),
                                                     ("mixed", 8, "svr"), ("fp64", 3, "svr")])
def test_sync_results_independent_of_timing(relib, precision, team, thermostat):
    """Workgroups of the persistent teams paused at random after team
    barriers (the debug_delay_us hook: one in four, up to 30 us): synchronous
    runs, with list updates and exchanges, stay bit-identical to the
    lockstep engine, so no result depends on when the members of a team
    leave a barrier.  Under the velocity rescale every member computes the
    rescale factor after the force phase's barrier and the next first half
    ends at another one."""
    R, N, Nx = 6, 1200, 10
    T = W.ladder(0.7, 1.6, R)
    out = {}
    for eng, delay in (("lockstep", 0), ("persistent", 30)):
        e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, Nx, 5, precision=precision, engine=eng,
                         team_size=team if eng == "persistent" else 0, debug_delay_us=delay,
                         watchdog_seconds=10, thermostat=thermostat, svr_tau=0.2)
        e.step(53)
        e.step(47)
        out[eng] = (states(e, R), e.query_slots().copy(), e.query_steps()[1].copy(), e.query_energies().copy())
        e.close()
    a, b = out["lockstep"], out["persistent"]
    assert a[2].min() >= 5 and np.array_equal(a[2], b[2])
    assert np.array_equal(a[1], b[1])
    for r in range(R):
        assert np.array_equal(a[0][r][0], b[0][r][0]) and np.array_equal(a[0][r][1], b[0][r][1]), r
    assert np.allclose(a[3], b[3], rtol=1e-13, atol=0)
    with pytest.raises(Exception):
        relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, Nx, 5, debug_delay_us=-1)


def test_team_rebalancing(relib):
    """Automatic teams are re-planned from the measured list-update rates
    once every replica has done 500 steps: on a hot/cold ladder the hot
    replicas (more frequent list updates) get more workgroups, every team
    stays within one XCD's 32 workgroups, and the run is bitwise the same as
    with teams proportional to N."""
    R, N = 32, 3000  # (teams of at most 12 workgroups; 8 each to start with)
    T = W.ladder(0.6, 3.0, R)
    out = {}
    for bal in (True, False):
        e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, 25, 6, team_balance=bal, watchdog_seconds=10)
        t0 = e.query_teams()
        assert np.all(t0 == t0[0])  # equal replicas: equal teams to start with
        e.step(500)
        e.step(60)  # (re-planned at the start of this call)
        t1 = e.query_teams()
        if bal:
            assert t1.sum() <= 256 and t1.min() >= 1
            _, reb = e.query_steps()
            hot, cold = int(np.argmax(reb)), int(np.argmin(reb))
            assert t1[hot] > t1[cold], (t1, reb)
        else:
            assert np.array_equal(t1, t0)
        out[bal] = [e.get_state(r) for r in range(R)] + [e.query_energies(), e.query_slots()]
        e.close()
    for a, b in zip(out[True], out[False]):
        if isinstance(a, tuple):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        else:
            assert np.array_equal(a, b)
