"""GPU tests of the stochastic-velocity-rescaling thermostat (the thermostat
of the Example section; Bussi, Donadio and Parrinello 2007): velocity Verlet
steps with the rescale at every step boundary, through the C-ABI.

* 100 steps from the same injected state: positions and kinetic energy of
  the oracle (FP64 1e-9, mixed 1e-4), both batched engines and the plain
  per-replica form, over two calls;
* lockstep and persistent engines give bit-identical runs with exchanges;
* a synchronous FP64 run makes the oracle's exchange decisions;
* the kinetic energy on the GPU has the canonical mean and variance;
* an asynchronous run keeps the rule and the replicas' temperatures.
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


def melted(N, rho, seed, T):
    L = oracle.box_length(N, rho)
    x = W.perturbed_fcc(N, L, 0.05, seed)
    v = W.maxwell(N, T, seed + 1)
    rep = oracle.Replica(x, v, L, RC)
    oracle.md(rep, 80, SKIN, DT, 1.0, T, seed, 0)
    return L, W.snap_to_grid(rep.x.reshape(-1, 3), L), W.round_f32(rep.v.reshape(-1, 3))


def mi_dist(a, b, L):
    d = a - b
    d -= L * np.round(d / L)
    return np.abs(d).max()


@pytest.mark.parametrize("engine,precision", [("lockstep", "fp64"), ("lockstep", "mixed"), ("persistent", "fp64"),
                                              ("persistent", "mixed"), ("plain", "fp64")])
def test_svr_trajectory_matches_oracle(relib, engine, precision):
    R, N, seed = 3, 500, 11
    T = W.ladder(0.8, 1.6, R)
    form = "plain" if engine == "plain" else "batched"
    eng = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, 1000, seed, precision=precision, form=form,
                       engine="lockstep" if engine == "plain" else engine, thermostat="svr", watchdog_seconds=5)
    states = []
    for r in range(R):
        L, x, v = melted(N, 0.8442, 60 + r, T[r])
        eng.set_state(r, x, v)
        states.append((L, x, v))
    eng.step(37)
    eng.step(63)
    assert list(eng.query_steps()[0]) == [100] * R
    U = eng.query_energies()
    for r in range(R):
        L, x, v = states[r]
        rep = oracle.Replica(x, v, L, RC)
        oracle.md(rep, 100, SKIN, DT, 0.0, T[r], seed, r, thermostat="svr", tau=0.5)
        xg, vg = eng.get_state(r)
        tol = 1e-9 if precision == "fp64" else 1e-4
        assert mi_dist(xg, rep.x.reshape(-1, 3), L) <= tol, r
        Kg, Ko = 0.5 * (vg * vg).sum(), 0.5 * (rep.v * rep.v).sum()
        assert abs(Kg - Ko) / Ko <= (1e-10 if precision == "fp64" else 1e-4), (r, Kg, Ko)
        assert abs(U[r] - rep.U) / abs(rep.U) <= (1e-10 if precision == "fp64" else 1e-4)
    eng.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_svr_persistent_equals_lockstep(relib, precision):
    R, N, Nx = 6, 700, 10
    T = W.ladder(0.7, 1.6, R)
    out = {}
    for eng in ("lockstep", "persistent"):
        e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, Nx, 4, precision=precision, engine=eng,
                         thermostat="svr", svr_tau=0.2, watchdog_seconds=5)
        e.step(37)
        e.step(83)
        st = [e.get_state(r) for r in range(R)]
        out[eng] = (st, e.query_slots(), e.query_acceptance()[1], e.query_energies())
        e.close()
    a, b = out["lockstep"], out["persistent"]
    for r in range(R):
        assert np.array_equal(a[0][r][0], b[0][r][0]) and np.array_equal(a[0][r][1], b[0][r][1]), r
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert np.allclose(a[3], b[3], rtol=1e-13, atol=0)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_svr_accepted_swaps_inside_one_call(relib, precision):
    """A narrow ladder (acceptance near 1) and teams of 4 workgroups: swaps
    accepted inside one persistent call must change the temperature every
    team member thermostats to, exactly as between lockstep launches."""
    R, N, Nx = 4, 600, 5
    T = W.ladder(1.0, 1.03, R)
    out = {}
    for eng in ("lockstep", "persistent"):
        kw = dict(team_size=4) if eng == "persistent" else {}
        e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, Nx, 8, precision=precision, engine=eng,
                         thermostat="svr", svr_tau=0.1, watchdog_seconds=5, **kw)
        e.step(120)
        st = [e.get_state(r) for r in range(R)]
        out[eng] = (st, e.query_slots(), e.query_acceptance(), e.query_energies())
        e.close()
    a, b = out["lockstep"], out["persistent"]
    assert int(np.sum(a[2][1])) >= 5  # accepted swaps inside the call
    for r in range(R):
        assert np.array_equal(a[0][r][0], b[0][r][0]) and np.array_equal(a[0][r][1], b[0][r][1]), r
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2][0], b[2][0]) and np.array_equal(a[2][1], b[2][1])
    assert np.allclose(a[3], b[3], rtol=1e-13, atol=0)


def test_svr_sync_run_matches_oracle_fp64(relib):
    R, N, Nx, steps, seed = 4, 256, 20, 200, 9
    T = W.ladder(0.7, 1.2, R)
    eng = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, Nx, seed, precision="fp64", engine="persistent",
                       thermostat="svr", watchdog_seconds=5)
    L = eng.query_box()[0]
    xs, vs = [], []
    for r in range(R):
        _, x, v = melted(N, 0.8442, 40 + r, T[r])
        eng.set_state(r, x, v)
        xs.append(x)
        vs.append(v)
    ens = oracle.Ensemble([N] * R, [L] * R, T, RC, SKIN, DT, 0.0, seed,
                          x=np.concatenate([a.reshape(-1) for a in xs]),
                          v=np.concatenate([a.reshape(-1) for a in vs]), thermostat="svr")
    eng.step(steps)
    ens.run_sync(steps, Nx)
    log, total = eng.query_exchange_log()
    glog = sorted(log, key=lambda g: (g.attempt, g.slot_lo))
    assert total == len(ens.log) > 0
    for g, o in zip(glog, ens.log):
        assert (g.attempt, g.slot_lo, g.rep_a, g.rep_b) == (o.attempt, o.slot_lo, o.rep_a, o.rep_b)
        assert abs(g.U_a - o.U_a) <= 1e-9 * abs(o.U_a)
        assert g.u == o.u and g.accepted == o.accepted
    assert np.array_equal(eng.query_slots(), ens.slot)
    eng.close()


def test_svr_canonical_kinetic_energy(relib):
    """4 replicas x 500 atoms, mixed precision, tau = 0.1: after 1000 steps,
    K sampled every 10 steps has mean N_f T / 2 and variance N_f T^2 / 2."""
    R, N = 4, 500
    T = W.ladder(0.9, 1.5, R)
    e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, 10**6, 13, thermostat="svr", svr_tau=0.1,
                     engine="persistent", watchdog_seconds=5)
    e.step(1000)
    Ks = [[] for _ in range(R)]
    for _ in range(600):
        e.step(10)
        for r in range(R):
            _, v = e.get_state(r)
            Ks[r].append(0.5 * (v * v).sum())
    Nf = 3 * N - 3
    for r in range(R):
        k = np.array(Ks[r])
        assert k.mean() == pytest.approx(0.5 * Nf * T[r], rel=0.012), r
        assert k.var() == pytest.approx(0.5 * Nf * T[r] ** 2, rel=0.3), r
    e.close()


def test_svr_async_run(relib):
    """Asynchronous exchanges under the velocity rescale: every replica does
    at least n steps, every logged decision follows the rule with the Philox
    uniform of the lower replica id, and the kinetic temperatures stay near
    the temperatures the replicas hold."""
    R, N, Nx, n, seed = 6, 500, 3, 600, 23
    T = W.ladder(0.8, 1.3, R)
    e = relib.Engine([N] * R, T, 0.8442, RC, SKIN, DT, Nx, seed, exchange="async", thermostat="svr",
                     svr_tau=0.1, watchdog_seconds=10)
    e.step(n)
    steps, _ = e.query_steps()
    assert steps.min() >= n
    log, total = e.query_exchange_log()
    assert total > 20
    for g in log:
        assert oracle.metropolis(g.U_a, g.U_b, g.T_a, g.T_b, g.u) == g.accepted
        assert g.u == oracle.uniform53(seed, g.attempt, min(g.rep_a, g.rep_b))
    Tr = e.query_temps()
    for r in range(R):
        _, v = e.get_state(r)
        Tk = (v * v).sum() / (3 * N - 3)
        assert abs(Tk - Tr[r]) / Tr[r] < 0.15, (r, Tk, Tr[r])
    e.close()
