"""Pins of the oracle's temperature-exchange rule (Implementation section:
Metropolis rule with the lower-ranked node's random number, temperatures
swapped and velocities scaled; alternating nearest-neighbour pattern).

Pinned by: detailed balance checked by exact enumeration on a toy discrete
system, the closed-form acceptance of Gamma-distributed energies
(harmonic systems) by quadrature, the special cases of the rule, and the
synchronous schedule (every attempt after exactly N_x steps).
"""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate, stats

RC = 2.5


def test_special_cases(orc):
    # equal temperatures: delta = 0 -> always accepted, whatever u
    for u in (0.0, 0.5, 1.0 - 2**-53):
        assert orc.metropolis(-10.0, 50.0, 1.0, 1.0, u) == 1
    # cold replica with the higher energy: delta > 0 -> accepted
    assert orc.metropolis(5.0, 1.0, 0.7, 0.8, 1.0 - 2**-53) == 1
    # hot replica with much higher energy: delta -> -inf -> rejected
    assert orc.metropolis(-1e6, 1e6, 0.7, 0.8, 0.0) == 0
    # boundary: u < exp(delta) strictly
    d = (1 / 0.7 - 1 / 0.8) * (1.0 - 2.0)
    assert orc.metropolis(1.0, 2.0, 0.7, 0.8, math.exp(d)) == 0
    assert orc.metropolis(1.0, 2.0, 0.7, 0.8, np.nextafter(math.exp(d), 0)) == 1


def test_pattern_and_scaling(orc):
    R = 6
    Tl = 0.7 * 1.2 ** np.arange(R)
    slot = np.array([3, 0, 5, 1, 2, 4], np.int32)
    U = np.array([-100.0, -101, -99, -102, -98, -97])
    for k in (0, 1, 2, 7):
        new, alpha, recs = orc.exchange(Tl, slot, U, 1, k)
        # attempt k pairs ladder slots (j, j+1) with j = k mod 2
        assert [r.slot_lo for r in recs] == list(range(k % 2, R - 1, 2))
        inv = np.argsort(slot)
        for r in recs:
            assert (r.rep_a, r.rep_b) == (inv[r.slot_lo], inv[r.slot_lo + 1])
            assert r.u == orc.uniform53(1, k, min(r.rep_a, r.rep_b))
            d = (1 / Tl[r.slot_lo] - 1 / Tl[r.slot_lo + 1]) * (U[r.rep_a] - U[r.rep_b])
            assert r.accepted == int(d >= 0 or r.u < math.exp(d))
            if r.accepted:
                assert new[r.rep_a] == r.slot_lo + 1 and new[r.rep_b] == r.slot_lo
                assert alpha[r.rep_a] ** 2 == pytest.approx(Tl[r.slot_lo + 1] / Tl[r.slot_lo], rel=1e-15)
                assert alpha[r.rep_b] ** 2 == pytest.approx(Tl[r.slot_lo] / Tl[r.slot_lo + 1], rel=1e-15)
            else:
                assert new[r.rep_a] == slot[r.rep_a] and alpha[r.rep_a] == 1.0
        assert sorted(new) == list(range(R))


@pytest.mark.parametrize("max_distance", [1, 2])
def test_detailed_balance_enumeration(orc, max_distance):
    """Three replicas on a three-level system.  Each iteration resamples
    every replica exactly from Boltzmann at the temperature it holds, then
    applies one exchange attempt (nearest neighbours, or also the pair of
    ladder ends at distance 2).  The extended-ensemble distribution
    pi(sigma, c) = prod_r exp(-E(c_r)/T_sigma(r)) / Z(T_sigma(r)) / R! is
    stationary; the post-exchange histogram must match it."""
    E = np.array([0.0, 1.0, 2.5])
    Tl = np.array([0.4, 0.9, 2.0])
    R = 3

    def boltz(T):
        w = np.exp(-E / T)
        return w / w.sum()

    rng = np.random.default_rng(2024)
    slot = np.arange(R, dtype=np.int32)
    counts = {}
    n_iter = 30000
    for it in range(n_iter):
        c = np.array([rng.choice(3, p=boltz(Tl[slot[r]])) for r in range(R)])
        slot, _, _ = orc.exchange(Tl, slot, E[c], 77, it, max_distance=max_distance)
        # record the configuration each replica carried into the exchange
        key = (tuple(slot), tuple(c))
        counts[key] = counts.get(key, 0) + 1
    keys, expect = [], []
    for perm in itertools.permutations(range(R)):
        for c in itertools.product(range(3), repeat=R):
            p = 1.0 / math.factorial(R)
            for r in range(R):
                p *= boltz(Tl[perm[r]])[c[r]]
            keys.append((perm, c))
            expect.append(p * n_iter)
    obs = np.array([counts.get(k, 0) for k in keys], float)
    expect = np.array(expect)
    # pool cells with tiny expectation
    big = expect >= 5
    chi2 = (((obs[big] - expect[big]) ** 2) / expect[big]).sum()
    rest_o, rest_e = obs[~big].sum(), expect[~big].sum()
    if rest_e > 0:
        chi2 += (rest_o - rest_e) ** 2 / rest_e
    dof = big.sum()
    p = stats.chi2.sf(chi2, dof)
    assert p > 1e-4, (chi2, dof)


@pytest.mark.parametrize("R,D", [(2, 1), (7, 1), (8, 3), (9, 4), (16, 5)])
def test_distance_pattern(orc, R, D):
    """Non-nearest-neighbour pattern: every ladder slot is in at most one
    pair, pairs are the attempt's distance apart, every distance 1..D is
    drawn, and D = 1 is the alternating nearest-neighbour pattern."""
    Tl = 0.7 * 1.05 ** np.arange(R)
    slot = np.arange(R, dtype=np.int32)[::-1].copy()
    U = np.linspace(-100, -90, R)
    seen = set()
    for k in range(200):
        d = orc.pattern_distance(9, k, D)
        assert 1 <= d <= D
        seen.add(d)
        _, _, recs = orc.exchange(Tl, slot, U, 9, k, max_distance=D)
        used = [r.slot_lo for r in recs] + [r.slot_hi for r in recs]
        assert len(used) == len(set(used))
        assert all(r.slot_hi - r.slot_lo == d for r in recs)
        if D == 1:
            assert [r.slot_lo for r in recs] == list(range(k % 2, R - 1, 2))
        # a slot without a partner has none at distance d on either side
        o = (k % 2) * d
        for j in range(R):
            expect_pair = (j >= o and ((j - o) // d) % 2 == 0 and j + d < R) or \
                          (j - d >= o and ((j - d - o) // d) % 2 == 0)
            assert (j in used) == expect_pair
    assert seen == set(range(1, D + 1))


def gamma_acceptance(d, T1, T2):
    """<min(1, exp((1/T1-1/T2)(U1-U2)))> for U_i = T_i G_i, G_i ~ Gamma(d/2)
    (potential energy of a d-dimensional harmonic system)."""
    g = stats.gamma(d / 2.0)
    b = 1 / T1 - 1 / T2

    def inner(g1):
        u1 = T1 * g1
        # acceptance is 1 when U1 >= U2, i.e. g2 <= u1/T2
        acc1 = g.cdf(u1 / T2)
        f = lambda g2: math.exp(b * (u1 - T2 * g2)) * g.pdf(g2)
        acc2 = integrate.quad(f, u1 / T2, np.inf, limit=200)[0]
        return (acc1 + acc2) * g.pdf(g1)

    return integrate.quad(inner, 0, np.inf, limit=200)[0]


@pytest.mark.parametrize("d,T1,T2", [(6, 1.0, 1.3), (30, 0.7, 0.8), (100, 1.0, 1.05)])
def test_gamma_closed_form_acceptance(orc, d, T1, T2):
    expect = gamma_acceptance(d, T1, T2)
    rng = np.random.default_rng(d)
    n = 40000
    acc = 0
    for i in range(n):
        U1 = T1 * rng.gamma(d / 2.0)
        U2 = T2 * rng.gamma(d / 2.0)
        acc += orc.metropolis(U1, U2, T1, T2, orc.uniform53(3, i, 0))
    p = acc / n
    assert abs(p - expect) < 4 * math.sqrt(expect * (1 - expect) / n), (p, expect)


def test_sync_schedule(orc):
    """Synchronous variant: attempts after exactly N_x steps of every
    replica (<N_x> = N_x); replaying the same schedule as an injected
    asynchronous schedule gives a bit-identical run."""
    R, N, Nx = 4, 108, 20
    L = [orc.box_length(N, 0.8442)] * R
    Tl = 0.7 * (1.2 / 0.7) ** (np.arange(R) / (R - 1))
    a = orc.Ensemble([N] * R, L, Tl, RC, 0.3, 0.005, 1.0, 1)
    b = orc.Ensemble([N] * R, L, Tl, RC, 0.3, 0.005, 1.0, 1)
    a.run_sync(100, Nx)
    assert len(a.log) == sum(len(range(k % 2, R - 1, 2)) for k in range(5))
    for rec in a.log:
        assert rec.step_a == rec.step_b == (rec.attempt + 1) * Nx
    join = np.array([[(k + 1) * Nx] * R for k in range(5)], np.int64)
    b.run_schedule(join, 0)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    assert np.array_equal(a.slot, b.slot)
    assert [(r.accepted, r.u) for r in a.log] == [(r.accepted, r.u) for r in b.log]
    assert a.attempts.sum() == len(a.log)


def test_uneven_schedule_and_rescale(orc):
    """An asynchronous schedule (different join steps per replica): each
    replica arrives at its own step, and an accepted swap scales that
    replica's velocities by sqrt(T_new/T_old) at the boundary; everything
    else equals independent runs of the replicas."""
    R, N = 4, 108
    L = [orc.box_length(N, 0.8442)] * R
    Tl = np.array([1.0, 1.0001, 1.0002, 1.0003])  # near-equal: swaps accepted
    e = orc.Ensemble([N] * R, L, Tl, RC, 0.3, 0.005, 1.0, 1)
    x0, v0 = e.x.copy(), e.v.copy()
    join = np.array([[10, 12, 9, 15]], np.int64)
    e.run_schedule(join, 0)
    assert list(e.steps) == [10, 12, 9, 15]
    assert any(r.accepted for r in e.log)
    for rec in e.log:
        assert (rec.step_a, rec.step_b) == (join[0][rec.rep_a], join[0][rec.rep_b])
    alpha = np.ones(R)
    for rec in e.log:
        if rec.accepted:
            alpha[rec.rep_a] = math.sqrt(rec.T_b / rec.T_a)
            alpha[rec.rep_b] = math.sqrt(rec.T_a / rec.T_b)
    for r in range(R):
        a, b = e.off[r], e.off[r] + 3 * N
        rep = orc.Replica(x0[a:b], v0[a:b], L[r], RC)
        orc.md(rep, join[0][r], 0.3, 0.005, 1.0, Tl[r], 1, r)
        assert np.array_equal(rep.x, e.x[a:b])
        assert np.allclose(alpha[r] * rep.v, e.v[a:b], rtol=1e-15, atol=0)
        assert e.U[r] == rep.U
    assert sorted(e.temps()) == sorted(Tl)
