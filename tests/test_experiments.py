"""Host logic of the Example-section experiments (no GPU): the log-T path
reconstruction from exchange records and the diffusion estimator, pinned on
synthetic processes whose diffusion coefficient is known in closed form."""
from collections import namedtuple

import numpy as np
import pytest

from paper_0812_1633_amd import experiments as E

Rec = namedtuple("Rec", "attempt slot_lo rep_a rep_b step_a step_b accepted")


def test_paper_ladder():
    T = E.paper_ladder(5)
    assert T[0] == 0.7
    assert np.allclose(T[1:] / T[:-1], 1.0275, rtol=1e-15, atol=0)


def test_logT_paths_follow_accepted_swaps():
    T = np.array([1.0, 2.0, 4.0])
    # attempt 0 pairs slots (0,1): replicas 0,1 swap at steps 10 / 12;
    # attempt 1 pairs slots (1,2): replica 0 (now slot 1) and 2 refuse;
    # attempt 2 pairs (0,1) again: replicas 1 (slot 0) and 0 (slot 1) swap back
    log = [Rec(0, 0, 0, 1, 10, 12, 1), Rec(1, 1, 0, 2, 20, 21, 0), Rec(2, 0, 1, 0, 33, 30, 1)]
    p = E.logT_paths(log, T, [0, 1, 2], [0, 0, 0])
    lt = np.log(T)
    assert p[0] == [(0, lt[0]), (10, lt[1]), (30, lt[0])]
    assert p[1] == [(0, lt[1]), (12, lt[0]), (33, lt[1])]
    assert p[2] == [(0, lt[2])]
    assert E._sample(p[0], np.array([0, 9, 10, 29, 30, 99])).tolist() == [lt[0], lt[0], lt[1], lt[1], lt[0], lt[0]]


@pytest.mark.parametrize("p,stride", [(0.3, 5), (0.6, 1), (0.2, 20)])
def test_diffusion_estimator_recovers_known_D(p, stride):
    """Independent jumps of +-delta with probability p every `stride` steps:
    MSD(lag) = p delta^2 lag / stride exactly, so D = p delta^2 / (2 stride dt)."""
    g = np.random.default_rng(int(100 * p) + stride)
    R, nattempt, delta, dt = 400, 400, np.log(1.0275), 0.005
    paths = []
    for _ in range(R):
        jumps = g.random(nattempt) < p
        sign = np.where(g.random(nattempt) < 0.5, -1.0, 1.0)
        steps = stride * np.arange(1, nattempt + 1)
        val = np.cumsum(np.where(jumps, sign * delta, 0.0))
        paths.append([(0, 0.0)] + [(int(s), float(v)) for s, v, j in zip(steps, val, jumps) if j])
    t0 = np.zeros(R, np.int64)
    t1 = np.full(R, stride * nattempt, np.int64)
    D, lags, m = E.diffusion_coefficient(paths, t0, t1, dt, stride)
    D_true = p * delta ** 2 / (2 * stride * dt)
    assert D == pytest.approx(D_true, rel=0.06)
    # the MSD itself is linear with the closed-form slope
    assert np.allclose(m, p * delta ** 2 * lags / stride, rtol=0.08)


def test_expected_min1_exp_closed_form():
    """E[min(1, e^x)] for Gaussian x against Monte Carlo, and the
    detailed-balance case m = -v/2, where it equals erfc(sqrt(v) / (2 sqrt 2))."""
    import math
    from paper_0812_1633_amd import experiments as E
    g = np.random.default_rng(0)
    for m, v in ((-0.3, 0.6), (0.2, 0.1), (-2.0, 1.5), (-0.05, 0.1)):
        x = g.normal(m, np.sqrt(v), 400000)
        mc = np.minimum(1.0, np.exp(x)).mean()
        assert E.expected_min1_exp(m, v) == pytest.approx(mc, abs=3e-3)
    for v in (0.1, 1.0, 4.0):
        assert E.expected_min1_exp(-v / 2, v) == pytest.approx(math.erfc(math.sqrt(v) / (2 * math.sqrt(2))), rel=1e-12)


def test_ladder_acceptance_on_synthetic_log():
    """Synthetic exchange records with Gaussian energies of known mean and
    variance per temperature: the per-pair estimate matches the closed form
    and the measured rate is the records' mean."""
    from types import SimpleNamespace
    from paper_0812_1633_amd import experiments as E
    T = np.array([1.0, 1.05, 1.1, 1.16])
    mu = -5000.0 + 900.0 * (T - 1.0) * 10
    sd = np.sqrt(1.0 * T ** 2 * 400.0)
    g = np.random.default_rng(1)
    recs = []
    for k in range(40000):
        j0 = k % 2
        for j in range(j0, len(T) - 1, 2):
            ua, ub = g.normal(mu[j], sd[j]), g.normal(mu[j + 1], sd[j + 1])
            recs.append(SimpleNamespace(attempt=k, slot_lo=j, slot_hi=j + 1, U_a=ua, U_b=ub, accepted=int(k % 3 == 0)))
    rows = E.ladder_acceptance(recs, T, 0)
    for r in rows:
        j = r["j"]
        dB = 1 / T[j] - 1 / T[j + 1]
        expect = E.expected_min1_exp(dB * (mu[j] - mu[j + 1]), dB * dB * (sd[j] ** 2 + sd[j + 1] ** 2))
        assert r["gaussian"] == pytest.approx(expect, abs=0.01)
        assert r["measured"] == pytest.approx(1 / 3, abs=0.01)
        assert r["cv_conf"] == pytest.approx(400.0, rel=0.05)
