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
