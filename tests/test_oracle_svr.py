"""Pins of the oracle's stochastic velocity rescale (the thermostat the
Example section names; Bussi, Donadio and Parrinello, J. Chem. Phys. 126,
014101 (2007)) against what the mathematics fixes, independently of the
formula as written in the oracle:

* the rescale alone, iterated with exact normal and chi-square draws, leaves
  the kinetic energy distributed as Gamma(N_f/2, scale T) (the canonical
  law it is built to sample) -- a dropped term, a wrong sign of the cross
  term or a wrong N_f scaling changes the stationary law;
* E[K' | K] = c K + (1 - c) Kbar (exponential relaxation to Kbar);
* limits: c = 1 leaves the velocities unchanged; c = 0 draws K' afresh
  from the canonical law whatever K was; K = 0 stays unchanged;
* the Philox noise: R1 standard normal, S chi-square with 3N - 4 degrees of
  freedom (its mean pins the number of terms);
* a Lennard-Jones run under the rescale: <K> = N_f T / 2 and
  Var K = N_f T^2 / 2 (canonical kinetic energy), total momentum conserved.
"""
import numpy as np
import pytest
from scipy import stats

import oracle


def test_limits():
    g = np.random.default_rng(1)
    for _ in range(50):
        K, Kbar, Nf = g.uniform(1, 50), g.uniform(1, 50), int(g.integers(3, 300))
        R1, S = g.normal(), g.chisquare(Nf - 1)
        assert oracle.svr_factor(K, Kbar, Nf, 1.0, R1, S) == 1.0
        a0 = oracle.svr_factor(K, Kbar, Nf, 0.0, R1, S)
        assert a0 * a0 * K == pytest.approx(Kbar * (R1 * R1 + S) / Nf, rel=1e-13)
    assert oracle.svr_factor(0.0, 5.0, 10, 0.5, 0.3, 9.0) == 1.0


@pytest.mark.parametrize("Nf,T,c", [(12, 1.5, 0.3), (3, 0.8, 0.9), (60, 2.0, 0.0)])
def test_stationary_law_is_canonical(Nf, T, c):
    g = np.random.default_rng(Nf)
    n, burn, thin = 120000, 2000, 20
    R1 = g.normal(size=n)
    S = g.chisquare(Nf - 1, size=n)
    K = 0.1 * Nf * T  # far from equilibrium on purpose
    Kbar = 0.5 * Nf * T
    out = np.empty(n)
    for i in range(n):
        a = oracle.svr_factor(K, Kbar, Nf, c, R1[i], S[i])
        K *= a * a
        out[i] = K
    ks = out[burn::thin]
    law = stats.gamma(a=0.5 * Nf, scale=T)
    assert stats.kstest(ks, law.cdf).pvalue > 1e-4
    # moments: mean N_f T / 2, variance N_f T^2 / 2
    m_err = 5 * np.sqrt(law.var() / ks.size)
    assert abs(ks.mean() - law.mean()) < m_err
    assert ks.var() == pytest.approx(law.var(), rel=0.08)


def test_conditional_mean():
    g = np.random.default_rng(7)
    Nf, K, Kbar, c = 40, 11.0, 25.0, 0.6
    n = 200000
    R1 = g.normal(size=n)
    S = g.chisquare(Nf - 1, size=n)
    Kn = np.array([K * oracle.svr_factor(K, Kbar, Nf, c, R1[i], S[i]) ** 2 for i in range(n)])
    expect = c * K + (1 - c) * Kbar
    assert abs(Kn.mean() - expect) < 5 * Kn.std() / np.sqrt(n)


def test_noise_law():
    seed, N, r = 3, 10, 2
    draws = np.array([oracle.svr_noise(seed, N, r, s) for s in range(1, 3001)])
    R1, S = draws[:, 0], draws[:, 1]
    n = len(R1)
    assert abs(R1.mean()) < 5 / np.sqrt(n)
    assert R1.var() == pytest.approx(1.0, rel=0.1)
    dof = 3 * N - 4
    assert abs(S.mean() - dof) < 5 * np.sqrt(2 * dof / n)
    assert S.var() == pytest.approx(2 * dof, rel=0.12)
    assert abs(np.corrcoef(R1, S)[0, 1]) < 5 / np.sqrt(n)
    # different replicas and steps draw different numbers
    assert oracle.svr_noise(seed, N, r, 5) != oracle.svr_noise(seed, N, r + 1, 5)


@pytest.mark.parametrize("N,rho,nsamp,mean_tol", [(256, 0.8442, 1000, 0.01), (64, 0.3, 3000, 0.006)])
def test_lj_run_is_canonical(N, rho, nsamp, mean_tol):
    """LJ atoms at T = 1.1 under velocity Verlet + the rescale (tau = 0.1):
    the kinetic energy has the canonical mean N_f T/2 with N_f = 3N - 3
    (the small system resolves the 3 removed degrees of freedom) and the
    canonical variance; the total momentum stays zero."""
    T, rc, skin, dt = 1.1, 2.5, 0.3, 0.005
    L = oracle.box_length(N, rho)
    x, v = oracle.init_replica(N, L, T, 5, 0)
    rep = oracle.Replica(x, v, L, rc)
    oracle.md(rep, 1000, skin, dt, 0.0, T, 5, 0, thermostat="svr", tau=0.1)  # equilibrate
    Nf = 3 * N - 3
    Ks = []
    for _ in range(nsamp):
        oracle.md(rep, 10, skin, dt, 0.0, T, 5, 0, thermostat="svr", tau=0.1)
        Ks.append(0.5 * (rep.v * rep.v).sum())
    Ks = np.array(Ks)
    assert Ks.mean() == pytest.approx(0.5 * Nf * T, rel=mean_tol)
    assert Ks.var() == pytest.approx(0.5 * Nf * T * T, rel=0.25)
    P = rep.v.reshape(-1, 3).sum(0)
    assert np.abs(P).max() < 1e-9
