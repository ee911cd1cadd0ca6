"""Pins of the oracle's random numbers.

Philox4x32-10 (Salmon et al., SC'11) is pinned against rocRAND's
host-callable Philox engine, an implementation independent of the oracle.
Box-Muller normals and the exchange uniforms are pinned by their
distributions (Kolmogorov-Smirnov) and by the closed-form identities of the
transform.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rocrand") / "philox_rocrand")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "support", "philox_rocrand.cpp")],
                          cwd=str(tmp_path_factory.getbasetemp()))
    return exe


def test_philox_matches_rocrand(orc, rocrand_philox):
    rng = np.random.default_rng(12345)
    rows = []
    for _ in range(300):
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        c[1] = c[1] % (2**30)  # rocRAND's offset argument is 4*(c0 + 2^32 c1) < 2^64
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        rows.append((c, k))
    rows += [(np.array([0, 0, 0, 0], np.uint64), np.array([0, 0], np.uint64)),
             (np.array([2**32 - 1, 0, 2**32 - 1, 2**32 - 1], np.uint64), np.array([2**32 - 1] * 2, np.uint64))]
    inp = "\n".join(" ".join(str(int(t)) for t in list(c) + list(k)) for c, k in rows) + "\n"
    out = subprocess.run([rocrand_philox], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [tuple(int(t) for t in line.split()) for line in out.strip().splitlines()]
    assert len(ref) == len(rows)
    for (c, k), r in zip(rows, ref):
        got = tuple(int(t) for t in orc.philox4x32_10(c.astype(np.uint32), k.astype(np.uint32)))
        assert got == r, (c, k, got, r)


def test_normals_are_standard_normal(orc):
    z = np.array([orc.normals3(7, i, 3, 5, 1) for i in range(40000)]).reshape(-1)
    assert abs(z.mean()) < 4.0 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4.0 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the three components are uncorrelated
    zz = z.reshape(-1, 3)
    c = np.corrcoef(zz.T)
    assert np.all(np.abs(c - np.eye(3)) < 4.0 / np.sqrt(zz.shape[0]))


def test_box_muller_identity(orc):
    """z0^2 + z1^2 = -2 ln u0 and atan2(z1, z0) = 2 pi u1 (mod 2 pi), with
    u = (w + 1/2) 2^-32 of the Philox words of the same counter."""
    for i in range(50):
        seed, c0, c1, c2, p = 99, i, 11, 3, 1
        w = orc.philox4x32_10([c0, c1, c2, p], [seed & 0xFFFFFFFF, seed >> 32])
        u = (w.astype(np.float64) + 0.5) / 2.0**32
        z = orc.normals3(seed, c0, c1, c2, p)
        assert z[0] ** 2 + z[1] ** 2 == pytest.approx(-2 * np.log(u[0]), rel=1e-12)
        ang = np.arctan2(z[1], z[0]) % (2 * np.pi)
        assert ang == pytest.approx(2 * np.pi * u[1], rel=1e-9, abs=1e-9)
        assert abs(z[2]) == pytest.approx(np.sqrt(-2 * np.log(u[2])) * abs(np.cos(2 * np.pi * u[3])), rel=1e-12)


def test_uniform53(orc):
    u = np.array([orc.uniform53(1, k, r) for k in range(2000) for r in range(10)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    # 53-bit: multiples of 2^-53, built from the top bits of words 0 and 1
    w = orc.philox4x32_10([5, 0, 3, 2], [1, 0])
    expect = ((int(w[0]) >> 5) * 2**26 + (int(w[1]) >> 6)) / 2.0**53
    assert orc.uniform53(1, 5, 3) == expect
    # the uniform depends on (attempt, lower id) only: different attempts differ
    assert orc.uniform53(1, 5, 3) != orc.uniform53(1, 6, 3)
    assert orc.uniform53(1, 5, 3) != orc.uniform53(2, 5, 3)
