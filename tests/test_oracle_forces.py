"""Pins of the oracle's Lennard-Jones forces and energy (Example section:
LJ liquid, cutoff 2.5, LJ units).

Pinned by: two-atom closed forms, the perfect FCC lattice (zero force by
symmetry, energy from an independent enumeration of lattice shells), the
gradient identity F = -dU/dx by central differences, Newton's third law, and
brute force over explicit periodic images on tiny systems.
"""
import itertools

import numpy as np
import pytest

RC = 2.5


def two_atoms(r, L=10.0, axis=(1.0, 0.0, 0.0)):
    a = np.asarray(axis, float)
    a /= np.linalg.norm(a)
    return np.array([[0.0, 0.0, 0.0], r * a])


def test_shift_value(orc):
    # u_lj(2.5) = 4 (2.5^-12 - 2.5^-6)
    assert orc.lj_shift(2.5) == pytest.approx(4 * (2.5**-12 - 2.5**-6), rel=1e-15)
    assert orc.lj_shift(2.5) == pytest.approx(-0.0163169, abs=1e-7)
    assert orc.lj_shift(3.0) == pytest.approx(-0.0054794, abs=1e-7)


def test_two_atom_minimum(orc):
    rmin = 2.0 ** (1.0 / 6.0)
    F, U, _ = orc.forces(two_atoms(rmin), 10.0, RC)
    assert np.abs(F).max() < 1e-12
    assert U == pytest.approx(-1.0 - orc.lj_shift(RC), rel=1e-14)


def test_two_atom_r1(orc):
    # u(1) = 0 - shift, |f| = 24, repulsive: atom 0 pushed away from atom 1
    F, U, _ = orc.forces(two_atoms(1.0, axis=(1, 2, -2)), 10.0, RC)
    assert U == pytest.approx(-orc.lj_shift(RC), rel=1e-14)
    assert np.linalg.norm(F[0]) == pytest.approx(24.0, rel=1e-14)
    d = np.array([1, 2, -2]) / 3.0
    assert F[0] @ d == pytest.approx(-24.0, rel=1e-14)
    assert np.allclose(F[0], -F[1], atol=0, rtol=0)


def test_two_atom_attractive_and_cutoff(orc):
    r = 1.5
    F, U, _ = orc.forces(two_atoms(r), 10.0, RC)
    f = 24 * (2 * r**-13 - r**-7)  # -du/dr
    assert f < 0
    assert F[1, 0] == pytest.approx(f, rel=1e-13)  # atom 1 pulled towards atom 0
    assert U == pytest.approx(4 * (r**-12 - r**-6) - orc.lj_shift(RC), rel=1e-13)
    # at and beyond r_c: nothing (strict r < r_c)
    for rr in (RC, RC + 1e-9, 3.0):
        F, U, _ = orc.forces(two_atoms(rr), 10.0, RC)
        assert U == 0.0 and np.all(F == 0.0)
    # just inside: energy continuous (-> 0), force not (truncated)
    F, U, _ = orc.forces(two_atoms(RC - 1e-9), 10.0, RC)
    assert abs(U) < 1e-9
    assert F[1, 0] == pytest.approx(24 * (2 * RC**-13 - RC**-7), rel=1e-6)


def test_two_atom_across_boundary(orc):
    """Minimum image: atoms at -L/2+0.4 and L/2-0.6 are 1.0 apart."""
    L = 8.0
    x = np.array([[-L / 2 + 0.4, 0.1, 0.2], [L / 2 - 0.6, 0.1, 0.2]])
    F, U, _ = orc.forces(x, L, RC)
    assert U == pytest.approx(-orc.lj_shift(RC), rel=1e-12)
    # atom 0 is pushed in +x (away from its image neighbour at -L/2-0.6)
    assert F[0, 0] == pytest.approx(24.0, rel=1e-12)


def fcc_shell_energy(a, rc):
    """Energy per atom of a perfect FCC crystal with cubic cell a: half the
    sum over lattice vectors (a/2)(h,k,l), h+k+l even, 0 < |v| < rc."""
    m = int(np.ceil(2 * rc / a)) + 1
    shift = 4 * (rc**-12 - rc**-6)
    e = 0.0
    for h, k, l in itertools.product(range(-m, m + 1), repeat=3):
        if (h + k + l) % 2 or (h, k, l) == (0, 0, 0):
            continue
        r = 0.5 * a * np.sqrt(h * h + k * k + l * l)
        if r < rc:
            e += 4 * (r**-12 - r**-6) - shift
    return 0.5 * e


@pytest.mark.parametrize("n,rho", [(4, 0.8442), (5, 0.8442), (5, 1.0), (6, 0.7)])
def test_fcc_lattice(orc, n, rho):
    N = 4 * n**3
    L = orc.box_length(N, rho)
    x, _ = orc.init_replica(N, L, 1.0, 1, 0)
    F, U, _ = orc.forces(x, L, RC)
    assert np.abs(F).max() < 1e-11
    assert U / N == pytest.approx(fcc_shell_energy(L / n, RC), rel=1e-12)


def random_liquid(N, L, seed, dmin=0.95):
    """Random positions with no pair closer than dmin (rejection)."""
    rng = np.random.default_rng(seed)
    x = np.zeros((0, 3))
    while len(x) < N:
        p = rng.uniform(-L / 2, L / 2, 3)
        if len(x):
            d = x - p
            d -= L * np.round(d / L)
            if (d * d).sum(1).min() < dmin * dmin:
                continue
        x = np.vstack([x, p])
    return x


def test_gradient_identity(orc):
    """F = -grad U by central differences (the shifted energy is continuous
    at r_c, so the identity holds away from pairs sitting on the cutoff)."""
    L = 6.0
    x = random_liquid(60, L, 3)
    F, U, _ = orc.forces(x, L, RC)
    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(40):
        i, k = rng.integers(60), rng.integers(3)
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        up = orc.forces(xp, L, RC)[1]
        um = orc.forces(xm, L, RC)[1]
        fd = -(up - um) / (2 * h)
        assert fd == pytest.approx(F[i, k], rel=2e-6, abs=2e-6)


def test_newton_third_law_and_virial(orc):
    L = 7.0
    x = random_liquid(100, L, 5)
    F, U, W = orc.forces(x, L, RC)
    assert np.abs(F.sum(0)).max() < 1e-10
    # virial W = sum_i x_i . F_i is not translation invariant under periodic
    # images; use the pair form on a system that does not wrap instead
    x2 = random_liquid(30, 30.0, 6) * 0.2  # compact cluster, far from the box faces
    F2, U2, W2 = orc.forces(x2, 30.0, RC)
    assert W2 == pytest.approx(float((x2 * F2).sum()), rel=1e-10, abs=1e-9)


def test_explicit_images_brute_force(orc):
    """Tiny boxes: the sum over all pairs and all periodic images within r_c
    (each pair has at most one image within r_c < L/2)."""
    rng = np.random.default_rng(11)
    for trial in range(5):
        N = int(rng.integers(3, 9))
        L = 5.2 + trial * 0.1
        x = random_liquid(N, L, 100 + trial, dmin=0.9)
        F_ref = np.zeros((N, 3))
        U_ref = 0.0
        shift = 4 * (RC**-12 - RC**-6)
        for i in range(N):
            for j in range(N):
                for img in itertools.product((-1, 0, 1), repeat=3):
                    if i == j and img == (0, 0, 0):
                        continue
                    d = x[i] - (x[j] + L * np.array(img))
                    r2 = d @ d
                    if r2 < RC * RC:
                        r = np.sqrt(r2)
                        U_ref += 0.5 * (4 * (r**-12 - r**-6) - shift)
                        F_ref[i] += 24 * (2 * r**-14 - r**-8) * d
        F, U, _ = orc.forces(x, L, RC)
        assert U == pytest.approx(U_ref, rel=1e-12, abs=1e-12)
        assert np.allclose(F, F_ref, rtol=1e-11, atol=1e-11)


def _force_on_all(orc, x, L, rc):
    rows = [orc.force_on(x, L, rc, i) for i in range(len(x))]
    return np.array([f for f, _ in rows]), np.array([e for _, e in rows])


@pytest.mark.parametrize("rc", [2.5, 3.0])
def test_force_on_rows(orc, rc):
    """The one-atom force (the checker of sampled atoms in large systems)
    equals the corresponding row of the all-pairs forces, and its pair-energy
    sums add up to twice the potential energy (every pair seen from both of
    its atoms)."""
    L = 7.5
    x = random_liquid(120, L, 21)
    F, U, _ = orc.forces(x, L, rc)
    Fr, e = _force_on_all(orc, x, L, rc)
    scale = np.sqrt((F * F).sum(1).mean())
    assert np.abs(Fr - F).max() <= 1e-13 * scale
    assert e.sum() == pytest.approx(2.0 * U, rel=1e-13)
    assert np.abs(Fr.sum(0)).max() < 1e-10  # Newton's third law, from the rows


def test_force_on_is_minus_gradient(orc):
    """The one-atom force is minus the derivative of the energy that the
    one-atom energy sums define (U = half their total), by central
    differences: a check that uses force_on alone."""
    L = 6.0
    x = random_liquid(50, L, 8)
    h = 1e-6

    def U_of(y):
        return 0.5 * sum(orc.force_on(y, L, RC, i)[1] for i in range(len(y)))

    rng = np.random.default_rng(4)
    for _ in range(12):
        i, k = int(rng.integers(50)), int(rng.integers(3))
        Fi, _ = orc.force_on(x, L, RC, i)
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fd = -(U_of(xp) - U_of(xm)) / (2 * h)
        assert fd == pytest.approx(Fi[k], rel=2e-6, abs=2e-6)
