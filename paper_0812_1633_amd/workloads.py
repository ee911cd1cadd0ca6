"""Seeded synthetic workloads: configurations and injected states.

Input recipes only -- nothing here computes any part of the method.  Both
the GPU library (through the tests and the benchmark) and the oracle take
their inputs from here.

The paper's own workload is a synthetic Lennard-Jones liquid (Example
section: 4000 particles, density 0.844, cutoff 2.5, neighbour list to 3.0,
time step 0.005, geometric ladder from T = 0.7); the configurations below
are LJ liquids of that kind at the sizes of the benchmark ladder.
"""
from __future__ import annotations

import numpy as np

# name -> configuration.  N: atoms per replica (int, or "uneven"); T ladder
# geometric from Tmin to Tmax; precision is the form the configuration is
# quoted for.
CONFIGS = {
    # plain method, small: FP64, Langevin gamma = 1
    "lj-4x256-fp64": dict(R=4, N=256, rho=0.8442, Tmin=0.7, Tmax=1.2, rc=2.5, skin=0.3, dt=0.005,
                          gamma=1.0, Nx=100, steps=2000, seed=1),
    # headline: 32 replicas x 4000 atoms, FP32 forces + FP64 energies vs FP64
    "lj-32x4000": dict(R=32, N=4000, rho=0.8442, Tmin=0.7, Tmax=2.0, rc=2.5, skin=0.3, dt=0.005,
                       gamma=1.0, Nx=50, steps=10000, seed=1),
    # batched asynchronous form
    "lj-128x32000-async": dict(R=128, N=32000, rho=0.8442, Tmin=0.7, Tmax=3.0, rc=2.5, skin=0.3,
                               dt=0.005, gamma=1.0, Nx=50, steps=2000, seed=1),
    # uneven batch: N log-uniform in [500, 50000], rho uniform in [0.7, 0.9]
    "lj-64-uneven": dict(R=64, N="uneven", rho=None, Tmin=0.6, Tmax=2.5, rc=2.5, skin=0.3, dt=0.005,
                         gamma=1.0, Nx=20, steps=2000, seed=1),
    # large ladder
    "lj-256x108000": dict(R=256, N=108000, rho=0.8442, Tmin=0.7, Tmax=3.5, rc=3.0, skin=0.4, dt=0.004,
                          gamma=1.0, Nx=10, steps=5000, seed=1),
}


def ladder(Tmin, Tmax, R):
    """Geometric temperature ladder T_k = Tmin (Tmax/Tmin)^(k/(R-1))."""
    if R == 1:
        return np.array([float(Tmin)])
    return float(Tmin) * (float(Tmax) / float(Tmin)) ** (np.arange(R) / (R - 1.0))


def uneven_sizes(R=64, seed=1, nmin=500, nmax=50000, rho_lo=0.7, rho_hi=0.9):
    """Atom counts log-uniform in [nmin, nmax] and densities uniform in
    [rho_lo, rho_hi] (numpy PCG64 stream of the given seed)."""
    g = np.random.default_rng(seed)
    u = g.random(R)
    w = g.random(R)
    N = np.rint(np.exp(np.log(nmin) + u * np.log(nmax / nmin))).astype(np.int32)
    rho = rho_lo + (rho_hi - rho_lo) * w
    return N, rho


def expand(name, **over):
    """Configuration with per-replica arrays: N (R,), rho (R,), T (R,)."""
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    R = cfg["R"]
    if isinstance(cfg["N"], str):
        N, rho = uneven_sizes(R, cfg["seed"])
    else:
        N = np.full(R, int(cfg["N"]), np.int32)
        rho = np.full(R, float(cfg["rho"]))
    cfg["N_list"] = N
    cfg["rho_list"] = rho
    cfg["T_list"] = ladder(cfg["Tmin"], cfg["Tmax"], R)
    return cfg


def grid_unit(L):
    """Spacing of the 32-bit periodic position grid of a box of side L."""
    return float(L) * 2.0 ** -32


def snap_to_grid(x, L):
    """Round positions to the 32-bit grid of the box (wrapped into
    [-L/2, L/2)).  Grid positions are exact in FP32-grid, FP64 and the
    library's fixed-point representation alike (L is a multiple of 2^-12)."""
    s = grid_unit(L)
    k = np.rint(np.asarray(x, np.float64) / s).astype(np.int64)
    k = ((k + 2**31) % 2**32) - 2**31
    return k.astype(np.float64) * s


def round_f32(v):
    """Velocities representable in FP32 (exact in both precisions)."""
    return np.asarray(v, np.float64).astype(np.float32).astype(np.float64)


def perturbed_fcc(N, L, amp, seed):
    """N sites of an FCC lattice filling the box (vacancies at random when
    4 n^3 > N), each displaced by a Gaussian of standard deviation amp: a
    dense, disordered configuration with liquid-like pair distances."""
    n = 1
    while 4 * n**3 < N:
        n += 1
    a = L / n
    g = np.random.default_rng(seed)
    b = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    cells = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    sites = (cells[:, None, :] + b[None] + 0.25).reshape(-1, 3) * a - 0.5 * L
    if len(sites) > N:
        sites = sites[np.sort(g.choice(len(sites), N, replace=False))]
    x = sites + amp * g.standard_normal(sites.shape)
    return snap_to_grid(x, L)


def maxwell(N, T, seed):
    """Velocities with the Maxwell-Boltzmann distribution at T (m = 1),
    FP32-representable."""
    g = np.random.default_rng(seed)
    return round_f32(np.sqrt(T) * g.standard_normal((N, 3)))
