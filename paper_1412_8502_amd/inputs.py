"""Seeded synthetic initial states shaped like the paper's workloads.

This module draws random numbers and nothing else: it holds none of the
method's arithmetic (no forces, no integration, no clustering), so the GPU
library and the CPU oracle can both be fed from it without sharing code.

Recipe (the paper starts every run from uniformly distributed random
positions, Sec. III.B, and gives N, the proton fraction Y_P, the density n and
the temperature T of each run, Sec. II.B.2 and III):

* box side L = (N / n)^(1/3) fm;
* positions i.i.d. uniform in [0, L)^3;
* Z = round(Y_P N) protons, particle ids 0..Z-1 are the protons;
* velocities i.i.d. normal with standard deviation sqrt(T / M) per component
  (Maxwell-Boltzmann at temperature T, in units of c).
All draws come from numpy's PCG64 generator with the given seed.
"""
from __future__ import annotations

import numpy as np

MASS_MEV = 939.0


def box_side(n_particles: int, density: float) -> float:
    """Side (fm) of the cube holding n_particles at density (fm^-3)."""
    return float((n_particles / density) ** (1.0 / 3.0))


def proton_count(n_particles: int, y_p: float) -> int:
    return int(round(y_p * n_particles))


def make_state(n_particles: int, y_p: float, density: float, temperature: float,
               seed: int, mass: float = MASS_MEV):
    """Returns dict(pos [N,3] f64 in [0,L), vel [N,3] f64 (c), species [N] u8
    (1 = proton, 0 = neutron), L, Z, seed, and the recipe parameters)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = box_side(n_particles, density)
    pos = rng.random((n_particles, 3)) * L
    pos[pos >= L] = 0.0  # a product that rounded up to L is the same point as 0
    vel = rng.standard_normal((n_particles, 3)) * np.sqrt(temperature / mass)
    Z = proton_count(n_particles, y_p)
    species = np.zeros(n_particles, np.uint8)
    species[:Z] = 1
    return dict(pos=pos, vel=vel, species=species, L=L, Z=Z, seed=seed,
                n=n_particles, y_p=y_p, density=density, T=temperature)


# ---- the workloads the benchmark and parity tests use -------------------
# name -> (N, Y_P, n [fm^-3], T [MeV], seed)
WORKLOADS = {
    # small case the oracle finishes in seconds
    "n3200_yp040_n0.040": (3200, 0.40, 0.040, 1.0, 1000),
    # the headline single-system workload: 51 200 nucleons at 0.08 fm^-3
    "n51200_yp020_n0.080": (51200, 0.20, 0.080, 0.75, 1001),
    # decompression start state
    "n51200_yp030_n0.080": (51200, 0.30, 0.080, 0.5, 1003),
    # large: 409 600 nucleons
    "n409600_yp040_n0.080": (409600, 0.40, 0.080, 1.0, 1004),
    "n409600_yp005_n0.080": (409600, 0.05, 0.080, 1.0, 1005),
}


def workload(name: str):
    N, yp, dens, T, seed = WORKLOADS[name]
    return make_state(N, yp, dens, T, seed)


def batch_grid(master_seed: int = 2000):
    """The 15-run (Y_P, T) grid of the paper's production runs (Sec. III.B):
    Y_P in {0.05, 0.10, 0.20, 0.30, 0.40} x T in {0.5, 0.75, 1.0} MeV.  Each
    system's N is drawn from {6400, 12800, 25600, 51200} and its density
    uniformly in [0.02, 0.08] fm^-3 from the master seed; system s then uses
    seed master_seed + 1 + s.  Returns a list of make_state dicts."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    systems = []
    s = 0
    for yp in (0.05, 0.10, 0.20, 0.30, 0.40):
        for T in (0.5, 0.75, 1.0):
            N = int(rng.choice([6400, 12800, 25600, 51200]))
            dens = float(rng.uniform(0.02, 0.08))
            systems.append(make_state(N, yp, dens, T, master_seed + 1 + s))
            s += 1
    return systems
