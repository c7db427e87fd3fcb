"""Decompression runs in the setting of the paper's expansion study (Sec.
III.B and Table II): N nucleons start uniformly at random at n = 0.08 fm^-3,
are equilibrated at temperature T in a fixed box, and are then stretched at
the rate xi_dot (Eq. 3a: L(t) = L(0)(1 + xi_dot t), positions not rescaled)
for t = ((n0 / n_end)^(1/3) - 1) / xi_dot, i.e. until the density reaches
n_end; the velocity rescale to T every 100 steps stays on throughout.  The
final configuration is analysed with the cluster algorithm of Sec. II.C
(r_pp = 4.5 fm, r_np = 3 fm): the mass fraction of free neutrons and the mean
and population standard deviation of A and Z over clusters with A >= 12, the
statistics Table II reports, plus the mass fraction in light clusters
(A < 12) and the largest cluster.

Every step runs through the library (mixed precision, cell sweeps); this
module only sequences the runs and reduces the labels on the host.

    python -m paper_1412_8502_amd.expansion --yp 0.2 --xi -5 [--equil 500000]

prints one JSON line per run.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def cluster_stats(label: np.ndarray, species: np.ndarray, a_min: int = 12) -> dict:
    """Table II statistics from cluster labels (-1 = free neutron)."""
    n = label.size
    bound = label >= 0
    K = int(label.max()) + 1 if bound.any() else 0
    A = np.bincount(label[bound], minlength=K)
    Z = np.bincount(label[bound], weights=(species[bound] == 1), minlength=K).astype(np.int64)
    heavy = A >= a_min
    free_n = int(((~bound) & (species == 0)).sum())
    out = {"clusters": K, "clusters_A_ge_12": int(heavy.sum()),
           "mass_fraction_free_neutrons": free_n / n,
           "mass_fraction_light_clusters": float(A[~heavy].sum()) / n,
           "largest_A": int(A.max()) if K else 0}
    if heavy.any():
        out.update(mean_A=float(A[heavy].mean()), sd_A=float(A[heavy].std()),
                   mean_Z=float(Z[heavy].mean()), sd_Z=float(Z[heavy].std()))
    return out


def run(n: int, yp: float, T: float, xi_log10: float, equil_steps: int, seed: int,
        n0: float = 0.08, n_end: float = 0.01, dt: float = 2.0, report_every: int = 50000,
        log=print, return_state: bool = False):
    """One run; returns the result dict (and, with return_state, also the
    final positions [n][3] and box side as numpy / float)."""
    import torch
    from . import binding as B
    from .inputs import make_state

    st = make_state(n, yp, n0, T, seed)
    dev = torch.device("cuda:0")
    pos = torch.tensor(st["pos"], device=dev)
    vel = torch.tensor(st["vel"], device=dev)
    sp = torch.tensor(st["species"], device=dev)
    L0 = st["L"]
    t0 = time.perf_counter()
    # equilibration in the fixed box
    sim = B.Sim(pos, vel, sp, L0, dt=dt, xi_dot=0.0, T=T, rescale_every=100,
                precision=B.PASTA_MIXED)
    done = 0
    while done < equil_steps:
        k = min(report_every, equil_steps - done)
        sim.step(k)
        done += k
        ep = sim.energies()["epot"]
        log(f"  equilibration {done}/{equil_steps} steps: E_pot/N = {ep / n:.4f} MeV "
            f"({time.perf_counter() - t0:.0f} s)")
    del sim
    # expansion: a new box law from the equilibrated state (step 0 = start)
    xi = 10.0 ** xi_log10
    stretch = (n0 / n_end) ** (1.0 / 3.0)
    steps = int(round((stretch - 1.0) / xi / dt))
    sim = B.Sim(pos, vel, sp, L0, dt=dt, xi_dot=xi, T=T, rescale_every=100,
                precision=B.PASTA_MIXED, L_max=L0 * stretch * (1.0 + 1e-9))
    done = 0
    while done < steps:
        k = min(report_every, steps - done)
        sim.step(k)
        done += k
        en = sim.energies()
        ep, L = en["epot"], en["L"]
        log(f"  expansion {done}/{steps} steps: n = {n / L ** 3:.5f} fm^-3, E_pot/N = "
            f"{ep / n:.4f} MeV ({time.perf_counter() - t0:.0f} s)")
    L_end = sim.energies()["L"]
    del sim
    cl = B.pasta_cluster(pos, sp, L_end)
    stats = cluster_stats(cl["label"].cpu().numpy(), st["species"])
    res = {"N": n, "Y_P": yp, "T_MeV": T, "log10_xi_dot": xi_log10, "dt_fm_c": dt,
           "equilibration_steps": equil_steps, "expansion_steps": steps,
           "n_final": n / L_end ** 3, "seed": seed, "seconds": time.perf_counter() - t0,
           **stats}
    if return_state:
        return res, pos.cpu().numpy(), L_end
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=51200)
    ap.add_argument("--yp", type=float, nargs="+", default=[0.2])
    ap.add_argument("--T", type=float, default=1.0)
    ap.add_argument("--xi", type=float, default=-5.0, help="log10 of xi_dot in c/fm")
    ap.add_argument("--equil", type=int, default=500000)
    ap.add_argument("--seed", type=int, default=3000)
    args = ap.parse_args(argv)
    for k, yp in enumerate(args.yp):
        print(f"run Y_P = {yp}", file=sys.stderr, flush=True)
        res = run(args.n, yp, args.T, args.xi, args.equil, args.seed + k,
                  log=lambda s: print(s, file=sys.stderr, flush=True))
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
