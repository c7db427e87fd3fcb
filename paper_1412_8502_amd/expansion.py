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

prints one JSON line per run.  A long run can be cut into segments: with
--checkpoint PATH and --max-seconds S (or --max-steps K) it stops at the
first report boundary past the limit, writes positions, velocities and the
phase and step reached to PATH (.npz), and prints a line with "status":
"checkpointed"; --resume PATH continues it.  The resumed simulation takes
the saved state at its global step (the box law and the thermostat cadence
are functions of that step), so a resumed run in the same process takes the
same steps as an uncut one.
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


_PARAM_NAMES = ("n", "yp", "T", "xi_log10", "equil_steps", "seed", "n0", "n_end", "dt")


def save_checkpoint(path, params: dict, phase: int, done: int, seconds: float, segments: int,
                    pos: np.ndarray, vel: np.ndarray) -> None:
    """Writes a run's state (phase 0 = equilibration, 1 = expansion; done =
    steps taken in that phase) as plain arrays (no pickled objects)."""
    np.savez(path, params=np.array([float(params[k]) for k in _PARAM_NAMES]),
             phase=np.int64(phase), done=np.int64(done), seconds=np.float64(seconds),
             segments=np.int64(segments), pos=np.asarray(pos, np.float64),
             vel=np.asarray(vel, np.float64))


def load_checkpoint(path, params: dict) -> dict:
    """Reads a checkpoint and checks that it belongs to a run with these
    parameters; raises ValueError otherwise."""
    with np.load(path) as f:
        ck = {k: f[k] for k in f.files}
    want = np.array([float(params[k]) for k in _PARAM_NAMES])
    if ck["params"].shape != want.shape or not np.array_equal(ck["params"], want):
        got = dict(zip(_PARAM_NAMES, ck["params"].tolist()))
        raise ValueError(f"checkpoint {path} is of another run: {got}")
    n = int(params["n"])
    if ck["pos"].shape != (n, 3) or ck["vel"].shape != (n, 3) or int(ck["phase"]) not in (0, 1):
        raise ValueError(f"checkpoint {path}: bad state arrays or phase")
    return {"phase": int(ck["phase"]), "done": int(ck["done"]), "seconds": float(ck["seconds"]),
            "segments": int(ck["segments"]), "pos": ck["pos"], "vel": ck["vel"]}


def run(n: int, yp: float, T: float, xi_log10: float, equil_steps: int, seed: int,
        n0: float = 0.08, n_end: float = 0.01, dt: float = 2.0, report_every: int = 50000,
        log=print, return_state: bool = False, checkpoint=None, resume=None,
        max_seconds: float | None = None, max_steps: int | None = None):
    """One run (or one segment of it); returns the result dict (and, with
    return_state, also the final positions [n][3] and box side as numpy /
    float).  A segment that stops at max_seconds / max_steps (checked at each
    report boundary) writes `checkpoint` and returns {"status":
    "checkpointed", ...} with no statistics; `resume` continues from such a
    file."""
    import torch
    from . import binding as B
    from .inputs import make_state

    params = {"n": n, "yp": yp, "T": T, "xi_log10": xi_log10, "equil_steps": equil_steps,
              "seed": seed, "n0": n0, "n_end": n_end, "dt": dt}
    if (max_seconds is not None or max_steps is not None) and checkpoint is None:
        raise ValueError("a segment limit needs a checkpoint path")
    st = make_state(n, yp, n0, T, seed)
    phase, done, secs0, segments = 0, 0, 0.0, 1
    if resume is not None:
        ck = load_checkpoint(resume, params)
        st["pos"], st["vel"] = ck["pos"], ck["vel"]
        phase, done, secs0, segments = ck["phase"], ck["done"], ck["seconds"], ck["segments"] + 1
        log(f"  resumed {resume}: phase {phase}, step {done}, segment {segments}")
    dev = torch.device("cuda:0")
    pos = torch.tensor(st["pos"], device=dev)
    vel = torch.tensor(st["vel"], device=dev)
    sp = torch.tensor(st["species"], device=dev)
    L0 = st["L"]
    xi = 10.0 ** xi_log10
    stretch = (n0 / n_end) ** (1.0 / 3.0)
    steps = int(round((stretch - 1.0) / xi / dt))
    t0 = time.perf_counter()
    seg_steps = 0

    def start(xi_dot, L_max, at):
        # the state at global step `at`: the box law and the thermostat
        # cadence continue as in an uncut run
        return B.Sim(pos, vel, sp, L0, dt=dt, xi_dot=xi_dot, T=T, rescale_every=100,
                     precision=B.PASTA_MIXED, step0=at, L_max=L_max)

    def advance(sim, total, label):
        nonlocal done, seg_steps
        while done < total:
            if ((max_seconds is not None and time.perf_counter() - t0 >= max_seconds) or
                    (max_steps is not None and seg_steps >= max_steps)):
                return False
            k = min(report_every, total - done)
            sim.step(k)
            done += k
            seg_steps += k
            en = sim.energies()
            log(f"  {label} {done}/{total} steps: n = {n / en['L'] ** 3:.5f} fm^-3, E_pot/N = "
                f"{en['epot'] / n:.4f} MeV ({time.perf_counter() - t0:.0f} s)")
        return True

    def stop():
        save_checkpoint(checkpoint, params, phase, done, secs0 + time.perf_counter() - t0,
                        segments, pos.cpu().numpy(), vel.cpu().numpy())
        return {"status": "checkpointed", "checkpoint": str(checkpoint), "phase": phase,
                "done": done, "segments": segments, **params}

    if phase == 0:
        # equilibration in the fixed box
        sim = start(0.0, None, done)
        finished = advance(sim, equil_steps, "equilibration")
        del sim
        if not finished:
            return stop()
        phase, done = 1, 0
    # expansion: a new box law from the equilibrated state (step 0 = start)
    sim = start(xi, L0 * stretch * (1.0 + 1e-9), done)
    finished = advance(sim, steps, "expansion")
    L_end = sim.energies()["L"]
    del sim
    if not finished:
        return stop()
    cl = B.pasta_cluster(pos, sp, L_end)
    stats = cluster_stats(cl["label"].cpu().numpy(), st["species"])
    res = {"status": "done", "N": n, "Y_P": yp, "T_MeV": T, "log10_xi_dot": xi_log10,
           "dt_fm_c": dt, "equilibration_steps": equil_steps, "expansion_steps": steps,
           "n_final": n / L_end ** 3, "seed": seed,
           "seconds": secs0 + time.perf_counter() - t0, "segments": segments, **stats}
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
    ap.add_argument("--checkpoint", help="where a stopped segment writes its state (.npz)")
    ap.add_argument("--resume", help="checkpoint to continue from")
    ap.add_argument("--max-seconds", type=float, help="stop this segment after about S s")
    ap.add_argument("--max-steps", type=int, help="stop this segment after about K steps")
    args = ap.parse_args(argv)
    seg = (args.checkpoint, args.resume, args.max_seconds, args.max_steps)
    if any(a is not None for a in seg) and len(args.yp) > 1:
        ap.error("checkpointed runs take one --yp")
    for k, yp in enumerate(args.yp):
        print(f"run Y_P = {yp}", file=sys.stderr, flush=True)
        res = run(args.n, yp, args.T, args.xi, args.equil, args.seed + k,
                  log=lambda s: print(s, file=sys.stderr, flush=True),
                  checkpoint=args.checkpoint, resume=args.resume,
                  max_seconds=args.max_seconds, max_steps=args.max_steps)
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
