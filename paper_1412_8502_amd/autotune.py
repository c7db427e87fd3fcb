"""Autotuner front end: runs the library's pasta_autotune on a state, caches
the choice per workload shape in a JSON file, and applies it with
pasta_set_tuning.

Shape key: precision, N rounded to a power of two, density to 0.01 fm^-3
and proton fraction to 0.05 -- the quantities the pair-kernel costs depend on
(Coulomb work ~ Z^2, nuclear candidates ~ N n).  The cache lives in
$PASTA_TUNING_CACHE, else ~/.cache/pasta_md/tuning.json.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import time

import torch

from . import binding as B


def cache_path() -> str:
    p = os.environ.get("PASTA_TUNING_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "pasta_md", "tuning.json")


def shape_key(n: int, z: int, L: float, precision: int) -> str:
    dens = n / L ** 3
    yp = z / max(n, 1)
    nb = 2 ** int(round(math.log2(max(n, 1))))
    return f"p{precision}_n{nb}_d{round(dens, 2):.2f}_y{round(yp * 20) / 20:.2f}"


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pasta_autotune(pos, species, L: float, precision: int, reps: int = 5, pot=None,
                   stream=None):
    """Times every candidate setting on this state (see include/pasta.h).
    Returns (best dict, [(candidate dict, ms), ...])."""
    B._check_state(pos, species)
    pot = pot or B.pasta_potential_paper()
    n = pos.shape[0]
    nb = ctypes.c_size_t()
    B._check(B.lib.pasta_autotune_workspace(ctypes.byref(pot), precision, n, L,
                                            ctypes.byref(nb)))
    work = B._workspace(nb.value, pos.device)
    best = B.pasta_tuning()
    cap = 64
    ms = (ctypes.c_double * cap)()
    cands = (B.pasta_tuning * cap)()
    ncand = ctypes.c_int32(cap)
    B._check(B.lib.pasta_autotune(ctypes.byref(pot), precision, n, L, B._p(pos), B._p(species),
                                  B._p(work), work.numel(), B._stream(stream), reps,
                                  ctypes.byref(best), ms, cands, ctypes.byref(ncand)))
    keys = ("nuclear_variant", "coulomb_splits", "fused_forces", "coulomb_form", "nuclear_tile")
    table = [({f: getattr(cands[k], f) for f in keys}, ms[k])
             for k in range(min(ncand.value, cap))]
    return {f: getattr(best, f) for f in keys}, table


# the step runoff of the last measured tune() call: [(setting, ms per step)] or None
last_runoff = None


def step_runoff(pos, species, L: float, precision: int, finalists, seconds: float = 0.25,
                est_ms: float = 1.0):
    """Times each finalist setting on simulation steps of this state (zero
    starting velocities, no thermostat): the per-step cell rebuild and the
    combine's drift and binning are part of the step, and they are not in
    the force-only timings of pasta_autotune.  Two alternating passes of
    about `seconds` each per finalist; each keeps its faster pass.  Leaves
    the process-wide setting unchanged.  Returns [(setting, ms per step)]."""
    steps = max(10, min(400, int(seconds / max(est_ms, 1e-3) * 1e3)))
    best = [float("inf")] * len(finalists)
    old = B.pasta_get_tuning()
    try:
        for _ in range(2):
            for i, cand in enumerate(finalists):
                B.pasta_set_tuning(**cand)
                sim = B.Sim(pos.clone(), torch.zeros_like(pos), species, L, dt=2.0,
                            precision=precision)
                sim.step(5)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sim.step(steps)
                torch.cuda.synchronize()
                best[i] = min(best[i], (time.perf_counter() - t0) / steps * 1e3)
                sim.close()
    finally:
        B.pasta_set_tuning(**old)
    return list(zip(finalists, best))


def tune(pos, species, L: float, precision: int, use_cache: bool = True, apply: bool = True,
         margin: float = 0.03, max_finalists: int = 4):
    """Cached autotune for this workload shape; applies the result
    process-wide when `apply`.  The force-only timings of pasta_autotune
    rank the candidates; those within `margin` of the fastest (at most
    `max_finalists`) are then timed on simulation steps (step_runoff), and
    the fastest step wins.  Returns (setting, source, table)."""
    n = pos.shape[0]
    z = int((species == 1).sum().item())
    key = shape_key(n, z, L, precision)
    path = cache_path()
    data = _load_cache(path) if use_cache else {}
    table = None
    if key in data:
        best, source = data[key]["best"], "cache"
    else:
        best, table = pasta_autotune(pos, species, L, precision)
        fast = min(ms for _, ms in table)
        finalists = []
        for cand, ms in sorted(table, key=lambda r: r[1]):
            if ms <= fast * (1.0 + margin) and cand not in finalists:
                finalists.append(cand)
        finalists = finalists[:max_finalists]
        runoff = None
        if len(finalists) > 1 and n > 0:
            runoff = step_runoff(pos, species, L, precision, finalists, est_ms=fast)
            best = min(runoff, key=lambda r: r[1])[0]
        global last_runoff
        last_runoff = runoff
        source = "measured"
        if use_cache:
            data[key] = {"best": best, "table": table, "runoff": runoff}
            _store_cache(path, data)
    if apply:
        B.pasta_set_tuning(**best)
    return best, source, table


def tune_list_skin(pos, vel, species, L: float, precision: int, T: float, skins=(1.0, 1.5, 2.0, 3.0),
                   warmup: int = 50, steps: int = 200, dt: float = 2.0, rescale_every: int = 100):
    """Chooses the halo of the neighbour-list form by running the simulation:
    the list form's cost is (force on the lists) + (build) / (steps between
    builds), and the rebuild interval depends on the dynamics, so each
    candidate halo advances a copy of the state `warmup` + `steps` steps and
    the steps are timed.  Leaves the process-wide setting unchanged.
    Returns (best halo, [(halo, ms per step, builds during the timed steps)])."""
    table = []
    old = B.pasta_get_tuning()
    try:
        for skin in skins:
            B.pasta_set_tuning(nuclear_variant=2, list_skin=float(skin))
            p, v = pos.clone(), vel.clone()
            sim = B.Sim(p, v, species, L, dt=dt, T=T, rescale_every=rescale_every,
                        precision=precision)
            sim.step(warmup)
            b0 = sim.list_stats()["builds"]
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sim.step(steps)
            e1.record()
            e1.synchronize()
            table.append((float(skin), e0.elapsed_time(e1) / steps,
                          sim.list_stats()["builds"] - b0))
            sim.close()
    finally:
        B.pasta_set_tuning(**old)
    best = min(table, key=lambda r: r[1])[0]
    return best, table


def tune_batch(pos, vel, species, ns, L0s, integs, precision: int, mode: int = 0,
               variants=(1, 3), coulomb_forms=None, wgs_per_cu=(3, 4, 5), steps: int = 60,
               warmup: int = 10, steps_per_graph: int = 10):
    """Chooses the batched path's kernel setting on its own workload by timed
    runs: the nuclear variant, the Coulomb form (gather tiles, pairwise
    super-block items with partials, and in mixed precision pairwise items
    into fixed-point accumulators) and, for the persistent mode, the
    workgroups per CU of the persistent kernel.  Each candidate advances a
    copy of the systems `warmup` + `steps` steps.  Leaves the process-wide
    setting unchanged.  Returns (best dict, [(candidate dict, ms per step)])."""
    if coulomb_forms is None:
        coulomb_forms = (0, 1, 2) if precision == B.PASTA_MIXED else (0, 1)
    table = []
    old = B.pasta_get_tuning()
    grids = wgs_per_cu if mode == 0 else (0,)
    try:
        for v in variants:
            for cf in coulomb_forms:
                for w in grids:
                    B.pasta_set_tuning(nuclear_variant=v, coulomb_form=cf, batch_wgs_per_cu=w)
                    p, q = pos.clone(), vel.clone()
                    b = B.Batch(p, q, species, ns, L0s, integs, precision=precision, mode=mode,
                                steps_per_graph=steps_per_graph)
                    b.step(warmup)
                    torch.cuda.synchronize()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    b.step(steps)
                    e1.record()
                    e1.synchronize()
                    table.append(({"nuclear_variant": v, "coulomb_form": cf,
                                   "batch_wgs_per_cu": w}, e0.elapsed_time(e1) / steps))
                    b.close()
    finally:
        B.pasta_set_tuning(**old)
    best = min(table, key=lambda r: r[1])[0]
    return best, table
