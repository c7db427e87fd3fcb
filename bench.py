"""Throughput benchmark of the MD hot path on one MI355X.

Workload: N = 51 200 nucleons, Y_P = 0.20, n = 0.080 fm^-3 (L = 86.18 fm),
T = 0.75 MeV, random-uniform start, velocity Verlet at dt = 2 fm/c with the
velocity rescale every 100 steps (the paper's protocol), box fixed.  A step is
the whole hot path: first half kick + drift + cell binning, scan, stable
scatter + staging, the all-pairs screened-Coulomb kernel, the nuclear
cell-tile kernel with the fused second half kick, and the thermostat on every
100th step.  The mixed-precision path is the headline; the FP64 path is timed
beside it.

Prints one JSON line: pair interactions per second (useful pairs: unordered
nuclear pairs inside 11.5 fm plus all unordered proton pairs of the uncut
Coulomb term), MD steps per second, the roofline entry of the dominant
kernel and the CPU oracle baseline.  Beside the headline: the FP64 path and
its roofline, the neighbour-list and dense-kernel forms, N = 409 600 at
Y_P = 0.40 and 0.05 in both precisions, the 20 000-step decompression
window (0.080 -> 0.00125 fm^-3), and the batched 15-system grid.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "n51200_yp020_n0.080"
LARGE_WORKLOADS = ("n409600_yp040_n0.080", "n409600_yp005_n0.080")
DECOMPRESSION_WORKLOAD = "n51200_yp030_n0.080"
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector (packed FMA), published
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # the same without packed FP32 (256 CU x 2.4 GHz x 128)
PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector, published
# Algorithmic work per ordered pair inside the cutoff (what the method must
# compute, whichever kernel form computes it; FMA = 2 flops, transcendentals
# counted apart as T):
#   nuclear: difference 3, r^2 5, scale 1, g^2 1, V 3, force scalar 3,
#            force 6, energy 1 -> 23 flops + 1 T (one exp)
#   Coulomb: difference 3, nearest image 6, r^2 5, r 1, 1/r 1, V 2, force
#            scalar 3, force 6, energy 1 -> 28 flops + 2 T (rsqrt, exp)
FLOPS_NUC_PAIR, T_NUC_PAIR = 23, 1
FLOPS_COUL_PAIR, T_COUL_PAIR = 28, 2


def pair_work(nuc_pairs, coul_pairs):
    """(flops, transcendentals) of one force evaluation, from the unordered
    pair counts (each unordered pair is two ordered ones)."""
    return (2 * nuc_pairs * FLOPS_NUC_PAIR + 2 * coul_pairs * FLOPS_COUL_PAIR,
            2 * nuc_pairs * T_NUC_PAIR + 2 * coul_pairs * T_COUL_PAIR)


def roofline_entry(kernel, nuc_pairs, coul_pairs, avg_ms, precision):
    """Roofline of the pair-force launch: algorithmic flops per launch over
    its average duration (HIP events on the simulation's stream)."""
    flops, tops = pair_work(nuc_pairs, coul_pairs)
    ach = flops / (avg_ms * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if precision == 0 else PEAK_FP32_TFLOPS
    out = {"kernel": kernel, "bound": "alu", "achieved": round(ach, 3), "peak": peak,
           "unit": "TFLOP/s", "frac": round(ach / peak, 4),
           "flops_per_launch": flops, "transcendentals_per_launch": tops,
           "transcendentals_per_s": round(tops / (avg_ms * 1e-3), 1),
           "avg_launch_ms": round(avg_ms, 5)}
    if precision != 0:
        out["frac_vs_nonpacked_fp32"] = round(ach / PEAK_FP32_NONPACKED_TFLOPS, 4)
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel_name, tuning):
    """HBM bytes per launch of the pair-force kernel from the counter runs
    recorded under profiles/ (FETCH_SIZE and WRITE_SIZE, each scaled by what
    the counter reads for a copy of known size), or None when the kernel
    sources differ from the ones the counters were taken on or no record
    matches this kernel and setting."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_pair_forces_n51200.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for src in rec.get("sources", []):
        try:
            with open(os.path.join(ROOT, src), "rb") as f:
                data = f.read()
        except OSError:
            return None
        h.update(src.encode())
        h.update(data)
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    want = [tuning.get("nuclear_variant"), tuning.get("coulomb_splits"), tuning.get("fused_forces"),
            tuning.get("coulomb_form", 0)]
    for e in rec.get("entries", []):
        if e.get("kernel") == kernel_name and e.get("tuning") == want:
            return e["bytes_per_launch"]
    return None


def host_environment():
    """ROCm version and the GPU clocks (rocm-smi, if it answers within a few
    seconds), read before this process touches the GPU."""
    import subprocess
    env = {}
    try:
        with open("/opt/rocm/.info/version") as f:
            env["rocm"] = f.read().strip()
    except OSError:
        env["rocm"] = None
    try:
        out = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True,
                             timeout=10).stdout
        env["clocks"] = [l.strip() for l in out.splitlines() if "sclk" in l or "mclk" in l][:4]
    except (OSError, subprocess.SubprocessError):
        env["clocks"] = None
    return env


def device_environment(torch):
    p = torch.cuda.get_device_properties(0)
    return {"device": p.name, "arch": getattr(p, "gcnArchName", None),
            "compute_units": p.multi_processor_count, "hip": torch.version.hip,
            "torch": torch.__version__}


def memory_kernels(per_kernel, n):
    """Achieved algorithmic GB/s of the memory-side kernels of a step against
    the 8 TB/s HBM peak.  Bytes per particle: integrate (the combine with the
    second half kick, the next step's half kick, drift and binning) reads the
    raw nuclear (F, V) 32 B, positions and velocities 48 B and species 1 B,
    writes positions and velocities 48 B, F 24 B and the bin key 4 B: 157 B
    (the Coulomb partials it also sums are left out); build (scatter and
    rank; the scan is per cell) reads the key twice and the slot array once
    (12 B), writes the slot array, the permutation and the staging entry
    (24 B) and moves positions and velocities (96 B): 132 B."""
    out = {}
    for name, keys, per in (("integrate", ("combine+kick",), 157),
                            ("build", ("scan", "scatter", "rank+stage"), 132)):
        ms = sum(per_kernel.get(k, {}).get("ms_per_step", 0.0) for k in keys)
        if ms > 0:
            gbs = per * n / (ms * 1e-3) * 1e-9
            out[name] = {"kernels": list(keys), "ms_per_step": round(ms, 5),
                         "algorithmic_bytes": per * n, "GB_per_s": round(gbs, 1),
                         "frac_of_8TBps": round(gbs / 8000.0, 4)}
    return out


def stencil_candidates(pos, L, r_nuc=11.5, min_occ=32):
    """Ordered candidate pairs that the 27-cell stencil presents to the
    nuclear kernels at these positions (self pairs excluded), on the force
    path's grid: cells of side at least r_nuc, at most k per side with
    k^3 * min_occ <= N.  The kernels cull this further (the staging keeps
    the sources within r_nuc of a work item's bounding box); the ratio to
    the useful ordered pairs measures the stencil's waste."""
    import numpy as np
    n = len(pos)
    nc = int(np.floor(L / r_nuc))
    while nc > 1 and L / nc < r_nuc:
        nc -= 1
    nc = max(nc, 1)
    k = 1
    while (k + 1) ** 3 * min_occ <= n:
        k += 1
    nc = min(nc, k)
    c = np.clip(np.floor(np.asarray(pos) * (nc / L)).astype(np.int64), 0, nc - 1)
    counts = np.bincount((c[:, 0] * nc + c[:, 1]) * nc + c[:, 2],
                         minlength=nc ** 3).reshape(nc, nc, nc).astype(np.float64)
    offs = (-1, 0, 1) if nc >= 3 else ((0, 1) if nc == 2 else (0,))
    neigh = np.zeros_like(counts)
    for dx in offs:
        for dy in offs:
            for dz in offs:
                neigh += np.roll(counts, (dx, dy, dz), axis=(0, 1, 2))
    return float((counts * neigh).sum() - n), nc


def run_path(B, torch, st, precision, steps, warmup, timing, pot=None, windows=0):
    dev = torch.device("cuda:0")
    pos = torch.tensor(st["pos"], device=dev)
    vel = torch.tensor(st["vel"], device=dev)
    sp = torch.tensor(st["species"], device=dev)
    sim = B.Sim(pos, vel, sp, st["L"], dt=2.0, T=st["T"], rescale_every=100,
                precision=precision, pot=pot)
    sim.step(warmup)
    torch.cuda.synchronize()
    nuc0, coul = sim.pair_counts()
    # timed region 1: the step loop alone
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t0
    nuc1, _ = sim.pair_counts()
    # further timed windows of the step loop (their median beside the main window)
    win = []
    for _ in range(windows):
        kw = max(50, steps // 5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(kw)
        torch.cuda.synchronize()
        win.append((time.perf_counter() - t0) / kw * 1e3)
    kt = None
    dt_timed = None
    if timing:
        # timed region 2: the same number of steps with HIP events around
        # every launch (per-kernel durations for the roofline)
        sim.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dt_timed = time.perf_counter() - t0
        kt = sim.kernel_times()
        sim.set_timing(False)
    en = sim.energies()
    ls = sim.list_stats()
    sim.close()
    stencil, ncell = stencil_candidates(pos.cpu().numpy(), st["L"])
    return dict(seconds=dt_plain, seconds_with_events=dt_timed, nuc_pairs=(nuc0 + nuc1) / 2,
                coul_pairs=coul, kernel_times=kt, energies=en, list_stats=ls,
                stencil_candidates=stencil, ncell=ncell, windows_ms=win,
                steps=steps + (steps if timing else 0) + warmup)


def run_batch(B, torch, states, precision, mode, steps, warmup, spg=10, tune=False):
    """The 15-system grid advanced together (one persistent launch per step
    for mode 0, one launch per phase for mode 1), from a captured hipGraph.
    tune: choose the kernel setting on this workload first (timed runs)."""
    import numpy as np
    dev = torch.device("cuda:0")
    pos = torch.tensor(np.concatenate([s["pos"] for s in states]), device=dev)
    vel = torch.tensor(np.concatenate([s["vel"] for s in states]), device=dev)
    sp = torch.tensor(np.concatenate([s["species"] for s in states]), device=dev)
    ns, L0s = [s["n"] for s in states], [s["L"] for s in states]
    integs = [dict(dt=2.0, T=s["T"], rescale_every=100) for s in states]
    saved = B.pasta_get_tuning()
    best, table = None, None
    if tune:
        from paper_1412_8502_amd.autotune import tune_batch
        best, table = tune_batch(pos, vel, sp, ns, L0s, integs, precision, mode=mode)
        B.pasta_set_tuning(**best)
    b = B.Batch(pos, vel, sp, ns, L0s, integs, precision=precision, mode=mode,
                steps_per_graph=spg)
    B.pasta_set_tuning(**saved)
    b.step(warmup)
    torch.cuda.synchronize()
    nn, nc = b.pair_counts()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info = b.info()
    b.close()
    return dict(seconds=dt, pairs_per_step=float(sum(nn) + sum(nc)), grid=info["grid"],
                tuning=best, tuning_table=[[c, round(ms, 5)] for c, ms in table] if table else None)


def batch_overhead_section(B, torch, steps=200, warmup=20):
    """Per-step time of the batched path, per-phase launches against the
    persistent kernel at 1, 3 and 5 workgroups per CU, from a system whose
    pair work is negligible up to the headline size: the persistent form's
    extra cost per step grows with its workgroup count (each workgroup
    orders its arrivals at every device-wide barrier with agent-scope
    fences), not with the work."""
    import numpy as np
    from paper_1412_8502_amd.inputs import make_state
    dev = torch.device("cuda:0")
    cases = (("1 x 2000", [(2000, 0.2, 0.08, 1.0, 1)]),
             ("1 x 6400", [(6400, 0.2, 0.08, 1.0, 1)]),
             ("8 x 6400", [(6400, 0.2, 0.08, 1.0, k) for k in range(8)]),
             ("1 x 51200", [(51200, 0.2, 0.08, 0.75, 1)]))
    saved = B.pasta_get_tuning()
    out = {"setting": "nuclear variant 3, pairwise Coulomb items, mixed, n = 0.08 fm^-3, "
                      "graphs of 10 steps, rescale every 100"}
    try:
        for name, specs in cases:
            sts = [make_state(*c) for c in specs]
            r = {}
            for mode, wpc in ((1, 0), (0, 1), (0, 3), (0, 5)):
                B.pasta_set_tuning(nuclear_variant=3, coulomb_form=1, batch_wgs_per_cu=wpc)
                pos = torch.tensor(np.concatenate([s["pos"] for s in sts]), device=dev)
                vel = torch.tensor(np.concatenate([s["vel"] for s in sts]), device=dev)
                sp = torch.tensor(np.concatenate([s["species"] for s in sts]), device=dev)
                b = B.Batch(pos, vel, sp, [s["n"] for s in sts], [s["L"] for s in sts],
                            [dict(dt=2.0, T=s["T"], rescale_every=100) for s in sts],
                            mode=mode, steps_per_graph=10)
                b.step(warmup)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                b.step(steps)
                torch.cuda.synchronize()
                us = (time.perf_counter() - t0) / steps * 1e6
                grid = b.info()["grid"]
                b.close()
                key = "per_phase" if mode == 1 else f"persistent_{wpc}_per_cu"
                r[key] = {"us_per_step": round(us, 1), "grid": grid}
            out[name] = r
            print(name, r, file=sys.stderr, flush=True)
    finally:
        B.pasta_set_tuning(**saved)
    return out


def build_section(B, torch, sizes=(4 << 20, 8 << 20, 16 << 20), reps=5):
    """The standalone cell-list build (pasta_cell_list: bin count, scan,
    scatter, stable rank; cells of side >= r_nuc, one bin per cell and
    species) on uniformly random states of 4-16 M particles at 0.08 fm^-3,
    first in random order, then with the particles already in cell order
    (the simulation's steady state, where a wavefront's lanes share bins and
    its atomic increments aggregate).
    Algorithmic bytes per particle: positions and species read (25 B), the
    bin key written and read twice (12 B), the scatter's slot array written
    and read (8 B), the permutation written (4 B): 49 B.  The rank pass
    also reads every member of the particle's bin (about 75 at this
    density), which the algorithmic count leaves out."""
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    out = {"algorithmic_bytes_per_particle": 49, "density_fm3": 0.08, "r_cut_fm": 11.5}
    for n in sizes:
        L = (n / 0.08) ** (1.0 / 3.0)
        pos = torch.rand((n, 3), generator=gen, device=dev, dtype=torch.float64) * L
        pos = torch.clamp(pos, 0.0, L * (1.0 - 1e-15))
        sp = (torch.rand(n, generator=gen, device=dev) < 0.3).to(torch.uint8)
        B.pasta_cell_list(pos, sp, L, 11.5)
        r = {"L_fm": round(L, 2)}
        for order in ("random", "cell_sorted"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                nc, start, perm = B.pasta_cell_list(pos, sp, L, 11.5)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
            r["cells_per_side"] = nc
            r[order] = {"ms_per_build": round(ms, 3), "particles_per_s": n / ms * 1e3,
                        "algorithmic_GB_per_s": round(49 * n / ms * 1e-6, 1)}
            if order == "random":  # the same particles in cell order
                idx = perm.long()
                pos, sp = pos[idx].contiguous(), sp[idx].contiguous()
                B.pasta_cell_list(pos, sp, L, 11.5)
        out[f"n{n}"] = r
        print(n, r, file=sys.stderr, flush=True)
        del pos, sp, start, perm
    return out


def single_via_batch(B, torch, st, steps, warmup):
    """One system through the batched path in both modes, each tuned on it."""
    vb = run_batch(B, torch, [st], B.PASTA_MIXED, 1, steps, warmup, tune=True)
    vb0 = run_batch(B, torch, [st], B.PASTA_MIXED, 0, steps, warmup, tune=True)
    out = {"multi_kernel_ms_per_step": vb["seconds"] / steps * 1e3,
           "multi_kernel_tuning": vb["tuning"],
           "persistent_ms_per_step": vb0["seconds"] / steps * 1e3,
           "persistent_tuning": vb0["tuning"]}
    log(f"single system via batch: {out}")
    return out


def run_sequential(B, torch, states, precision, steps, warmup):
    """The same systems one after another on the single-system path, each
    with the kernel setting the autotuner picks on its own start state (the
    tuning is outside the timed steps; the process-wide setting is restored
    afterwards)."""
    from paper_1412_8502_amd.autotune import tune
    dev = torch.device("cuda:0")
    total, pairs, settings = 0.0, 0.0, []
    old = B.pasta_get_tuning()
    try:
        for st in states:
            pos = torch.tensor(st["pos"], device=dev)
            vel = torch.tensor(st["vel"], device=dev)
            sp = torch.tensor(st["species"], device=dev)
            best, _, _ = tune(pos, sp, st["L"], precision, use_cache=False)
            settings.append([best["nuclear_variant"], best["fused_forces"], best["coulomb_form"]])
            sim = B.Sim(pos, vel, sp, st["L"], dt=2.0, T=st["T"], rescale_every=100,
                        precision=precision)
            sim.step(warmup)
            torch.cuda.synchronize()
            nn, nc = sim.pair_counts()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(steps)
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
            pairs += nn + nc
            sim.close()
    finally:
        B.pasta_set_tuning(**old)
    return dict(seconds=total, pairs_per_step=pairs, settings=settings)


def kernel_ms(kt, steps):
    return {k: round(v[0] / max(steps, 1), 5) for k, v in kt.items() if v[1]}


def kernel_variant(tuning):
    """The fused kernel's variant template argument for a tuning: variant 3
    with a 256- or 1024-source tile runs as 5 or 6."""
    v, tile = tuning.get("nuclear_variant"), tuning.get("nuclear_tile", 0)
    if v == 3 and tile in (256, 1024):
        return 5 if tile == 256 else 6
    return v


# public coulomb_form -> the fused kernel's Coulomb template argument, and a name
FUSED_COULOMB_ARG = {0: 0, 1: 1, 2: 3}
COULOMB_FORM_NAMES = {0: "gather", 1: "pairwise", 2: "pairwise fixed-point"}


def pair_kernel_name(tuning, use_lists=False):
    if tuning.get("fused_forces") or kernel_variant(tuning) >= 4:
        tile = tuning.get("nuclear_tile", 0)
        return "pair forces (nuclear %s%s + %s Coulomb tiles, one launch)" % (
            "list items" if use_lists else "cell tiles",
            " of %d sources" % tile if tile else "",
            COULOMB_FORM_NAMES[tuning.get("coulomb_form", 0)])
    return "nuclear+kick"


def large_section(B, torch, steps=20, warmup=5):
    """N = 409 600 at Y_P = 0.40 and 0.05 (the paper's large runs,
    Sec. II.B.2), each precision autotuned on its own state: steps/s, pair
    interactions/s, per-kernel times and the pair kernel's roofline."""
    from paper_1412_8502_amd.autotune import tune
    from paper_1412_8502_amd.inputs import workload
    dev = torch.device("cuda:0")
    out = {"steps": steps, "warmup": warmup}
    saved = B.pasta_get_tuning()
    for name in LARGE_WORKLOADS:
        st = workload(name)
        ent = {"N": st["n"], "Z": st["Z"], "L_fm": st["L"], "Y_P": st["y_p"],
               "density": st["density"], "T_MeV": st["T"]}
        tpos = torch.tensor(st["pos"], device=dev)
        tsp = torch.tensor(st["species"], device=dev)
        for prec, label in ((B.PASTA_MIXED, "mixed"), (B.PASTA_FP64, "fp64")):
            best, _, _ = tune(tpos, tsp, st["L"], prec, use_cache=False, apply=True)
            r = run_path(B, torch, st, prec, steps, warmup, timing=True)
            kt = r["kernel_times"]
            ms_f, nl = kt["nuclear+kick"]
            useful = r["nuc_pairs"] + r["coul_pairs"]
            ent[label] = {
                "ms_per_step": r["seconds"] / steps * 1e3,
                "md_steps_per_s": steps / r["seconds"],
                "pair_interactions_per_s": useful * steps / r["seconds"],
                "useful_pairs_per_step": {"nuclear": r["nuc_pairs"], "coulomb": r["coul_pairs"]},
                "tuning": best,
                "per_kernel_ms": kernel_ms(kt, steps),
                "roofline": roofline_entry(pair_kernel_name(best), r["nuc_pairs"],
                                           r["coul_pairs"], ms_f / max(nl, 1), prec)}
            log(f"large {name} {label}: {ent[label]['ms_per_step']:.3f} ms/step, "
                f"tuning {best}")
        ent["mixed_over_fp64_speedup"] = ent["fp64"]["ms_per_step"] / ent["mixed"]["ms_per_step"]
        out[name] = ent
        del tpos, tsp
    B.pasta_set_tuning(**saved)
    return out


def decompression_section(B, torch, nsteps=20000, segment=2000):
    """The decompression window: N = 51 200, Y_P = 0.30, T = 0.5 MeV, box
    grown by Eq. (3a) from 0.080 to 0.00125 fm^-3 (L 86.18 -> 344.7 fm) over
    20 000 steps of 2 fm/c (xi_dot = 7.5e-5 c/fm), velocity rescale every 100
    steps, mixed precision, kernel setting tuned on the starting state.
    Steps/s over the whole window and per segment of 2000 steps (the cell
    grid goes from 7 to 29 cells per side as the box grows)."""
    from paper_1412_8502_amd.autotune import tune
    from paper_1412_8502_amd.inputs import workload
    dev = torch.device("cuda:0")
    st = workload(DECOMPRESSION_WORKLOAD)
    L0, xi, dt = st["L"], 7.5e-5, 2.0
    saved = B.pasta_get_tuning()
    pos = torch.tensor(st["pos"], device=dev)
    vel = torch.tensor(st["vel"], device=dev)
    sp = torch.tensor(st["species"], device=dev)
    best, _, _ = tune(pos, sp, L0, B.PASTA_MIXED, use_cache=False, apply=True)
    sim = B.Sim(pos, vel, sp, L0, dt=dt, xi_dot=xi, T=st["T"], rescale_every=100,
                precision=B.PASTA_MIXED, L_max=4.0 * L0 * (1 + 1e-12))
    segs = []
    total = 0.0
    done = 0
    torch.cuda.synchronize()
    while done < nsteps:
        k = min(segment, nsteps - done)
        t0 = time.perf_counter()
        sim.step(k)
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
        total += dt_s
        done += k
        L = L0 * (1.0 + xi * done * dt)
        segs.append([done, round(st["n"] / L ** 3, 6), round(dt_s / k * 1e3, 5)])
    en = sim.energies()
    sim.close()
    B.pasta_set_tuning(**saved)
    log(f"decompression: {nsteps} steps in {total:.2f} s")
    return {"workload": "N=51200 Y_P=0.30 T=0.5 MeV, n 0.080 -> 0.00125 fm^-3 "
                        "(L 86.18 -> 344.7 fm) over 20000 steps, xi_dot=7.5e-5 c/fm, dt=2 fm/c, "
                        "rescale every 100 steps, mixed",
            "steps": nsteps, "seconds": total, "md_steps_per_s": nsteps / total,
            "ms_per_step": total / nsteps * 1e3, "tuning": best, "final_L_fm": en["L"],
            "segments": "[last step, density fm^-3, ms per step over the segment]",
            "per_segment": segs}


def batched_section(B, torch, steps, warmup):
    from paper_1412_8502_amd.inputs import batch_grid
    states = batch_grid()
    nsys = len(states)
    out = {"systems": nsys, "N_total": int(sum(s["n"] for s in states)),
           "N_per_system": [s["n"] for s in states],
           "density_per_system": [round(s["density"], 5) for s in states],
           "steps": steps,
           "workload": "15 systems: Y_P in {0.05,0.10,0.20,0.30,0.40} x T in {0.5,0.75,1.0} MeV, "
                       "N from {6400,12800,25600,51200} and n in [0.02,0.08] fm^-3 by seed 2000, "
                       "dt=2 fm/c, rescale every 100 steps"}

    def entry(r):
        return {"ms_per_step": r["seconds"] / steps * 1e3,
                "system_steps_per_s": nsys * steps / r["seconds"],
                "pair_interactions_per_s": r["pairs_per_step"] * steps / r["seconds"]}
    pers = run_batch(B, torch, states, B.PASTA_MIXED, 0, steps, warmup, tune=True)
    log(f"batched persistent: {pers['seconds'] / steps * 1e3:.4f} ms/step, tuned "
        f"{pers['tuning']} from {pers['tuning_table']}")
    out["persistent_mixed"] = dict(entry(pers), grid=pers["grid"], tuning=pers["tuning"],
                                   tuning_trials_ms=pers["tuning_table"])
    multi = run_batch(B, torch, states, B.PASTA_MIXED, 1, steps, warmup, tune=True)
    log(f"batched multi-kernel: {multi['seconds'] / steps * 1e3:.4f} ms/step, tuned "
        f"{multi['tuning']}")
    out["multi_kernel_mixed"] = dict(entry(multi), tuning=multi["tuning"],
                                     tuning_trials_ms=multi["tuning_table"])
    seqm = run_sequential(B, torch, states, B.PASTA_MIXED, steps, warmup)
    log(f"sequential mixed: {seqm['seconds'] / steps * 1e3:.4f} ms/step")
    out["sequential_mixed"] = dict(entry(seqm), settings=seqm["settings"],
                                   settings_fields="[nuclear_variant, fused_forces, coulomb_form]"
                                                   " per system, autotuned on its start state")
    seq64 = run_sequential(B, torch, states, B.PASTA_FP64, max(50, steps // 5), warmup)
    log(f"sequential fp64: {seq64['seconds'] / max(50, steps // 5) * 1e3:.4f} ms/step")
    k64 = max(50, steps // 5)
    out["sequential_fp64"] = {"ms_per_step": seq64["seconds"] / k64 * 1e3,
                              "system_steps_per_s": nsys * k64 / seq64["seconds"],
                              "pair_interactions_per_s": seq64["pairs_per_step"] * k64 / seq64["seconds"],
                              "steps": k64, "settings": seq64["settings"]}
    best = min(out["persistent_mixed"]["ms_per_step"], out["multi_kernel_mixed"]["ms_per_step"])
    out["speedup_vs_sequential_mixed"] = out["sequential_mixed"]["ms_per_step"] / best
    out["speedup_vs_sequential_fp64"] = out["sequential_fp64"]["ms_per_step"] / best
    return out


def cpu_baseline(st, pairs_per_target_fn, budget_s=15.0):
    """The FP64 oracle (brute force over all sources, OpenMP over targets) on a
    bounded sample of targets of the same state."""
    import numpy as np
    import oracle
    oracle.build()
    threads = int(os.environ.get("ORACLE_THREADS", "0")) or (os.cpu_count() or 1)
    rng = np.random.Generator(np.random.PCG64(5))
    N = st["n"]
    calib = rng.choice(N, 256, replace=False)
    t0 = time.perf_counter()
    oracle.forces(st["pos"], st["species"], st["L"], targets=calib, nthreads=threads)
    tc = time.perf_counter() - t0
    m = int(min(N, max(256, 256 * budget_s / max(tc, 1e-6))))
    sample = rng.choice(N, m, replace=False)
    t0 = time.perf_counter()
    oracle.forces(st["pos"], st["species"], st["L"], targets=sample, nthreads=threads)
    t = time.perf_counter() - t0
    useful = pairs_per_target_fn(sample)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    # the oracle at the other sizes: one force evaluation and 20 steps at
    # N = 3200, one force evaluation at N = 409 600 estimated from 64 targets
    from paper_1412_8502_amd.inputs import workload
    other = {}
    s1 = workload("n3200_yp040_n0.040")
    t0 = time.perf_counter()
    oracle.forces(s1["pos"], s1["species"], s1["L"], nthreads=threads)
    other["force_eval_s_n3200"] = round(time.perf_counter() - t0, 4)
    t0 = time.perf_counter()
    oracle.run(s1["pos"], s1["vel"], s1["species"], s1["L"], 20, dt=2.0, T=s1["T"],
               nthreads=threads)
    other["steps20_s_n3200"] = round(time.perf_counter() - t0, 4)
    s5 = workload("n409600_yp040_n0.080")
    few = rng.choice(s5["n"], 64, replace=False)
    t0 = time.perf_counter()
    oracle.forces(s5["pos"], s5["species"], s5["L"], targets=few, nthreads=threads)
    other["force_eval_s_n409600_estimated"] = round((time.perf_counter() - t0) / 64 * s5["n"], 1)
    other["force_eval_s_n51200_estimated"] = round(t / m * N, 2)
    return dict(value=useful / t, unit="pair interactions/s", cores=threads, kind="oracle",
                sample=f"{m} of {N} targets of the same state, all {N} sources each "
                       f"(FP64 brute force), {t:.1f} s",
                md_steps_per_s_equiv=1.0 / (t / m * N), cpu_model=model,
                nproc=os.cpu_count(), usable_cpus=usable, other_sizes=other)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the N = 409 600 section")
    ap.add_argument("--no-decompression", action="store_true",
                    help="skip the 20 000-step decompression window")
    ap.add_argument("--section", choices=("large", "decompression", "batch", "batch-overhead",
                                          "build"),
                    default=None,
                    help="run only this section and print its JSON (for profiler runs)")
    ap.add_argument("--tuning", default=None,
                    help="variant,splits,fused[,coulomb_form[,nuclear_tile]]: use this kernel "
                         "setting instead of autotuning")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline path (no dense, list, FP64 or batched runs); "
                         "for profiler runs")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this size first (a "
                         "known-size kernel for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition of this path is a design, not a measured mode", file=sys.stderr)
        sys.exit(2)

    host_env = host_environment() if not args.section else None
    import numpy as np
    import torch
    from paper_1412_8502_amd import binding as B
    from paper_1412_8502_amd.inputs import workload

    if args.section == "batch":
        res = batched_section(B, torch, args.batch_steps, min(args.warmup, 20))
        st1 = workload(WORKLOAD)
        res["single_system_via_batch_path"] = single_via_batch(B, torch, st1, args.steps,
                                                               args.warmup)
        print(json.dumps({"section": "batch", "result": res}))
        return
    if args.section == "build":
        print(json.dumps({"section": args.section, "result": build_section(B, torch)}))
        return
    if args.section == "batch-overhead":
        print(json.dumps({"section": args.section, "result": batch_overhead_section(B, torch)}))
        return
    if args.section:
        fn = large_section if args.section == "large" else decompression_section
        print(json.dumps({"section": args.section, "result": fn(B, torch)}))
        return

    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    st = workload(WORKLOAD)
    N, Z = st["n"], st["Z"]
    K, W = args.steps, args.warmup
    log(f"workload {WORKLOAD}: N={N} Z={Z} L={st['L']:.4f} steps={K} warmup={W}")
    # autotune the pair kernels on this workload (not cached: measured here)
    from paper_1412_8502_amd.autotune import tune
    dev = torch.device("cuda:0")
    tpos = torch.tensor(st["pos"], device=dev)
    tsp = torch.tensor(st["species"], device=dev)
    if args.tuning:
        vals = [int(x) for x in args.tuning.split(",")]
        v, sp_, fu = vals[:3]
        cf = vals[3] if len(vals) > 3 else 0
        tile = vals[4] if len(vals) > 4 else 0
        tuned = dict(nuclear_variant=v, coulomb_splits=sp_, fused_forces=fu, coulomb_form=cf,
                     nuclear_tile=tile)
        tuned64, table, table64 = dict(tuned), [], []
        runoff = runoff64 = None
        B.pasta_set_tuning(**tuned)
    else:
        from paper_1412_8502_amd import autotune
        tuned64, _, table64 = tune(tpos, tsp, st["L"], B.PASTA_FP64, use_cache=False,
                                   apply=False)
        runoff64 = autotune.last_runoff
        tuned, _, table = tune(tpos, tsp, st["L"], B.PASTA_MIXED, use_cache=False, apply=True)
        runoff = autotune.last_runoff
    log(f"kernel setting mixed: {tuned}  fp64: {tuned64}")
    del tpos, tsp
    mixed_cells = run_path(B, torch, st, B.PASTA_MIXED, K, W, timing=True, windows=5)
    log(f"mixed, cell sweeps: {mixed_cells['seconds'] / K * 1e3:.4f} ms/step")
    if args.headline_only:
        useful = mixed_cells["nuc_pairs"] + mixed_cells["coul_pairs"]
        kt = mixed_cells["kernel_times"]
        ms_f, nl = kt["nuclear+kick"]
        print(json.dumps({"metric": "headline path only (profiler run)", "steps": K, "warmup": W,
                          "ms_per_step": mixed_cells["seconds"] / K * 1e3,
                          "value": useful * K / mixed_cells["seconds"],
                          "unit": "pair interactions/s", "tuning": tuned,
                          "pair_forces_avg_launch_ms": ms_f / max(nl, 1),
                          "roofline": roofline_entry(pair_kernel_name(tuned), mixed_cells["nuc_pairs"],
                                                     mixed_cells["coul_pairs"], ms_f / max(nl, 1),
                                                     B.PASTA_MIXED),
                          "per_kernel_ms": kernel_ms(kt, K)}))
        return
    # the neighbour-list form: halo chosen by short timed runs, then the same
    # timed protocol; the faster form is the headline
    from paper_1412_8502_amd.autotune import tune_list_skin
    tpos = torch.tensor(st["pos"], device=dev)
    tvel = torch.tensor(st["vel"], device=dev)
    tsp = torch.tensor(st["species"], device=dev)
    skin, skin_table = tune_list_skin(tpos, tvel, tsp, st["L"], B.PASTA_MIXED, st["T"])
    del tpos, tvel, tsp
    log(f"list halo trials (halo, ms/step, builds in 200 steps): {skin_table} -> {skin}")
    old = B.pasta_set_tuning(nuclear_variant=2, list_skin=skin)
    mixed_lists = run_path(B, torch, st, B.PASTA_MIXED, K, W, timing=True, windows=5)
    B.pasta_set_tuning(**old)
    log(f"mixed, neighbour lists: {mixed_lists['seconds'] / K * 1e3:.4f} ms/step, "
        f"{mixed_lists['list_stats']}")
    use_lists = mixed_lists["seconds"] < mixed_cells["seconds"]
    mixed = mixed_lists if use_lists else mixed_cells
    # the dense cell-tile nuclear kernel, for comparison with the default
    # screened + compacted one
    old = B.pasta_set_tuning(nuclear_variant=0, coulomb_splits=0, fused_forces=0)
    dense = run_path(B, torch, st, B.PASTA_MIXED, max(20, K // 5), min(W, 20), timing=True)
    B.pasta_set_tuning(**old)
    kd = max(20, K // 5)
    log(f"mixed, dense nuclear kernel: {dense['seconds'] / kd * 1e3:.4f} ms/step")
    # the Newton-3 half-stencil nuclear variant (each unordered pair once,
    # reactions in fixed point), for comparison with the full stencil
    old = B.pasta_set_tuning(nuclear_variant=4, fused_forces=1)
    n3 = run_path(B, torch, st, B.PASTA_MIXED, max(20, K // 5), min(W, 20), timing=True)
    B.pasta_set_tuning(**old)
    kn3 = max(20, K // 5)
    log(f"mixed, Newton-3 half stencil: {n3['seconds'] / kn3 * 1e3:.4f} ms/step")
    k64 = args.fp64_steps or max(20, K // 4)
    B.pasta_set_tuning(**tuned64)
    if use_lists:
        B.pasta_set_tuning(nuclear_variant=2, list_skin=skin)
    fp64 = run_path(B, torch, st, B.PASTA_FP64, k64, min(W, 20), timing=True)
    B.pasta_set_tuning(**tuned)
    log(f"fp64: {fp64['seconds'] / k64 * 1e3:.4f} ms/step")

    useful = mixed["nuc_pairs"] + mixed["coul_pairs"]
    ms_step = mixed["seconds"] / K * 1e3
    value = useful * K / mixed["seconds"]
    steps_s = K / mixed["seconds"]
    fp64_ms = fp64["seconds"] / k64 * 1e3

    # roofline of the dominant kernel (largest share of the step)
    kt = mixed["kernel_times"]
    dom = max(kt, key=lambda k: kt[k][0])
    ms_tot, launches = kt[dom]
    avg_ms = ms_tot / max(launches, 1)
    if dom == "nuclear+kick" and (tuned.get("fused_forces") or kernel_variant(tuned) >= 4):
        # one launch carries both the nuclear items and the Coulomb tiles
        roof = roofline_entry(pair_kernel_name(tuned, use_lists), mixed["nuc_pairs"],
                              mixed["coul_pairs"], avg_ms, B.PASTA_MIXED)
        roof["traffic"] = None if use_lists else measured_traffic(
            "k_forces_fused<MixedPolicy, 0, %d, %d>" % (
                kernel_variant(tuned), FUSED_COULOMB_ARG[tuned.get("coulomb_form", 0)]), tuned)
        roof["traffic_unit"] = "bytes per launch (HBM, counter runs in profiles/)"
    elif dom in ("coulomb", "nuclear+kick"):
        roof = roofline_entry(dom, mixed["nuc_pairs"] if dom == "nuclear+kick" else 0,
                              mixed["coul_pairs"] if dom == "coulomb" else 0, avg_ms,
                              B.PASTA_MIXED)
        roof["traffic"] = None
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": 8000.0,
                "unit": "GB/s", "frac": None, "traffic": None, "avg_launch_ms": round(avg_ms, 5)}
    # the FP64 path's pair kernel against the FP64 vector peak
    kt64 = fp64["kernel_times"]
    ms64, nl64 = kt64.get("nuclear+kick", (0.0, 0))
    roof64 = roofline_entry(pair_kernel_name(tuned64, use_lists), fp64["nuc_pairs"],
                            fp64["coul_pairs"], ms64 / max(nl64, 1), B.PASTA_FP64) if nl64 else None

    # the same workload with the Coulomb term cut at 20 fm (an option; the
    # paper's Coulomb term is uncut): gather form with the FP64 cutoff test
    pot20 = B.pasta_potential_paper()
    pot20.r_coul = 20.0
    cut20 = run_path(B, torch, st, B.PASTA_MIXED, K, W, timing=False, pot=pot20)
    cut20_entry = {"ms_per_step": cut20["seconds"] / K * 1e3,
                   "md_steps_per_s": K / cut20["seconds"],
                   "pair_interactions_per_s": (cut20["nuc_pairs"] + cut20["coul_pairs"]) * K /
                   cut20["seconds"],
                   "useful_pairs_per_step": {"nuclear": cut20["nuc_pairs"],
                                             "coulomb_inside_20fm": cut20["coul_pairs"]},
                   "precision": "mixed"}
    log(f"mixed, Coulomb cut at 20 fm: {cut20_entry['ms_per_step']:.4f} ms/step")

    large = None
    decomp = None
    if not args.no_large:
        large = large_section(B, torch)
    if not args.no_decompression:
        decomp = decompression_section(B, torch)
        B.pasta_set_tuning(**tuned)

    batched = None
    via_batch = None
    if not args.no_batch:
        batched = batched_section(B, torch, args.batch_steps, min(W, 20))
        # the same N = 51 200 system through the batched machinery (one
        # system, graph replay, each mode tuned on it) for comparison
        via_batch = single_via_batch(B, torch, st, K, W)

    cpu = None
    if not args.no_cpu_baseline:
        nuc_per = 2 * mixed["nuc_pairs"] / N
        sp = st["species"]

        def pairs_for(sample):
            return float(len(sample) * nuc_per + (sp[sample] == 1).sum() * (Z - 1))
        cpu = cpu_baseline(st, pairs_for)

    per_kernel = {k: {"ms_per_step": round(v[0] / max(K, 1), 5), "launches": v[1]}
                  for k, v in kt.items() if v[1]}
    out = {
        "metric": "pair interactions/s & MD steps/s at N=51,200; mixed/batched vs FP64 GPU",
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-pair/f64-acc",
        "data": "synthetic (seeded uniform-random start, Maxwell-Boltzmann velocities)",
        "config": {"workload": "N=51200 Y_P=0.20 n=0.080 fm^-3 L=86.18 fm T=0.75 MeV dt=2 fm/c "
                               "rescale every 100 steps, uncut screened Coulomb, r_nuc=11.5 fm",
                   "N": N, "Z": Z, "L_fm": st["L"], "precision": "mixed",
                   "parallelism": "single GPU"},
        "md_steps_per_s": steps_s,
        "timing_windows": {
            "main_window_ms_per_step": ms_step,
            "further_windows_ms_per_step": [round(x, 5) for x in mixed["windows_ms"]],
            "median_of_windows_ms_per_step": float(np.median([ms_step] + mixed["windows_ms"])),
            "note": "the same simulation, 5 further windows of K/5 steps after the main K; "
                    "the single-system path launches its kernels per step (no graph to build)"},
        "environment": dict(device_environment(torch), **(host_env or {})),
        "useful_pairs_per_step": {"nuclear": mixed["nuc_pairs"], "coulomb": mixed["coul_pairs"]},
        "evaluated_pairs_per_step": {
            "nuclear_stencil_ordered": mixed["stencil_candidates"],
            "nuclear_useful_ordered": 2 * mixed["nuc_pairs"],
            "stencil_over_useful": mixed["stencil_candidates"] / max(1.0, 2 * mixed["nuc_pairs"]),
            "cells_per_side": mixed["ncell"],
            "coulomb_evaluated": mixed["coul_pairs"],
            "note": "nuclear: ordered candidate pairs of the 27-cell stencil at the final state "
                    "(the kernels' staging culls them further to the sources within r_nuc of "
                    "each work item's bounding box); coulomb: every unordered proton pair once "
                    "(pairwise form)"},
        "evaluated_tests_per_s": (mixed["stencil_candidates"] + mixed["coul_pairs"]) * 1e3 / ms_step,
        "fp64": {"ms_per_step": fp64_ms, "md_steps_per_s": 1e3 / fp64_ms,
                 "pair_interactions_per_s": (fp64["nuc_pairs"] + fp64["coul_pairs"]) * 1e3 / fp64_ms,
                 "steps": k64,
                 "per_kernel_ms": kernel_ms(fp64["kernel_times"], k64)},
        "mixed_over_fp64_speedup": fp64_ms / ms_step,
        "autotuned": {"mixed": tuned, "fp64": tuned64,
                      "candidates": "[fused_forces, nuclear_variant, coulomb_form, "
                                    "coulomb_splits, ms]",
                      "mixed_candidates_ms": [[c["fused_forces"], c["nuclear_variant"],
                                               c.get("coulomb_form", 0), c["coulomb_splits"],
                                               round(ms, 5)] for c, ms in table],
                      "fp64_candidates_ms": [[c["fused_forces"], c["nuclear_variant"],
                                              c.get("coulomb_form", 0), c["coulomb_splits"],
                                              round(ms, 5)] for c, ms in table64],
                      "step_runoff": "candidates within 3 % of the fastest force-only time, "
                                     "timed on simulation steps: [fused_forces, "
                                     "nuclear_variant, coulomb_form, nuclear_tile, ms per step]",
                      "mixed_runoff_ms": [[c["fused_forces"], c["nuclear_variant"],
                                           c.get("coulomb_form", 0), c.get("nuclear_tile", 0),
                                           round(ms, 5)] for c, ms in (runoff or [])],
                      "fp64_runoff_ms": [[c["fused_forces"], c["nuclear_variant"],
                                          c.get("coulomb_form", 0), c.get("nuclear_tile", 0),
                                          round(ms, 5)] for c, ms in (runoff64 or [])]},
        "dense_nuclear_variant": {"ms_per_step": dense["seconds"] / kd * 1e3,
                                  "nuclear_ms": dense["kernel_times"]["nuclear+kick"][0] / kd},
        "newton3_half_stencil_variant": {"ms_per_step": n3["seconds"] / kn3 * 1e3,
                                         "per_kernel_ms": kernel_ms(n3["kernel_times"], kn3)},
        "nuclear_form": "neighbour lists" if use_lists else "cell sweeps",
        "cell_sweeps": {"ms_per_step": mixed_cells["seconds"] / K * 1e3,
                        "per_kernel_ms": {k: round(v[0] / K, 5)
                                          for k, v in mixed_cells["kernel_times"].items() if v[1]}},
        "neighbour_lists": {"ms_per_step": mixed_lists["seconds"] / K * 1e3, "halo_fm": skin,
                            "halo_trials_ms": [[h, round(ms, 5), nb] for h, ms, nb in skin_table],
                            "builds": mixed_lists["list_stats"]["builds"],
                            "steps_run": mixed_lists["steps"],
                            "overflows": mixed_lists["list_stats"]["overflows"],
                            "per_kernel_ms": {k: round(v[0] / K, 5)
                                              for k, v in mixed_lists["kernel_times"].items()
                                              if v[1]}},
        "ms_per_step_with_events": mixed["seconds_with_events"] / K * 1e3,
        "per_kernel": per_kernel,
        "memory_kernels": memory_kernels(per_kernel, N),
        "roofline": roof,
        "fp64_roofline": roof64,
        "coulomb_cut_20fm": cut20_entry,
        "large": large,
        "decompression": decomp,
        "batched": batched,
        "single_system_via_batch_path": via_batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
