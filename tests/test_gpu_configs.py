"""The paper-shaped workloads end to end on the GPU.

* Decompression window: N = 51 200, Y_P = 0.30, T = 0.5 MeV, box grown from
  0.080 to 0.00125 fm^-3 (L 86.18 -> 344.7 fm, the paper's density endpoints)
  over 20 000 steps of 2 fm/c (xi_dot = 7.5e-5 c/fm), velocity rescale every
  100 steps, mixed precision, cell grid re-derived as the box grows.  The
  cluster algorithm runs every 2000 steps on the GPU state and must match the
  oracle bit for bit; the box side must equal Eq. (3a) exactly and sampled
  forces must match the oracle on every snapshot.
* Large: N = 409 600 at Y_P = 0.40 and the neutron-rich Y_P = 0.05 of the
  paper's large runs, 200 steps in FP64 and in mixed precision, then forces
  on 2000 sampled targets against the oracle (per-particle gate) and the
  device clusters bit for bit against the oracle's cluster algorithm, with
  scipy's periodic k-d tree and connected components as a second witness.
* Energy drift at the headline size (N = 51 200): six FP64 and six mixed NVE
  runs of 1000 steps from the same warmed positions.
"""
import numpy as np
import pytest

from parity import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import oracle
    from paper_1412_8502_amd import binding as B
    from paper_1412_8502_amd import inputs
    assert torch.cuda.is_available()
    oracle.build()
    return dict(torch=torch, B=B, O=oracle, I=inputs, dev=torch.device("cuda:0"))


def say(*a):
    print(*a, flush=True)


def test_decompression_window(env):
    t, B, O = env["torch"], env["B"], env["O"]
    st = env["I"].workload("n51200_yp030_n0.080")
    L0, xi, dt = st["L"], 7.5e-5, 2.0
    pos = t.tensor(st["pos"], device=env["dev"])
    vel = t.tensor(st["vel"], device=env["dev"])
    sp = t.tensor(st["species"], device=env["dev"])
    sim = B.Sim(pos, vel, sp, L0, dt=dt, xi_dot=xi, T=0.5, rescale_every=100,
                precision=B.PASTA_MIXED, L_max=4.0 * L0 * (1 + 1e-12))
    rng = np.random.Generator(np.random.PCG64(3))
    for k in range(11):
        if k:
            sim.step(2000)
        en = sim.energies()
        L = en["L"]
        assert en["step"] == 2000 * k
        assert L == O.box_length(L0, xi, dt, 2000 * k)
        P = pos.cpu().numpy()
        cl = B.pasta_cluster(pos, sp, L)
        ref = O.cluster(P, st["species"], L)
        assert cl["nclusters"] == ref["nclusters"] and cl["nfree"] == ref["nfree"]
        assert np.array_equal(cl["label"].cpu().numpy(), ref["label"])
        assert np.array_equal(cl["hist_A"].cpu().numpy(), ref["hist_A"])
        assert np.array_equal(cl["hist_Z"].cpu().numpy(), ref["hist_Z"])
        f, _ = sim.forces()
        tg = rng.choice(st["n"], 2000, replace=False)
        of, _ = O.forces(P, st["species"], L, targets=tg)
        stats = O.cluster_stats(ref, st["species"])
        say(f"  step {2000 * k:5d}: n = {st['n'] / L ** 3:.5f} fm^-3, K = {ref['nclusters']}, "
            f"free n = {ref['nfree']}, A>=12: {stats.get('n_heavy', 0)}")
        check(f.cpu().numpy()[tg], of, 1, what=f"decompression step {2000 * k}", say=say)
    assert L == pytest.approx(4.0 * L0, rel=1e-12)
    sim.close()


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("name", ["n409600_yp040_n0.080", "n409600_yp005_n0.080"])
def test_large_system(env, name, prec):
    """200 steps at N = 409 600, then sampled forces against the oracle and
    the device clusters against the oracle's cluster algorithm, bit for bit
    (labels, cluster count, free neutrons, A and Z histograms)."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree
    t, B, O = env["torch"], env["B"], env["O"]
    say("large", name, "prec", prec)
    st = env["I"].workload(name)
    L = st["L"]
    pos = t.tensor(st["pos"], device=env["dev"])
    vel = t.tensor(st["vel"], device=env["dev"])
    sp = t.tensor(st["species"], device=env["dev"])
    sim = B.Sim(pos, vel, sp, L, dt=2.0, T=1.0, rescale_every=100, precision=prec)
    sim.step(200)
    en = sim.energies()
    assert np.isfinite(en["ekin"]) and np.isfinite(en["epot"]) and en["step"] == 200
    P = pos.cpu().numpy()
    s = st["species"]
    # forces on the GPU's own final state against the oracle: 1000 protons
    # and 1000 neutrons
    f, _ = sim.forces()
    rng = np.random.Generator(np.random.PCG64(4))
    tg = np.concatenate([rng.choice(st["Z"], 1000, replace=False),
                         st["Z"] + rng.choice(st["n"] - st["Z"], 1000, replace=False)])
    of, _ = O.forces(P, s, L, targets=tg)
    check(f.cpu().numpy()[tg], of, prec, what=f"{name} after 200 steps", say=say)
    sim.close()
    cl = B.pasta_cluster(pos, sp, L)
    lab = cl["label"].cpu().numpy()
    hA, hZ = cl["hist_A"].cpu().numpy(), cl["hist_Z"].cpu().numpy()
    # the oracle's cluster algorithm on the same bits
    ref = O.cluster(P, s, L)
    assert cl["nclusters"] == ref["nclusters"] and cl["nfree"] == ref["nfree"]
    assert np.array_equal(lab, ref["label"])
    assert np.array_equal(hA, ref["hist_A"]) and np.array_equal(hZ, ref["hist_Z"])
    # second witness: the partition of the protons is the connected
    # components of the r <= 4.5 fm graph, numbered by smallest proton index
    pidx = np.nonzero(s == 1)[0]
    tree = cKDTree(np.mod(P[pidx], L), boxsize=L)
    pairs = tree.query_pairs(4.5, output_type="ndarray")
    g = coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(len(pidx),) * 2)
    ncomp, comp = connected_components(g, directed=False)
    first = np.full(ncomp, np.iinfo(np.int64).max)
    np.minimum.at(first, comp, pidx)
    rank = np.empty(ncomp, np.int64)
    rank[np.argsort(first)] = np.arange(ncomp)
    assert cl["nclusters"] == ncomp
    assert np.array_equal(lab[pidx], rank[comp])
    assert (np.arange(len(hA)) * hA).sum() + cl["nfree"] == st["n"]
    assert (np.arange(len(hZ)) * hZ).sum() == st["Z"]
    say(f"  large: K = {ncomp}, free = {cl['nfree']}, largest A = {np.nonzero(hA)[0].max()}")


def test_energy_drift_headline(env):
    """Energy conservation at N = 51 200 (Y_P = 0.20, 0.08 fm^-3): 500 steps
    with the velocity rescaled every step take the random start's close
    pairs out; from those warmed positions, K = 6 NVE runs of 1000 steps of
    dt = 2 fm/c, each with fresh Maxwell-Boltzmann velocities at T (seeded
    per run, the same K velocity sets for FP64 and for mixed), H/N recorded
    every 20 fm/c.

    Stated bound (per nucleon, means over the K runs): the mixed runs'
    max |H(t) - H(0)|/N is within the FP64 runs' plus 1e-4 MeV, and their
    systematic drift (the mean slope of a straight-line fit of H/N, per 1000
    steps) within the FP64 runs' plus 1e-4 MeV: the FP32 pair arithmetic
    adds no drift of its own.  The means are taken because each trajectory
    is chaotic: one run's max and slope scatter by about the standard
    deviation of H (~2e-4 MeV here) from run to run, more than the 1e-4
    margin; over K = 6 runs the scatter of the means is ~2.5x smaller.  For
    both precisions, halving dt (2000 steps of 1 fm/c over the same span,
    first velocity set) at least halves the standard deviation of H (the
    error is Verlet's).  The FP64 drift itself is tied to the oracle's at
    N = 600 (test_gpu_parity.py::test_energy_drift), where the oracle runs
    the same protocol; an oracle run of 1000 steps at N = 51 200 would take
    most of an hour on the host."""
    t, B = env["torch"], env["B"]
    st = env["I"].workload("n51200_yp020_n0.080")
    pos = t.tensor(st["pos"], device=env["dev"])
    vel = t.tensor(st["vel"], device=env["dev"])
    sp = t.tensor(st["species"], device=env["dev"])
    sim = B.Sim(pos, vel, sp, st["L"], dt=2.0, T=st["T"], rescale_every=1, precision=0)
    sim.step(500)
    t.cuda.synchronize()
    p0 = pos.clone()
    sim.close()
    K = 6
    vsets = []
    for k in range(K):
        rng = np.random.Generator(np.random.PCG64(5000 + k))
        v = rng.standard_normal((st["n"], 3)) * np.sqrt(st["T"] / env["I"].MASS_MEV)
        vsets.append(t.tensor(v, device=env["dev"]))

    def series(prec, dt, v0):
        p, v = p0.clone(), v0.clone()
        s = B.Sim(p, v, sp, st["L"], dt=dt, T=st["T"], precision=prec)
        e = s.energies()
        H = [(e["ekin"] + e["epot"]) / st["n"]]
        for _ in range(100):
            s.step(int(round(20.0 / dt)))
            e = s.energies()
            H.append((e["ekin"] + e["epot"]) / st["n"])
        s.close()
        return np.array(H)

    tt = np.linspace(0.0, 2000.0, 101)
    D, drift = {}, {}
    for prec in (0, 1):
        ds, sl = [], []
        for k in range(K):
            h2 = series(prec, 2.0, vsets[k])
            assert np.all(np.isfinite(h2))
            ds.append(np.abs(h2 - h2[0]).max())
            sl.append(np.polyfit(tt, h2, 1)[0] * 2000.0)
            if k == 0:
                h1 = series(prec, 1.0, vsets[k])
                assert np.all(np.isfinite(h1))
                say(f"  prec {prec}: std of H {h2.std():.3e} (dt=2) {h1.std():.3e} (dt=1)")
                assert h1.std() <= 0.5 * h2.std()
        D[prec], drift[prec] = float(np.mean(ds)), abs(float(np.mean(sl)))
        say(f"  prec {prec}: max|H-H0| per run {' '.join(f'{x:.2e}' for x in ds)}"
            f" mean {D[prec]:.3e}; slopes per run {' '.join(f'{x:.2e}' for x in sl)}"
            f" |mean| {drift[prec]:.3e} MeV/nucleon per 1000 steps")
    assert D[1] <= D[0] + 1e-4
    assert drift[1] <= drift[0] + 1e-4


def test_expansion_run_statistics(env):
    """A short decompression run through expansion.run (equilibration, then
    the box law at xi_dot = 1e-3 c/fm down to 0.01 fm^-3): the reported
    density and Table II statistics must equal the oracle's cluster algorithm
    and statistics on the run's final state."""
    from paper_1412_8502_amd import expansion
    O = env["O"]
    res, P, L = expansion.run(3200, 0.3, 1.0, -3.0, 1000, seed=77, report_every=500,
                              log=say, return_state=True)
    st = env["I"].make_state(3200, 0.3, 0.08, 1.0, 77)
    assert res["expansion_steps"] == 500
    assert res["n_final"] == pytest.approx(0.01, rel=1e-9)
    assert L == O.box_length(st["L"], 1e-3, 2.0, 500)
    ref = O.cluster_stats(O.cluster(P, st["species"], L), st["species"])
    say(f"  run: {res}")
    assert res["clusters"] == ref["nclusters"]
    assert res["clusters_A_ge_12"] == ref["n_heavy"]
    assert res["mass_fraction_free_neutrons"] == ref["x_free"]
    if ref["n_heavy"]:
        assert res["mean_A"] == ref["A_mean"] and res["sd_A"] == ref["A_std"]
        assert res["mean_Z"] == ref["Z_mean"] and res["sd_Z"] == ref["Z_std"]


def test_expansion_checkpoint_resume(env, tmp_path):
    """A decompression run cut into three segments through checkpoint files
    (mid-equilibration, then mid-expansion) takes the same steps as the uncut
    run: the resumed simulation starts at the saved global step, so the box
    law and the thermostat cadence continue, and the final positions, box
    side and statistics equal the uncut run's bit for bit."""
    from paper_1412_8502_amd import expansion
    args = (3200, 0.3, 1.0, -3.0, 1000)
    kw = dict(seed=78, report_every=250, log=say)
    ref, P_ref, L_ref = expansion.run(*args, return_state=True, **kw)
    ck = tmp_path / "run.npz"
    r1 = expansion.run(*args, checkpoint=ck, max_steps=750, **kw)
    assert r1["status"] == "checkpointed" and (r1["phase"], r1["done"]) == (0, 750)
    r2 = expansion.run(*args, checkpoint=ck, resume=ck, max_steps=500, **kw)
    assert r2["status"] == "checkpointed" and (r2["phase"], r2["done"]) == (1, 250)
    r3, P, L = expansion.run(*args, resume=ck, return_state=True, **kw)
    say(f"  max |dx| = {np.abs(P - P_ref).max():.3e}")
    assert r3["status"] == "done" and r3["segments"] == 3
    assert L == L_ref
    assert np.array_equal(P, P_ref)
    for k in ("clusters", "clusters_A_ge_12", "mass_fraction_free_neutrons", "largest_A"):
        assert r3[k] == ref[k]
