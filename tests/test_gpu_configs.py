"""The paper-shaped workloads end to end on the GPU.

* Decompression window: N = 51 200, Y_P = 0.30, T = 0.5 MeV, box grown from
  0.080 to 0.00125 fm^-3 (L 86.18 -> 344.7 fm, the paper's density endpoints)
  over 20 000 steps of 2 fm/c (xi_dot = 7.5e-5 c/fm), velocity rescale every
  100 steps, mixed precision, cell grid re-derived as the box grows.  The
  cluster algorithm runs every 2000 steps on the GPU state and must match the
  oracle bit for bit; the box side must equal Eq. (3a) exactly and sampled
  forces must match the oracle on every snapshot.
* Large: N = 409 600, Y_P = 0.40, 200 steps, then device clusters checked by
  properties that hold at any size (scipy's periodic k-d tree and connected
  components), and sampled forces against the oracle.
"""
import numpy as np
import pytest

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


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


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
        tg = rng.choice(st["n"], 200, replace=False)
        of, _ = O.forces(P, st["species"], L, targets=tg)
        err = rel(f.cpu().numpy()[tg], of)
        stats = O.cluster_stats(ref, st["species"])
        say(f"  step {2000 * k:5d}: n = {st['n'] / L ** 3:.5f} fm^-3, K = {ref['nclusters']}, "
            f"free n = {ref['nfree']}, A>=12: {stats.get('n_heavy', 0)}, force err {err:.2e}")
        assert err <= 1e-5
    assert L == pytest.approx(4.0 * L0, rel=1e-12)
    sim.close()


def test_large_system(env):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree
    t, B, O = env["torch"], env["B"], env["O"]
    st = env["I"].workload("n409600_yp040_n0.080")
    L = st["L"]
    pos = t.tensor(st["pos"], device=env["dev"])
    vel = t.tensor(st["vel"], device=env["dev"])
    sp = t.tensor(st["species"], device=env["dev"])
    sim = B.Sim(pos, vel, sp, L, dt=2.0, T=1.0, rescale_every=100, precision=B.PASTA_MIXED)
    sim.step(200)
    en = sim.energies()
    assert np.isfinite(en["ekin"]) and np.isfinite(en["epot"])
    P = pos.cpu().numpy()
    s = st["species"]
    # sampled forces against the oracle on the GPU's own state
    f, _ = sim.forces()
    rng = np.random.Generator(np.random.PCG64(4))
    tg = rng.choice(st["n"], 200, replace=False)
    of, _ = O.forces(P, s, L, targets=tg)
    assert rel(f.cpu().numpy()[tg], of) <= 1e-5
    sim.close()
    # clusters: the partition of the protons must be the connected components
    # of the r <= 4.5 fm graph, numbered by smallest proton index
    cl = B.pasta_cluster(pos, sp, L)
    lab = cl["label"].cpu().numpy()
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
    # neutrons: nearest proton within 3 fm (sampled)
    nidx = np.nonzero(s == 0)[0]
    smp = rng.choice(nidx, 5000, replace=False)
    d, j = tree.query(np.mod(P[smp], L), k=1, distance_upper_bound=3.0)
    expect = np.where(np.isfinite(d), rank[comp[np.minimum(j, len(pidx) - 1)]], -1)
    assert np.array_equal(lab[smp], expect)
    # histogram invariants
    hA, hZ = cl["hist_A"].cpu().numpy(), cl["hist_Z"].cpu().numpy()
    assert (np.arange(len(hA)) * hA).sum() + cl["nfree"] == st["n"]
    assert (np.arange(len(hZ)) * hZ).sum() == st["Z"]
    say(f"  large: K = {ncomp}, free = {cl['nfree']}")


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
