"""GPU parity of the neighbour-list form of the nuclear force (Sec. II.B.1:
lists of the sources within r_nuc + delta_r, rebuilt only when a source
outside a list could have come into range) against the FP64 oracle.

The lists change which candidates are visited and in what order, never the
pair set inside r_nuc, so the bar is the same as for the cell sweeps:
forces and energies to the normwise and per-particle gates of
tests/parity.py, trajectories as in test_gpu_parity.py, pair counts exact.
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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    oracle.build()
    return dict(torch=torch, B=B, O=oracle, I=inputs, dev=torch.device("cuda:0"))


def say(*a):
    print(*a, flush=True)


def wrapped_diff(a, b, L):
    d = a - b
    return d - L * np.round(d / L)


class lists:
    """Switches the process-wide setting to the list form for a block."""

    def __init__(self, B, skin=2.0, fused=None, pool_scale=1.0):
        self.B, self.kw = B, dict(nuclear_variant=2, list_skin=skin, list_pool_scale=pool_scale)
        if fused is not None:
            self.kw["fused_forces"] = fused

    def __enter__(self):
        self.old = self.B.pasta_set_tuning(**self.kw)

    def __exit__(self, *exc):
        self.B.pasta_set_tuning(**self.old)


def make_sim(env, st, **kw):
    t = env["torch"]
    pos = t.tensor(st["pos"], device=env["dev"])
    vel = t.tensor(st["vel"], device=env["dev"])
    sp = t.tensor(st["species"], device=env["dev"])
    return env["B"].Sim(pos, vel, sp, st["L"], **kw), pos, vel


CASES = [
    # (N, Y_P, density, seed)
    (3200, 0.40, 0.040, 1000),   # the small configuration
    (1000, 0.30, 0.060, 5),      # L = 25.5: one list cell per side
    (4097, 0.20, 0.080, 6),      # ragged
    (6000, 1.00, 0.050, 8),      # all protons
    (5000, 0.00, 0.070, 9),      # no protons
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("skin,fused", [(0.5, 1), (2.0, 0), (2.0, 1), (4.0, 1)])
def test_list_forces_one_shot(env, case, prec, skin, fused):
    N, yp, dens, seed = case
    say("list forces", case, "prec", prec, "skin", skin, "fused", fused)
    B, t = env["B"], env["torch"]
    st = env["I"].make_state(N, yp, dens, 1.0, seed=seed)
    pos = t.tensor(st["pos"], device=env["dev"])
    sp = t.tensor(st["species"], device=env["dev"])
    with lists(B, skin, fused):
        f, e = B.pasta_forces(pos, sp, st["L"], precision=prec)
    of, oe = env["O"].forces(st["pos"], st["species"], st["L"])
    check(f.cpu().numpy(), of, prec, e.cpu().numpy(), oe, what=f"lists {case}", say=say)


@pytest.mark.parametrize("prec", [0, 1])
def test_list_forces_full_size(env, prec):
    B, t = env["B"], env["torch"]
    st = env["I"].workload("n51200_yp020_n0.080")
    pos = t.tensor(st["pos"], device=env["dev"])
    sp = t.tensor(st["species"], device=env["dev"])
    with lists(B, 2.0):
        f, e = B.pasta_forces(pos, sp, st["L"], precision=prec)
    # every target (the oracle's 51 200 exact sums)
    of, oe = env["O"].forces(st["pos"], st["species"], st["L"])
    check(f.cpu().numpy(), of, prec, e.cpu().numpy(), oe, what="lists 51200", say=say)


@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 2e-4)])
@pytest.mark.parametrize("fused", [0, 1])
def test_list_trajectory_vs_oracle(env, prec, tol, fused):
    """20 steps with an expanding box and a velocity rescale every 5 steps;
    one particle is given a large velocity so that displacements force
    rebuilds along the way."""
    B = env["B"]
    st = dict(env["I"].workload("n3200_yp040_n0.040"))
    st["vel"] = st["vel"].copy()
    st["vel"][17] = [0.45, -0.3, 0.2]  # about 1.2 fm per step
    xi = 1e-3
    L_max = st["L"] * (1 + xi * 2.0 * 20)
    with lists(B, 2.0, fused):  # fused_forces is read at every launch
        sim, pos, vel = make_sim(env, st, dt=2.0, xi_dot=xi, T=1.0, rescale_every=5,
                                 precision=prec, L_max=L_max)
        sim.step(20)
        en = sim.energies()
        stats = sim.list_stats()
    op, ov, oL, oek, oep, of = env["O"].run(st["pos"], st["vel"], st["species"], st["L"], 20,
                                            dt=2.0, xi_dot=xi, T=1.0, rescale_every=5)
    dx = np.abs(wrapped_diff(pos.cpu().numpy(), op, oL)).max()
    say(f"  prec {prec} fused {fused}: max |dx| {dx:.3e}, lists {stats}")
    assert en["L"] == oL and en["step"] == 20
    assert dx <= tol
    assert np.abs(vel.cpu().numpy() - ov).max() <= 10 * tol
    assert stats["builds"] >= 3 and stats["overflows"] == 0
    # the forces at the final GPU state, against the oracle on the same bits
    f, _ = sim.forces()
    of2, _ = env["O"].forces(pos.cpu().numpy(), st["species"], oL)
    check(f.cpu().numpy(), of2, prec, what="lists after 20 steps", say=say)
    nn, _ = sim.pair_counts()
    assert nn == env["O"].pair_counts(pos.cpu().numpy(), st["species"], oL)[0]
    sim.close()


def test_list_halo_sets_rebuild_rate(env):
    """A thin halo rebuilds almost every step, a thick one rarely; both follow
    the oracle."""
    B = env["B"]
    st = env["I"].make_state(2400, 0.3, 0.05, 1.0, seed=81)
    out = {}
    for skin in (0.05, 3.0):
        with lists(B, skin):
            sim, pos, vel = make_sim(env, st, dt=2.0, T=1.0, precision=0)
        sim.step(15)
        out[skin] = (pos.cpu().numpy(), sim.list_stats())
        sim.close()
    op, *_ = env["O"].run(st["pos"], st["vel"], st["species"], st["L"], 15, dt=2.0)
    for skin, (p, stats) in out.items():
        dx = np.abs(wrapped_diff(p, op, st["L"])).max()
        say(f"  skin {skin}: {stats}, max |dx| {dx:.2e}")
        assert dx <= 1e-9
    assert out[0.05][1]["builds"] >= 14
    assert out[3.0][1]["builds"] < out[0.05][1]["builds"]


@pytest.mark.parametrize("prec", [0, 1])
def test_list_overflow_falls_back(env, prec):
    """With almost no list memory every build runs out; the forces then come
    from the screened cell sweep over the build's cells and still match."""
    B = env["B"]
    st = env["I"].make_state(3000, 0.3, 0.06, 1.0, seed=83)
    with lists(B, 2.0, pool_scale=1e-3):
        sim, pos, vel = make_sim(env, st, dt=2.0, T=1.0, rescale_every=4, precision=prec)
    sim.step(8)
    stats = sim.list_stats()
    say("  overflow stats", stats)
    assert stats["overflows"] >= 1
    op, ov, oL, *_ = env["O"].run(st["pos"], st["vel"], st["species"], st["L"], 8, dt=2.0,
                                  T=1.0, rescale_every=4)
    assert np.abs(wrapped_diff(pos.cpu().numpy(), op, oL)).max() <= (1e-9 if prec == 0 else 2e-4)
    f, _ = sim.forces()
    of, _ = env["O"].forces(pos.cpu().numpy(), st["species"], oL)
    check(f.cpu().numpy(), of, prec, what="lists after overflow", say=say)
    sim.close()


def test_list_growing_box_regrids(env):
    """The box grows by 40 % over 2000 steps: the list cells are re-derived
    at every rebuild (4 -> 6 per side), forces checked on snapshots."""
    B = env["B"]
    st = env["I"].make_state(20000, 0.3, 0.08, 0.75, seed=85)
    xi = 0.4 / (2000 * 2.0)
    with lists(B, 2.0):
        sim, pos, vel = make_sim(env, st, dt=2.0, xi_dot=xi, T=0.75, rescale_every=100,
                                 precision=1, L_max=st["L"] * 1.4 * (1 + 1e-12))
    rng = np.random.Generator(np.random.PCG64(86))
    for k in range(5):
        if k:
            sim.step(500)
        L = sim.energies()["L"]
        f, _ = sim.forces()
        tg = rng.choice(st["n"], 2000, replace=False)
        of, _ = env["O"].forces(pos.cpu().numpy(), st["species"], L, targets=tg)
        stats = sim.list_stats()
        say(f"  step {500 * k}: L {L:.3f}, lists {stats}")
        check(f.cpu().numpy()[tg], of, 1, what=f"lists step {500 * k}", say=say)
        assert stats["overflows"] == 0
    assert L == pytest.approx(st["L"] * 1.4, rel=1e-12)
    sim.close()


def test_list_restart_deterministic(env):
    """Two restarts from the same checkpoint (each rebuilds the lists) give
    identical bits."""
    t, B = env["torch"], env["B"]
    st = env["I"].make_state(2000, 0.3, 0.05, 1.0, seed=87)
    with lists(B, 1.0):
        sim, pos, vel = make_sim(env, st, dt=2.0, T=1.0, rescale_every=7, precision=1)
    sim.step(9)
    cp = (pos.clone(), vel.clone(), sim.get_step())
    runs = []
    for _ in range(2):
        sim.set_state(*cp)
        sim.step(11)
        runs.append((pos.clone(), vel.clone()))
    assert t.equal(runs[0][0], runs[1][0]) and t.equal(runs[0][1], runs[1][1])
    sim.close()


def test_list_matches_cell_sweep(env):
    """The list form and the cell sweep integrate the same dynamics: after
    40 FP64 steps they agree to rounding growth."""
    B = env["B"]
    st = env["I"].make_state(5000, 0.2, 0.08, 0.75, seed=89)
    res = []
    for variant in (1, 2):
        old = B.pasta_set_tuning(nuclear_variant=variant, list_skin=1.5)
        try:
            sim, pos, vel = make_sim(env, st, dt=2.0, T=0.75, rescale_every=10, precision=0)
        finally:
            B.pasta_set_tuning(**old)
        sim.step(40)
        res.append((pos.cpu().numpy(), sim.energies()))
        sim.close()
    dx = np.abs(wrapped_diff(res[0][0], res[1][0], st["L"])).max()
    say(f"  list vs cell sweep after 40 steps: max |dx| {dx:.2e}")
    assert dx <= 1e-6
    assert res[1][1]["ekin"] == pytest.approx(res[0][1]["ekin"], rel=1e-7)
