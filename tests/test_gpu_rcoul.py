"""GPU parity of the optional Coulomb cutoff r_coul (the paper's Coulomb term
is uncut; a 20 fm cutoff is the variant some benchmarks quote): forces and
energies against the oracle with the same r_coul, on the small configuration
(N = 3200, L = 43.09 fm, so L / r_coul is barely above 2) and on every target
of the N = 51 200 workload, pairs placed exactly around the cutoff (the
include test is decided on the FP64 r^2 of the definition in both
precisions), a trajectory and the pair counts."""
import numpy as np
import pytest

from parity import check

pytestmark = pytest.mark.gpu

R_COUL = 20.0


@pytest.fixture(scope="module")
def env():
    import torch
    import oracle
    from paper_1412_8502_amd import binding as B
    from paper_1412_8502_amd import inputs
    assert torch.cuda.is_available()
    oracle.build()
    pot = B.pasta_potential_paper()
    pot.r_coul = R_COUL
    return dict(torch=torch, B=B, O=oracle, I=inputs, dev=torch.device("cuda:0"), pot=pot)


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name", ["n3200_yp040_n0.040", "n51200_yp020_n0.080"])
def test_cutoff_forces(env, name, prec, fused):
    t, B, O = env["torch"], env["B"], env["O"]
    st = env["I"].workload(name)
    pos = t.tensor(st["pos"], device=env["dev"])
    sp = t.tensor(st["species"], device=env["dev"])
    old = B.pasta_set_tuning(fused_forces=fused, coulomb_form=1)  # the cutoff takes the gather form
    try:
        f, e = B.pasta_forces(pos, sp, st["L"], precision=prec, pot=env["pot"])
    finally:
        B.pasta_set_tuning(**old)
    of, oe = O.forces(st["pos"], st["species"], st["L"], params=dict(r_coul=R_COUL))
    check(f.cpu().numpy(), of, prec, e.cpu().numpy(), oe, what=f"r_coul {name} fused {fused}",
          say=say)
    # the cut changes the result: the uncut forces differ
    ouf, _ = O.forces(st["pos"], st["species"], st["L"])
    assert np.abs(of - ouf).max() > 1e-4


@pytest.mark.parametrize("prec", [0, 1])
def test_cutoff_band(env, prec):
    """Proton pairs at 20 fm and a few ulps to 1e-7 fm either side, along each
    axis, alone in the box: kept exactly when the oracle keeps them."""
    t, B, O = env["torch"], env["B"], env["O"]
    L = 60.0
    kept = 0
    for axis in range(3):
        for dr in (-1e-7, -1e-9, -1e-12, -3.6e-15, 0.0, 3.6e-15, 1e-12, 1e-9, 1e-7):
            p = np.full((2, 3), 7.0)
            p[1, axis] = 7.0 + R_COUL + dr
            s = np.array([1, 1], np.uint8)
            of, oe = O.forces(p, s, L, params=dict(r_coul=R_COUL))
            f, e = B.pasta_forces(t.tensor(p, device=env["dev"]), t.tensor(s, device=env["dev"]),
                                  L, precision=prec, pot=env["pot"])
            f, e = f.cpu().numpy(), e.cpu().numpy()
            assert (np.abs(f).sum() > 0) == (np.abs(of).sum() > 0), (axis, dr, f, of)
            kept += int(np.abs(of).sum() > 0)
            check(f, of, prec, e, oe, what=f"band {axis} {dr}", say=lambda *a: None)
    assert kept == 3 * 4  # the four separations below 20 fm, on each axis


@pytest.mark.parametrize("prec,tol", [(0, 1e-9), (1, 2e-4)])
def test_cutoff_trajectory_and_counts(env, prec, tol):
    t, B, O = env["torch"], env["B"], env["O"]
    st = env["I"].workload("n3200_yp040_n0.040")
    pos = t.tensor(st["pos"], device=env["dev"])
    vel = t.tensor(st["vel"], device=env["dev"])
    sp = t.tensor(st["species"], device=env["dev"])
    sim = B.Sim(pos, vel, sp, st["L"], dt=2.0, T=1.0, rescale_every=7, precision=prec,
                pot=env["pot"])
    sim.step(20)
    op, ov, oL, *_ = O.run(st["pos"], st["vel"], st["species"], st["L"], 20, dt=2.0, T=1.0,
                           rescale_every=7, params=dict(r_coul=R_COUL))
    d = pos.cpu().numpy() - op
    d -= st["L"] * np.round(d / st["L"])
    say(f"  prec {prec}: max |dx| {np.abs(d).max():.3e}")
    assert np.abs(d).max() <= tol
    P = pos.cpu().numpy()
    nn, nc = sim.pair_counts()
    onn, onc = O.pair_counts(P, st["species"], st["L"], params=dict(r_coul=R_COUL))
    assert (nn, nc) == (onn, onc)
    assert nc < st["Z"] * (st["Z"] - 1) // 2
    f, _ = sim.forces()
    of, _ = O.forces(P, st["species"], st["L"], params=dict(r_coul=R_COUL))
    check(f.cpu().numpy(), of, prec, what="r_coul after 20 steps", say=say)
    sim.close()
