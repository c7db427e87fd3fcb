"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these checks retypes the oracle's formulas: they use closed forms
derived from Eq. (1) (extrema, curvature, limits), invariants (Newton's third
law, lattice symmetry, translation/permutation equivariance, time
reversibility, Verlet's dt^2 error law), numbers the paper prints (Table I,
the density endpoints of the box law) and independent library routines
(scipy's connected components, numpy's lexsort) on small inputs.
"""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


@pytest.fixture(scope="module")
def paper():
    with open(GOLDEN) as f:
        return json.load(f)


def two_body(oracle_mod, s0, s1, r, L=100.0, axis=0, x0=30.0):
    pos = np.full((2, 3), 50.0)
    pos[0, axis] = x0
    pos[1, axis] = x0 + r
    sp = np.array([s0, s1], np.uint8)
    f, e = oracle_mod.forces(pos, sp, L)
    return f, e.sum()


# ------------------------------------------------------------ constants ----
def test_constants_match_table_I(oracle_mod, paper):
    t = paper["table_I"]
    P = oracle_mod.PAPER
    assert (P["a"], P["b"], P["c"], P["Lambda"]) == (t["a_MeV"], t["b_MeV"], t["c_MeV"], t["Lambda_fm2"])
    assert P["mass"] == paper["mass_MeV"]["value"]
    assert P["lambda_s"] == paper["screening_length_fm"]["value"]
    assert P["r_nuc"] == paper["nuclear_cutoff_fm"]["value"]
    assert math.isinf(P["r_coul"]) and paper["coulomb_cutoff"]["value"] is None
    assert abs(P["alpha_hbarc"] - 1.4399645) < 1e-7


# ------------------------------------------------ two-body closed forms ----
@pytest.mark.parametrize("kind", ["np", "nn"])
def test_two_body_minimum(oracle_mod, paper, kind):
    """V = a g^2 + B g with g = exp(-r^2/2Lambda); dV/dg = 0 gives
    g* = -B/(2a), r*^2 = -2 Lambda ln g*, V* = -B^2/(4a); F(r*) = 0."""
    t = paper["table_I"]
    a, b, c, Lam = t["a_MeV"], t["b_MeV"], t["c_MeV"], t["Lambda_fm2"]
    B = b - c if kind == "np" else b + c
    gs = -B / (2 * a)
    rs = math.sqrt(-2 * Lam * math.log(gs))
    Vs = -B * B / (4 * a)
    s0, s1 = (0, 1) if kind == "np" else (0, 0)
    f, e = two_body(oracle_mod, s0, s1, rs)
    assert e == pytest.approx(Vs, rel=1e-13)
    assert abs(f[0, 0]) < 1e-12 and abs(f[1, 0]) < 1e-12
    # known values: 1.92458 fm / -5.681818 MeV (n-p), 3.42800 fm / -0.0090909 MeV (like)
    if kind == "np":
        assert rs == pytest.approx(1.92458, abs=1e-5) and Vs == pytest.approx(-5.681818, abs=1e-6)
    else:
        assert rs == pytest.approx(3.42800, abs=1e-5) and Vs == pytest.approx(-0.0090909, abs=1e-7)
    # slightly inside r* the pair repels, slightly outside it attracts
    f_in, _ = two_body(oracle_mod, s0, s1, rs - 0.01)
    f_out, _ = two_body(oracle_mod, s0, s1, rs + 0.01)
    assert f_in[0, 0] < 0 < f_out[0, 0]  # particle 0 sits at lower x


def test_contact_limits(oracle_mod, paper):
    """V(0) = a + b - c = 60 MeV for n-p and a + b + c = 108 MeV for n-n."""
    _, e_np = two_body(oracle_mod, 0, 1, 1e-7)
    _, e_nn = two_body(oracle_mod, 0, 0, 1e-7)
    assert e_np == pytest.approx(60.0, abs=1e-9)
    assert e_nn == pytest.approx(108.0, abs=1e-9)
    # a proton and a neutron in contact feel no Coulomb term: symmetric in species
    _, e_pn = two_body(oracle_mod, 1, 0, 1e-7)
    assert e_pn == e_np


def test_nuclear_cutoff_strict(oracle_mod):
    """Nuclear term zero and not computed at or beyond 11.5 fm (n-n pair)."""
    _, e_in = two_body(oracle_mod, 0, 0, 11.5 - 1e-9)
    _, e_at = two_body(oracle_mod, 0, 0, 11.5)
    _, e_out = two_body(oracle_mod, 0, 0, 11.6)
    assert e_in != 0.0
    assert e_at == 0.0 and e_out == 0.0


def test_screened_coulomb_constants(oracle_mod, paper):
    """Beyond the nuclear cutoff a p-p pair carries only the screened Coulomb
    term V = alpha_hbarc e^{-r/lambda}/r: r V(r) at two distances recovers
    lambda = 10 fm and alpha hbar c = 1.4399645 MeV fm."""
    r1, r2 = 12.0, 31.0
    _, v1 = two_body(oracle_mod, 1, 1, r1)
    _, v2 = two_body(oracle_mod, 1, 1, r2)
    lam = (r2 - r1) / math.log((r1 * v1) / (r2 * v2))
    assert lam == pytest.approx(paper["screening_length_fm"]["value"], rel=1e-12)
    assert r1 * v1 * math.exp(r1 / lam) == pytest.approx(1.4399645, rel=1e-7)
    # a neutron-proton pair at the same distance feels nothing
    _, v_np = two_body(oracle_mod, 0, 1, r1)
    assert v_np == 0.0


def test_coulomb_cutoff_option(oracle_mod):
    """The optional Coulomb cutoff r_coul (not in the paper, whose Coulomb term
    is uncut): a proton pair at r < r_coul carries the full screened Coulomb
    force and energy (closed form, no shift), one at r = r_coul exactly or
    beyond carries nothing; pair counts follow."""
    L, rc = 100.0, 20.0
    params = dict(r_coul=rc)
    for r, inside in ((19.5, True), (20.0, False), (20.5, False)):
        pos = np.full((2, 3), 50.0)
        pos[0, 0], pos[1, 0] = 30.0, 30.0 + r
        sp = np.array([1, 1], np.uint8)
        f, e = oracle_mod.forces(pos, sp, L, params=params)
        nn, nc = oracle_mod.pair_counts(pos, sp, L, params=params)
        assert nn == 0 and nc == (1 if inside else 0)
        if inside:
            v = 1.4399645 * math.exp(-r / 10.0) / r
            fmag = v * (1.0 / r + 1.0 / 10.0) / r * r   # |F| = -dV/dr
            assert e.sum() == pytest.approx(v, rel=1e-7)
            # the pair repels: particle 0 (lower x) is pushed to -x
            assert f[0, 0] == pytest.approx(-fmag, rel=1e-7) and f[1, 0] == -f[0, 0]
        else:
            assert np.all(f == 0.0) and e.sum() == 0.0
    # uncut by default: the same pair at 20.5 fm interacts
    pos = np.array([[30.0, 50.0, 50.0], [50.5, 50.0, 50.0]])
    f, e = oracle_mod.forces(pos, np.array([1, 1], np.uint8), L)
    assert e.sum() > 0.0 and f[0, 0] < 0.0


def test_periodic_face(oracle_mod):
    """x = 1 and x = L - 1 interact as a pair 2 fm apart (nearest image)."""
    L = 40.0
    f_wrap, e_wrap = two_body(oracle_mod, 0, 1, L - 2.0, L=L, x0=1.0)
    f_dir, e_dir = two_body(oracle_mod, 0, 1, 2.0, L=L, x0=19.0)
    assert e_wrap == pytest.approx(e_dir, rel=1e-14)
    # across the face particle 0 (x=1) has its partner at lower x (image at -1)
    assert f_wrap[0, 0] == pytest.approx(-f_dir[0, 0], rel=1e-12)


# ------------------------------------------------------- many-body pins ----
def random_system(n, L, yp, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.random((n, 3)) * L
    sp = np.zeros(n, np.uint8)
    sp[: int(round(yp * n))] = 1
    # keep pairs further apart than 0.6 fm so the finite-difference test is
    # well conditioned
    for i in range(n):
        for _ in range(100):
            d = pos[:i] - pos[i]
            d -= L * np.round(d / L)
            if i == 0 or (np.sum(d * d, axis=1).min() > 0.36):
                break
            pos[i] = rng.random(3) * L
    return pos, sp


def total_energy(oracle_mod, pos, sp, L):
    return oracle_mod.forces(pos, sp, L)[1].sum()


def test_force_is_minus_gradient(oracle_mod):
    """F = -dE/dx by 4-point central differences (error O(h^4))."""
    L = 26.0
    pos, sp = random_system(40, L, 0.4, 7)
    f, _ = oracle_mod.forces(pos, sp, L)
    h = 1e-3
    rng = np.random.Generator(np.random.PCG64(3))
    checked = 0
    for i in rng.choice(40, 12, replace=False):
        for a in range(3):
            vals = []
            for s in (-2, -1, 1, 2):
                p = pos.copy()
                p[i, a] = (p[i, a] + s * h) % L
                vals.append(total_energy(oracle_mod, p, sp, L))
            grad = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
            scale = max(abs(f[i, a]), 1e-2)
            assert abs(-grad - f[i, a]) / scale < 1e-7, (i, a, -grad, f[i, a])
            checked += 1
    assert checked == 36


def test_newton_third_law(oracle_mod):
    L = 30.0
    pos, sp = random_system(300, L, 0.3, 11)
    f, _ = oracle_mod.forces(pos, sp, L)
    scale = np.abs(f).sum()
    assert np.abs(f.sum(axis=0)).max() <= 1e-13 * scale


@pytest.mark.parametrize("species", [0, 1])
def test_cubic_lattice_is_force_free(oracle_mod, species):
    """A simple cubic lattice with an odd number of sites per side is
    inversion symmetric about every site (no pair sits exactly at L/2)."""
    k, a = 7, 3.5
    g = (np.arange(k) + 0.25) * a
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    sp = np.full(len(pos), species, np.uint8)
    f, e = oracle_mod.forces(pos, sp, k * a)
    assert np.abs(f).max() < 1e-12
    assert np.ptp(e) < 1e-12 * max(1.0, np.abs(e).max())


def test_translation_and_permutation(oracle_mod):
    L = 28.0
    pos, sp = random_system(120, L, 0.4, 5)
    f, e = oracle_mod.forces(pos, sp, L)
    shift = np.array([7.3, -13.1, 25.9])
    f2, e2 = oracle_mod.forces((pos + shift) % L, sp, L)
    assert np.abs(f2 - f).max() < 1e-10 * np.abs(f).max()
    assert abs(e2.sum() - e.sum()) < 1e-11 * np.abs(e).sum()
    perm = np.random.Generator(np.random.PCG64(1)).permutation(len(pos))
    f3, e3 = oracle_mod.forces(pos[perm], sp[perm], L)
    assert np.abs(f3 - f[perm]).max() < 1e-12 * np.abs(f).max()


def test_targets_subset_and_thread_independence(oracle_mod):
    L = 30.0
    pos, sp = random_system(200, L, 0.4, 9)
    f1, e1 = oracle_mod.forces(pos, sp, L, nthreads=1)
    f4, e4 = oracle_mod.forces(pos, sp, L, nthreads=4)
    assert np.array_equal(f1, f4) and np.array_equal(e1, e4)
    t = np.array([5, 0, 199, 77])
    ft, et = oracle_mod.forces(pos, sp, L, targets=t)
    assert np.array_equal(ft, f1[t]) and np.array_equal(et, e1[t])
    # the two terms add up to the total
    fn, en = oracle_mod.forces(pos, sp, L, terms=1)
    fc, ec = oracle_mod.forces(pos, sp, L, terms=2)
    assert np.allclose(fn + fc, f1, rtol=0, atol=1e-12 * np.abs(f1).max())
    assert np.all(fc[sp == 0] == 0)


def test_pair_counts(oracle_mod):
    """Coulomb pairs are all Z(Z-1)/2 (uncut); nuclear pairs in a uniform
    random box follow N(N-1)/2 * (4 pi/3) r^3 / L^3 within a few sigma."""
    n, L, yp = 2000, 45.0, 0.3
    rng = np.random.Generator(np.random.PCG64(4))
    pos = rng.random((n, 3)) * L
    sp = np.zeros(n, np.uint8)
    sp[:600] = 1
    nn, nc = oracle_mod.pair_counts(pos, sp, L)
    assert nc == 600 * 599 // 2
    p = (4 * math.pi / 3) * 11.5 ** 3 / L ** 3
    mean = n * (n - 1) / 2 * p
    assert abs(nn - mean) < 5 * math.sqrt(mean * 40)  # pairs are correlated: generous sigma


# -------------------------------------------------------------- integrator --
def test_free_particle(oracle_mod):
    pos = np.array([[1.0, 2.0, 3.0]])
    vel = np.array([[0.05, -0.07, 0.11]])
    L = 30.0
    p, v, Lf, ek, ep, f = oracle_mod.run(pos, vel, np.array([0], np.uint8), L, 500, dt=2.0)
    expect = (pos + 1000.0 * vel) % L
    assert np.abs(p - expect).max() < 1e-10
    assert np.array_equal(v, vel) and ep == 0.0 and Lf == L


def test_box_law_density_endpoints(oracle_mod, paper):
    """Eq. (3): after t = 3e7 fm/c at xi_dot = 1e-7 the side is 4 l(0), i.e.
    0.08 -> 0.00125 fm^-3; after t = 1/xi_dot, 0.08 -> 0.01 fm^-3."""
    pr = paper["production_run"]
    L0 = 86.17738760127535
    L = oracle_mod.box_length(L0, pr["xi_dot_c_per_fm"], pr["dt_fm_c"], pr["steps"])
    assert (L0 / L) ** 3 * pr["n_start"] == pytest.approx(pr["n_end"], rel=1e-12)
    ex = paper["expansion_study"]
    for xi in (1e-5, 1e-6, 1e-7, 1e-8):
        steps = int(round(1.0 / xi / 2.0))
        L = oracle_mod.box_length(L0, xi, 2.0, steps)
        assert (L0 / L) ** 3 * ex["n_start"] == pytest.approx(ex["n_end"], rel=1e-12)


def test_expansion_does_not_move_particles(oracle_mod):
    """Positions are not rescaled with the box (Sec. II.A); the affine variant
    scales them by L_{n+1}/L_n."""
    pos = np.array([[10.0, 20.0, 30.0], [60.0, 70.0, 80.0]])
    vel = np.zeros_like(pos)
    sp = np.array([0, 0], np.uint8)
    L0 = 100.0
    p, _, Lf, *_ = oracle_mod.run(pos, vel, sp, L0, 10, dt=2.0, xi_dot=0.05)
    assert Lf == pytest.approx(L0 * (1 + 0.05 * 20), rel=1e-15)
    assert np.array_equal(p, pos)
    p2, *_ = oracle_mod.run(pos, vel, sp, L0, 10, dt=2.0, xi_dot=0.05, scale_positions=True)
    assert np.allclose(p2, pos * 2.0, rtol=1e-14)


def test_thermostat(oracle_mod):
    L = 30.0
    pos, sp = random_system(100, L, 0.3, 21)
    vel = np.random.Generator(np.random.PCG64(2)).standard_normal((100, 3)) * 0.05
    p, v, Lf, ek, ep, f = oracle_mod.run(pos, vel, sp, L, 10, dt=1.0, T=0.8, rescale_every=5)
    assert ek == pytest.approx(1.5 * 100 * 0.8, rel=1e-14)
    assert np.all((p >= 0) & (p < L))
    # a run ending off the rescale grid does not land on 1.5 N T
    _, _, _, ek2, *_ = oracle_mod.run(pos, vel, sp, L, 7, dt=1.0, T=0.8, rescale_every=5)
    assert abs(ek2 - 120.0) > 1e-6


def test_np_pair_oscillation_period(oracle_mod, paper):
    """A bound n-p pair oscillates about r* with omega^2 = V''(r*)/mu,
    mu = M/2 and V''(r*) = 2a (r* g*/Lambda)^2 (from V = a g^2 + B g)."""
    t = paper["table_I"]
    a, b, c, Lam = t["a_MeV"], t["b_MeV"], t["c_MeV"], t["Lambda_fm2"]
    M = paper["mass_MeV"]["value"]
    gs = (c - b) / (2 * a)
    rs = math.sqrt(-2 * Lam * math.log(gs))
    omega = math.sqrt(2 * a * (rs * gs / Lam) ** 2 / (M / 2))
    period = 2 * math.pi / omega
    amp = 0.01
    pos = np.array([[20.0, 25.0, 25.0], [20.0 + rs + amp, 25.0, 25.0]])
    vel = np.zeros_like(pos)
    sp = np.array([0, 1], np.uint8)
    dt = 0.05
    xs = []
    p, v = pos, vel
    for _ in range(int(4 * period / dt) + 10):
        p, v, *_ = oracle_mod.run(p, v, sp, 50.0, 1, dt=dt)
        xs.append(p[1, 0] - p[0, 0] - rs)
    xs = np.array(xs)
    cross = np.where((xs[:-1] > 0) & (xs[1:] <= 0))[0]
    # linear interpolation of the downward zero crossings
    tc = [(k + xs[k] / (xs[k] - xs[k + 1])) * dt for k in cross]
    meas = np.diff(tc).mean()
    assert meas == pytest.approx(period, rel=2e-3)


def nve_error(oracle_mod, pos, vel, sp, L, dt, t_end):
    e0 = oracle_mod.kinetic(vel) + total_energy(oracle_mod, pos, sp, L)
    err = 0.0
    p, v = pos, vel
    nsub = int(round(t_end / dt / 10))
    for _ in range(10):
        p, v, _, ek, ep, _ = oracle_mod.run(p, v, sp, L, nsub, dt=dt)
        err = max(err, abs(ek + ep - e0))
    return err


def test_verlet_energy_error_scales_as_dt_squared(oracle_mod):
    L = 24.0
    pos, sp = random_system(60, L, 0.3, 31)
    vel = np.random.Generator(np.random.PCG64(8)).standard_normal((60, 3)) * 0.02
    e1 = nve_error(oracle_mod, pos, vel, sp, L, 0.5, 20.0)
    e2 = nve_error(oracle_mod, pos, vel, sp, L, 0.25, 20.0)
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)


def test_time_reversibility(oracle_mod):
    L = 25.0
    pos, sp = random_system(64, L, 0.3, 41)
    vel = np.random.Generator(np.random.PCG64(9)).standard_normal((64, 3)) * 0.03
    p, v, *_ = oracle_mod.run(pos, vel, sp, L, 40, dt=1.0)
    p2, v2, *_ = oracle_mod.run(p, -v, sp, L, 40, dt=1.0)
    d = p2 - pos
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-8
    assert np.abs(v2 + vel).max() < 1e-9


# ---------------------------------------------------------------- clusters --
def test_chain_across_face(oracle_mod):
    L = 9 * 4.49
    n = 9
    for spacing, expect in ((4.49, 1), (4.51, 9)):
        L = n * spacing
        pos = np.zeros((n, 3))
        pos[:, 0] = (np.arange(n) * spacing + 0.3 * spacing) % L
        pos[:, 1:] = 5.0
        # L < 2 * 11.5 is fine for the cluster algorithm alone
        cl = oracle_mod.cluster(pos, np.ones(n, np.uint8), L)
        assert cl["nclusters"] == expect
        if expect == 1:
            assert np.all(cl["label"] == 0)
        else:
            assert np.array_equal(cl["label"], np.arange(n))


def test_link_radius_inclusive(oracle_mod):
    """'Within' r_pp and r_np is read as inclusive: a proton pair exactly
    4.5 fm apart is one cluster, a neutron exactly 3 fm away is bound
    (both squares, 20.25 and 9, are exact in binary)."""
    pos = np.array([[10.0, 20, 20], [14.5, 20, 20], [14.5, 23.0, 20]])
    sp = np.array([1, 1, 0], np.uint8)
    cl = oracle_mod.cluster(pos, sp, 50.0)
    assert cl["nclusters"] == 1 and list(cl["label"]) == [0, 0, 0]


def test_neutron_radius_and_tie(oracle_mod):
    L = 60.0
    # two protons 6 fm apart (separate clusters); neutron exactly 3 fm from both
    pos = np.array([[16.0, 30, 30], [10.0, 30, 30], [13.0, 30, 30],
                    [40.0, 30, 30], [42.99, 30, 30], [40.0, 33.01, 30]])
    sp = np.array([1, 1, 0, 1, 0, 0], np.uint8)
    cl = oracle_mod.cluster(pos, sp, L)
    lab = cl["label"]
    assert cl["nclusters"] == 3
    # protons numbered by smallest index: p0 -> 0, p1 -> 1, p3 -> 2
    assert list(lab[[0, 1, 3]]) == [0, 1, 2]
    assert lab[2] == 0          # tie -> lower proton index (p0)
    assert lab[4] == 2          # 2.99 fm from p3: bound
    assert lab[5] == -1         # 3.01 fm: free
    assert cl["nfree"] == 1
    assert cl["hist_A"][2] == 2 and cl["hist_A"][1] == 1
    assert cl["hist_Z"][1] == 3


def test_clusters_against_scipy(oracle_mod):
    """Proton clusters = connected components (scipy) of the r <= 4.5 graph;
    neutrons take the label of their nearest proton within 3 fm (argmin keeps
    the first, i.e. lowest, index on ties)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.Generator(np.random.PCG64(12))
    n, L = 600, 40.0
    pos = rng.random((n, 3)) * L
    sp = (rng.random(n) < 0.35).astype(np.uint8)
    d = pos[:, None, :] - pos[None, :, :]
    d = np.where(d > L / 2, d - L, np.where(d < -L / 2, d + L, d))
    r2 = (d[..., 0] ** 2 + d[..., 1] ** 2) + d[..., 2] ** 2
    p_idx = np.nonzero(sp == 1)[0]
    adj = (r2[np.ix_(p_idx, p_idx)] <= 20.25)
    ncomp, comp = connected_components(csr_matrix(adj), directed=False)
    # canonical: components ordered by their smallest proton index
    first = np.full(ncomp, n)
    for k, c in enumerate(comp):
        first[c] = min(first[c], p_idx[k])
    order = np.argsort(first)
    rank = np.empty(ncomp, int)
    rank[order] = np.arange(ncomp)
    expect = np.full(n, -1)
    expect[p_idx] = rank[comp]
    n_idx = np.nonzero(sp == 0)[0]
    dn = r2[np.ix_(n_idx, p_idx)]
    near = np.argmin(np.where(dn <= 9.0, dn, np.inf), axis=1)
    ok = dn[np.arange(len(n_idx)), near] <= 9.0
    expect[n_idx[ok]] = expect[p_idx[near[ok]]]
    cl = oracle_mod.cluster(pos, sp, L)
    assert cl["nclusters"] == ncomp
    assert np.array_equal(cl["label"], expect)
    A = np.bincount(expect[expect >= 0], minlength=ncomp)
    assert np.array_equal(cl["hist_A"][: A.max() + 1], np.bincount(A))
    assert cl["hist_A"].sum() == ncomp and cl["nfree"] == int((~ok).sum())
    assert (np.arange(n + 1) * cl["hist_Z"]).sum() == int(sp.sum())
    assert (np.arange(n + 1) * cl["hist_A"]).sum() + cl["nfree"] == n


def test_cluster_permutation_invariance(oracle_mod):
    rng = np.random.Generator(np.random.PCG64(13))
    n, L = 400, 30.0
    pos = rng.random((n, 3)) * L
    sp = (rng.random(n) < 0.4).astype(np.uint8)
    a = oracle_mod.cluster(pos, sp, L)
    perm = rng.permutation(n)
    b = oracle_mod.cluster(pos[perm], sp[perm], L)
    assert np.array_equal(a["hist_A"], b["hist_A"]) and np.array_equal(a["hist_Z"], b["hist_Z"])
    # same partition: pairs share a label in one iff they do in the other
    la, lb = a["label"][perm], b["label"]
    m = la >= 0
    assert np.array_equal(m, lb >= 0)
    pairs_a = la[m][:, None] == la[m][None, :]
    pairs_b = lb[m][:, None] == lb[m][None, :]
    assert np.array_equal(pairs_a, pairs_b)


# --------------------------------------------------------------- cell list --
def test_cell_list_definition(oracle_mod):
    rng = np.random.Generator(np.random.PCG64(14))
    n, L, rc = 5000, 86.17738760127535, 11.5
    pos = rng.random((n, 3)) * L
    sp = (rng.random(n) < 0.2).astype(np.uint8)
    nc, start, perm = oracle_mod.cell_list(pos, sp, L, rc)
    assert nc == 7 and L / nc >= rc and L / (nc + 1) < rc
    C = nc ** 3
    assert np.array_equal(np.sort(perm), np.arange(n))
    c3 = np.minimum((pos * (nc / L)).astype(np.int64), nc - 1)
    cell = (c3[:, 2] * nc + c3[:, 1]) * nc + c3[:, 0]
    binv = np.where(sp == 1, 0, C) + cell
    expect = np.lexsort((np.arange(n), binv))
    assert np.array_equal(perm, expect)
    assert start[0] == 0 and start[-1] == n and len(start) == 2 * C + 1
    assert np.array_equal(np.diff(start), np.bincount(binv, minlength=2 * C))
    # every particle lies inside its cell
    w = L / nc
    lo = c3 * w
    assert np.all(pos >= lo - 1e-12) and np.all(pos < lo + w + 1e-12)
    assert oracle_mod.cell_dims(43.0887, 11.5) == 3 and oracle_mod.cell_dims(23.0, 11.5) == 2


def test_cell_list_hand_placed(oracle_mod):
    """Particles placed at known cells of a 3 x 3 x 3 grid (L = 34.5 fm,
    cells of exactly 11.5 fm): the linear cell index is (cz*3 + cy)*3 + cx,
    protons fill bins 0..26 and neutrons 27..53, and within a bin the order
    is the particle index.  Written out by hand, not from a formula."""
    w = 11.5
    L = 3 * w

    def centre(cx, cy, cz):
        return [(cx + 0.5) * w, (cy + 0.5) * w, (cz + 0.5) * w]

    pos = np.array([centre(0, 0, 0),          # 0 neutron -> bin 27
                    centre(2, 0, 1),          # 1 proton  -> bin 11
                    centre(0, 2, 0),          # 2 proton  -> bin 6
                    centre(0, 0, 2),          # 3 proton  -> bin 18
                    centre(2, 2, 2),          # 4 neutron -> bin 53
                    [1.0, 2 * w + 0.5, 3.0],  # 5 proton  -> bin 6
                    [L - 0.01, L - 0.01, L - 0.01]])  # 6 neutron -> bin 53
    sp = np.array([0, 1, 1, 1, 0, 1, 0], np.uint8)
    nc, start, perm = oracle_mod.cell_list(pos, sp, L, 11.5)
    assert nc == 3
    assert list(perm) == [2, 5, 1, 3, 0, 4, 6]
    expect_start = np.zeros(55, np.int64)
    counts = {6: 2, 11: 1, 18: 1, 27: 1, 53: 2}
    for b in range(54):
        expect_start[b + 1] = expect_start[b] + counts.get(b, 0)
    assert np.array_equal(start, expect_start)


def test_cell_list_structure(oracle_mod):
    """Properties of the sorted order that any correct cell list has, checked
    without the binning formula: protons before neutrons, particle indices
    increasing within a bin, every particle inside its bin's cell, and the
    bins' members exactly the particles inside that cell."""
    rng = np.random.Generator(np.random.PCG64(15))
    n, L, rc = 4000, 50.0, 11.5
    pos = rng.random((n, 3)) * L
    sp = (rng.random(n) < 0.3).astype(np.uint8)
    nc, start, perm = oracle_mod.cell_list(pos, sp, L, rc)
    C, w = nc ** 3, L / nc
    Zc = int(sp.sum())
    assert np.all(sp[perm[:Zc]] == 1) and np.all(sp[perm[Zc:]] == 0)
    assert start[C] == Zc
    for b in range(2 * C):
        members = perm[start[b]:start[b + 1]]
        assert np.all(np.diff(members) > 0)
        c = b % C
        cx, cy, cz = c % nc, (c // nc) % nc, c // (nc * nc)
        lo = np.array([cx, cy, cz]) * w
        inside = np.all((pos >= lo - 1e-12) & (pos < lo + w + 1e-12), axis=1)
        inside &= (sp == 1) if b < C else (sp == 0)
        assert np.array_equal(np.sort(np.nonzero(inside)[0]), members)


def test_cluster_stats_hand_built(oracle_mod):
    """Table II statistics from a cluster result whose numbers are worked out
    by hand: clusters of A = 12 (Z = 4), 20 (Z = 8) and 3 (Z = 1, light),
    5 free neutrons, N = 40.  Free-neutron mass fraction 5/40; over A >= 12:
    mean A 16 and population SD 4 (the sample SD would be 5.657), mean Z 6
    and SD 2.  A cluster of A = 11 is left out, one of A = 12 is kept."""
    label = np.array([0] * 12 + [1] * 20 + [2] * 3 + [-1] * 5, np.int32)
    species = np.zeros(40, np.uint8)
    species[[0, 1, 2, 3]] = 1
    species[12:20] = 1
    species[32] = 1
    cl = dict(label=label, nclusters=3, nfree=5)
    s = oracle_mod.cluster_stats(cl, species)
    assert s["x_free"] == 0.125 and s["nclusters"] == 3 and s["n_heavy"] == 2
    assert s["A_mean"] == 16.0 and s["A_std"] == 4.0
    assert s["Z_mean"] == 6.0 and s["Z_std"] == 2.0
    # the A >= 12 boundary: an 11-nucleon cluster is excluded
    label2 = np.array([0] * 11 + [1] * 12 + [-1] * 2, np.int32)
    sp2 = np.zeros(25, np.uint8)
    sp2[[0, 11, 12, 13]] = 1
    s2 = oracle_mod.cluster_stats(dict(label=label2, nclusters=2, nfree=2), sp2)
    assert s2["n_heavy"] == 1 and s2["A_mean"] == 12.0 and s2["A_std"] == 0.0
    assert s2["Z_mean"] == 3.0 and s2["x_free"] == 2 / 25
    # no heavy cluster: only the free fraction and counts
    s3 = oracle_mod.cluster_stats(dict(label=np.array([0, 0, -1], np.int32), nclusters=1,
                                       nfree=1), np.array([1, 0, 0], np.uint8))
    assert s3["n_heavy"] == 0 and "A_mean" not in s3 and s3["x_free"] == 1 / 3


def test_cluster_stats_on_hand_built_positions(oracle_mod):
    """End to end through the cluster algorithm: a chain of 3 protons 4 fm
    apart with 9 neutrons each 2 fm from one of them (A = 12, Z = 3), an
    isolated proton with one neutron 2.5 fm away (A = 2, light), and two
    neutrons far from every proton (free).  N = 16: free fraction 2/16,
    one heavy cluster with A = 12, Z = 3 (SD 0)."""
    L = 60.0
    pos, sp = [], []
    for k in range(3):
        pos.append([10.0 + 4.0 * k, 10.0, 10.0])
        sp.append(1)
    for k in range(3):
        for d in ([0, 2.0, 0], [0, -2.0, 0], [0, 0, 2.0]):
            pos.append([10.0 + 4.0 * k + d[0], 10.0 + d[1], 10.0 + d[2]])
            sp.append(0)
    pos += [[40.0, 40.0, 40.0], [42.5, 40.0, 40.0], [25.0, 45.0, 5.0], [50.0, 20.0, 30.0]]
    sp += [1, 0, 0, 0]
    pos, sp = np.array(pos), np.array(sp, np.uint8)
    cl = oracle_mod.cluster(pos, sp, L)
    assert cl["nclusters"] == 2 and cl["nfree"] == 2
    s = oracle_mod.cluster_stats(cl, sp)
    assert s["x_free"] == 2 / 16 and s["n_heavy"] == 1
    assert s["A_mean"] == 12.0 and s["Z_mean"] == 3.0 and s["A_std"] == 0.0
