"""Host-side logic that needs no GPU: the seeded input generator, the
autotuner's shape key and cache, and the batch grid recipe."""
import json
import os

import numpy as np
import pytest


def test_make_state_recipe():
    from paper_1412_8502_amd.inputs import make_state, box_side
    st = make_state(3200, 0.40, 0.040, 1.0, seed=1000)
    assert st["L"] == pytest.approx((3200 / 0.04) ** (1 / 3), rel=1e-15)
    assert st["pos"].shape == (3200, 3) and st["pos"].dtype == np.float64
    assert np.all((st["pos"] >= 0) & (st["pos"] < st["L"]))
    assert st["Z"] == 1280 and st["species"][:1280].all() and not st["species"][1280:].any()
    # Maxwell-Boltzmann: each component has variance T/M
    assert st["vel"].var() == pytest.approx(1.0 / 939.0, rel=0.05)
    again = make_state(3200, 0.40, 0.040, 1.0, seed=1000)
    assert np.array_equal(st["pos"], again["pos"]) and np.array_equal(st["vel"], again["vel"])
    assert box_side(51200, 0.08) == pytest.approx(86.17738760127535, rel=1e-14)


def test_batch_grid_recipe():
    from paper_1412_8502_amd.inputs import batch_grid
    g = batch_grid()
    assert len(g) == 15
    assert sorted({(s["y_p"], s["T"]) for s in g}) == sorted(
        (yp, T) for yp in (0.05, 0.10, 0.20, 0.30, 0.40) for T in (0.5, 0.75, 1.0))
    for s in g:
        assert s["n"] in (6400, 12800, 25600, 51200)
        assert 0.02 <= s["density"] <= 0.08
        assert s["L"] >= 2 * 11.5


def test_autotune_shape_key_and_cache(tmp_path, monkeypatch):
    pytest.importorskip("torch")
    from paper_1412_8502_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_1412_8502_amd import autotune
    monkeypatch.setenv("PASTA_TUNING_CACHE", str(tmp_path / "c" / "t.json"))
    k1 = autotune.shape_key(51200, 10240, 86.17738760127535, 1)
    k2 = autotune.shape_key(51000, 10200, 86.1, 1)
    assert k1 == k2 == "p1_n65536_d0.08_y0.20"
    assert autotune.shape_key(51200, 10240, 86.17738760127535, 0) != k1
    path = autotune.cache_path()
    autotune._store_cache(path, {k1: {"best": {"nuclear_variant": 1, "coulomb_splits": 8}}})
    with open(path) as f:
        assert json.load(f)[k1]["best"]["coulomb_splits"] == 8


def _fp64math(tmp_path_factory):
    import ctypes
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    out = str(tmp_path_factory.mktemp("fp64math") / "libfp64math.so")
    subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-o", out,
                           os.path.join(here, "fp64math_host.cpp")])
    lib = ctypes.CDLL(out)
    lib.host_exp_nonpos.restype = ctypes.c_double
    lib.host_exp_nonpos.argtypes = [ctypes.c_double]
    lib.host_rsqrt_refine.restype = ctypes.c_double
    lib.host_rsqrt_refine.argtypes = [ctypes.c_double, ctypes.c_double]
    return lib


def test_fp64_exp_accuracy(tmp_path_factory):
    """The kernels' FP64 exp (Cody-Waite + Taylor) within 2 ulp of libm on
    the range the potentials use, and exact at 0."""
    import math
    lib = _fp64math(tmp_path_factory)
    rng = np.random.Generator(np.random.PCG64(5))
    xs = np.concatenate([-rng.random(20000) * 60.0, -rng.random(2000) * 700.0,
                         [0.0, -1e-300, -0.5 * math.log(2), -math.log(2), -52.9, -700.0]])
    worst = 0.0
    for x in xs:
        got, ref = lib.host_exp_nonpos(float(x)), math.exp(float(x))
        worst = max(worst, abs(got - ref) / math.ulp(ref))
    assert worst <= 2.0, worst
    assert lib.host_exp_nonpos(0.0) == 1.0


def test_fp64_rsqrt_refinement(tmp_path_factory):
    """Two Newton steps take a single-precision-quality estimate to full
    double precision (within 2 ulp of 1/sqrt)."""
    import math
    lib = _fp64math(tmp_path_factory)
    rng = np.random.Generator(np.random.PCG64(6))
    xs = np.exp(rng.uniform(-20, 20, 20000))
    worst = 0.0
    for x in xs:
        y0 = float(np.float32(1.0 / math.sqrt(x)))  # a coarse estimate
        got = lib.host_rsqrt_refine(float(x), y0)
        ref = 1.0 / math.sqrt(x)
        worst = max(worst, abs(got - ref) / math.ulp(ref))
    assert worst <= 2.0, worst


def _min_image(d, L):
    return d - L * np.round(d / L)


@pytest.mark.parametrize("scale_positions", [False, True])
def test_list_rebuild_bound(scale_positions):
    """The rebuild rule of the neighbour-list form: if every nearest-image
    displacement u_i since the build (measured in the current box) satisfies
    2 max|u| + sqrt(3) |L - L_b| < delta_r, then every pair inside r_nuc now
    was inside r_nuc + delta_r at the build.  Brute force over random
    configurations with particles near the faces, random moves of bounded
    length, wraps, and box growth or shrinkage (with and without the affine
    variant)."""
    rng = np.random.Generator(np.random.PCG64(2024))
    r_nuc = 11.5
    worst = -np.inf
    for trial in range(60):
        n = 300
        Lb = rng.uniform(23.5, 40.0)
        yb = rng.uniform(0, Lb, (n, 3))
        yb[: n // 4] = np.mod(rng.normal(0, 0.3, (n // 4, 3)), Lb)  # crowd a corner
        dL = rng.uniform(-0.4, 0.6)
        L = Lb + dL
        dmax = rng.uniform(0.05, 1.5)
        step = rng.normal(size=(n, 3))
        step *= (rng.uniform(0, 1, (n, 1)) * dmax) / np.linalg.norm(step, axis=1, keepdims=True)
        y = yb + step
        if scale_positions:
            y *= L / Lb
        y = np.mod(y, L)
        # displacement as the drift kernel measures it, in the current box
        u = _min_image(y - yb, L)
        umax = np.sqrt((u * u).sum(axis=1)).max()
        bound = 2 * umax + np.sqrt(3.0) * abs(L - Lb)
        d_now = _min_image(y[:, None, :] - y[None, :, :], L)
        r_now = np.sqrt((d_now ** 2).sum(-1))
        d_b = _min_image(yb[:, None, :] - yb[None, :, :], Lb)
        r_b = np.sqrt((d_b ** 2).sum(-1))
        close = r_now < r_nuc
        # the claim: r_b <= r_now + bound for every pair (in particular those
        # inside r_nuc now are inside r_nuc + delta_r once bound < delta_r)
        excess = (r_b - r_now - bound)[close]
        worst = max(worst, excess.max())
    assert worst <= 1e-9, worst


def test_expansion_cluster_stats():
    """Table II statistics from labels: free-neutron mass fraction, mean and
    population SD of A and Z over clusters with A >= 12, light clusters."""
    from paper_1412_8502_amd.expansion import cluster_stats
    # cluster 0: 12 nucleons (4 protons); cluster 1: 20 (8 protons);
    # cluster 2: 3 (1 proton, light); 5 free neutrons
    label = np.array([0] * 12 + [1] * 20 + [2] * 3 + [-1] * 5)
    species = np.zeros(40, np.uint8)
    species[[0, 1, 2, 3]] = 1
    species[12:20] = 1
    species[32] = 1
    s = cluster_stats(label, species)
    assert s["clusters"] == 3 and s["clusters_A_ge_12"] == 2
    assert s["mass_fraction_free_neutrons"] == 5 / 40
    assert s["mass_fraction_light_clusters"] == 3 / 40
    assert s["largest_A"] == 20
    assert s["mean_A"] == 16.0 and s["sd_A"] == 4.0
    assert s["mean_Z"] == 6.0 and s["sd_Z"] == 2.0


def test_expansion_checkpoint_roundtrip(tmp_path):
    """A decompression checkpoint keeps the state bit for bit and refuses to
    resume a run with other parameters or a malformed state."""
    from paper_1412_8502_amd.expansion import save_checkpoint, load_checkpoint
    rng = np.random.default_rng(5)
    params = {"n": 7, "yp": 0.3, "T": 1.0, "xi_log10": -7.0, "equil_steps": 500000,
              "seed": 3202, "n0": 0.08, "n_end": 0.01, "dt": 2.0}
    pos, vel = rng.random((7, 3)) * 40.0, rng.standard_normal((7, 3))
    path = tmp_path / "ck.npz"
    save_checkpoint(path, params, 1, 1250000, 612.5, 2, pos, vel)
    ck = load_checkpoint(path, params)
    assert (ck["phase"], ck["done"], ck["seconds"], ck["segments"]) == (1, 1250000, 612.5, 2)
    assert np.array_equal(ck["pos"], pos) and np.array_equal(ck["vel"], vel)
    for k, v in (("seed", 3203), ("yp", 0.2), ("xi_log10", -6.0), ("n", 8)):
        with pytest.raises(ValueError):
            load_checkpoint(path, {**params, k: v})
    save_checkpoint(path, params, 2, 0, 0.0, 1, pos, vel)
    with pytest.raises(ValueError):
        load_checkpoint(path, params)
