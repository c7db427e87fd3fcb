"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/pasta.h declares, and rejects bad arguments before
touching the device."""
import ctypes

import pytest


@pytest.fixture(scope="module")
def B():
    import os
    from paper_1412_8502_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_1412_8502_amd import binding
    return binding


def test_exports_every_declared_function(B):
    names = B.header_functions()
    assert len(names) >= 20
    missing = [f for f in names if not hasattr(B.lib, f)]
    assert missing == []


def test_paper_potential(B):
    p = B.pasta_potential_paper()
    assert (p.a, p.b, p.c, p.Lambda, p.lambda_s, p.mass, p.r_nuc) == \
        (110.0, -26.0, 24.0, 1.25, 10.0, 939.0, 11.5)
    assert p.r_coul == float("inf")  # the paper's Coulomb term is uncut
    assert abs(p.alpha_hbarc - 1.4399645) < 1e-7
    assert "gfx950" in B.pasta_version()


def test_workspace_queries(B):
    p = B.pasta_potential_paper()
    nb = ctypes.c_size_t()
    for prec in (B.PASTA_FP64, B.PASTA_MIXED):
        assert B.lib.pasta_forces_workspace(ctypes.byref(p), prec, 51200, 86.18,
                                            ctypes.byref(nb)) == 0
        assert nb.value > 51200 * 16 and nb.value % 256 == 0
    g = B.pasta_integrator(2.0, 7.5e-5, 0.5, 100, 0)
    small, big = ctypes.c_size_t(), ctypes.c_size_t()
    assert B.lib.pasta_sim_workspace(ctypes.byref(p), ctypes.byref(g), 1, 51200, 86.18, 86.18,
                                     ctypes.byref(small)) == 0
    assert B.lib.pasta_sim_workspace(ctypes.byref(p), ctypes.byref(g), 1, 51200, 86.18, 344.71,
                                     ctypes.byref(big)) == 0
    assert big.value > small.value  # the cell grid grows with L_max
    # the list form adds the list memory, sized by the starting density
    old = B.pasta_set_tuning(nuclear_variant=2, list_skin=2.0)
    try:
        dense, dilute = ctypes.c_size_t(), ctypes.c_size_t()
        assert B.lib.pasta_sim_workspace(ctypes.byref(p), ctypes.byref(g), 1, 51200, 86.18,
                                         344.71, ctypes.byref(dense)) == 0
        assert B.lib.pasta_sim_workspace(ctypes.byref(p), ctypes.byref(g), 1, 51200, 172.4,
                                         344.71, ctypes.byref(dilute)) == 0
        assert dense.value > dilute.value > 0
        assert dense.value > big.value
    finally:
        B.pasta_set_tuning(**old)
    assert B.lib.pasta_cluster_workspace(3200, 43.09, 4.5, 3.0, ctypes.byref(nb)) == 0
    assert B.lib.pasta_cell_list_workspace(3200, 43.09, 11.5, ctypes.byref(nb)) == 0
    # the cell-grid sizing query: the largest ncell with L / ncell >= r_cut
    nc = ctypes.c_int32()
    for L, rc, want in ((43.0887, 11.5, 3), (23.0, 11.5, 2), (86.18, 11.5, 7), (344.71, 11.5, 29),
                        (46.0, 11.5, 4), (45.99, 11.5, 3), (10.0, 11.5, 1)):
        assert B.lib.pasta_cell_dims(L, rc, ctypes.byref(nc)) == 0
        assert nc.value == want, (L, rc, nc.value)
    assert B.lib.pasta_cell_dims(-1.0, 11.5, ctypes.byref(nc)) == -1


def test_argument_errors(B):
    p = B.pasta_potential_paper()
    fake = ctypes.c_void_p(256 * 1024)  # never dereferenced: the calls fail first
    # negative n
    assert B.lib.pasta_forces(ctypes.byref(p), 0, 3, -1, 86.0, fake, fake, fake, None, fake,
                              1 << 30, None) == -1
    # bad precision / terms
    assert B.lib.pasta_forces(ctypes.byref(p), 7, 3, 10, 86.0, fake, fake, fake, None, fake,
                              1 << 30, None) == -1
    assert B.lib.pasta_forces(ctypes.byref(p), 0, 8, 10, 86.0, fake, fake, fake, None, fake,
                              1 << 30, None) == -1
    # box below twice the cutoff: nearest image ambiguous
    assert B.lib.pasta_forces(ctypes.byref(p), 0, 3, 10, 22.9, fake, fake, fake, None, fake,
                              1 << 30, None) == -2
    assert "2 max(r_nuc, r_coul)" in B.lib.pasta_last_error().decode()
    # a finite Coulomb cutoff needs L >= 2 r_coul; NaN or non-positive is refused
    cut = B.pasta_potential_paper()
    cut.r_coul = 20.0
    assert B.lib.pasta_forces(ctypes.byref(cut), 0, 3, 10, 39.9, fake, fake, fake, None, fake,
                              1 << 30, None) == -2
    for v in (float("nan"), 0.0, -5.0):
        cut.r_coul = v
        assert B.lib.pasta_forces(ctypes.byref(cut), 0, 3, 10, 50.0, fake, fake, fake, None,
                                  fake, 1 << 30, None) == -1
    # the batched path takes the uncut Coulomb term only
    cut.r_coul = 20.0
    ns = (ctypes.c_int64 * 1)(1000)
    lm = (ctypes.c_double * 1)(50.0)
    nbb = ctypes.c_size_t()
    assert B.lib.pasta_batch_workspace(ctypes.byref(cut), 1, 1, ns, lm, ctypes.byref(nbb)) == -1
    # workspace too small / misaligned
    assert B.lib.pasta_forces(ctypes.byref(p), 0, 3, 10, 30.0, fake, fake, fake, None, fake,
                              16, None) == -3
    assert B.lib.pasta_forces(ctypes.byref(p), 0, 3, 10, 30.0, fake, fake, fake, None,
                              ctypes.c_void_p(256 * 1024 + 8), 1 << 30, None) == -3
    # non-finite potential parameter
    bad = B.pasta_potential_paper()
    bad.Lambda = float("nan")
    assert B.lib.pasta_forces(ctypes.byref(bad), 0, 3, 10, 30.0, fake, fake, fake, None, fake,
                              1 << 30, None) == -1
    # null handles
    assert B.lib.pasta_sim_step(None, 1) == -1
    assert B.lib.pasta_sim_energies(None, None, None, None, None) == -1
    # cluster: box too small
    K = ctypes.c_int32()
    assert B.lib.pasta_cluster(10, 8.0, fake, fake, 4.5, 3.0, fake, fake, fake,
                               ctypes.byref(K), None, fake, 1 << 30, None) == -2
    # tuning: unknown variant, non-positive halo, unknown Coulomb form
    t = B.pasta_tuning()
    assert B.lib.pasta_get_tuning(ctypes.byref(t)) == 0
    for field, value in (("nuclear_variant", 5), ("list_skin", 0.0), ("list_skin", -1.0),
                         ("batch_wgs_per_cu", 9), ("batch_wgs_per_cu", -1),
                         ("list_pool_scale", 0.0), ("coulomb_form", 3), ("coulomb_form", -1),
                         ("fused_forces", 2),
                         ("nuclear_tile", 128), ("nuclear_tile", 2048), ("nuclear_tile", -1)):
        bad_t = B.pasta_tuning()
        ctypes.pointer(bad_t)[0] = t
        setattr(bad_t, field, value)
        assert B.lib.pasta_set_tuning(ctypes.byref(bad_t)) == -1, field
    cur = B.pasta_tuning()
    assert B.lib.pasta_get_tuning(ctypes.byref(cur)) == 0
    assert B.tuning_dict(cur) == B.tuning_dict(t)
    # the tile lengths the library has kernels for are accepted
    for tile in (0, 256, 512, 1024):
        ok_t = B.pasta_tuning()
        ctypes.pointer(ok_t)[0] = t
        ok_t.nuclear_tile = tile
        assert B.lib.pasta_set_tuning(ctypes.byref(ok_t)) == 0, tile
    assert B.lib.pasta_set_tuning(ctypes.byref(t)) == 0
    # bad integrator
    g = B.pasta_integrator(-1.0, 0.0, 1.0, 0, 0)
    nb = ctypes.c_size_t()
    assert B.lib.pasta_sim_workspace(ctypes.byref(p), ctypes.byref(g), 0, 10, 30.0, 30.0,
                                     ctypes.byref(nb)) == -1


def test_python_binding_rejects_cpu_tensors(B):
    import torch
    pos = torch.zeros((4, 3), dtype=torch.float64)
    sp = torch.zeros(4, dtype=torch.uint8)
    with pytest.raises(ValueError):
        B.pasta_forces(pos, sp, 30.0)
