"""Invariants of the synthetic input generator (no GPU)."""
import numpy as np
import pytest

import synth


def test_config0_shape(cfg0_system):
    s = cfg0_system
    assert (s.m, s.n, s.nx, s.ny, s.nz) == (7800, 2304, 16, 16, 9)
    # depth supports per period 2,4,...,20 s on nodes 0..40 km
    counts = [len(synth.depth_kernel(s.cfg.z_nodes, T)[1]) for T in s.periods]
    assert counts == [1, 2, 3, 4, 5, 6, 6, 7, 8, 9]
    assert 0.9e6 < s.nnz < 1.1e6


def test_reproducible():
    a = synth.make_system(synth.small_config(seed=3))
    b = synth.make_system(synth.small_config(seed=3))
    c = synth.make_system(synth.small_config(seed=4))
    assert np.array_equal(a.val, b.val) and np.array_equal(a.col, b.col)
    assert np.array_equal(a.dt, b.dt)
    assert not np.array_equal(a.dt[: min(a.m, c.m)], c.dt[: min(a.m, c.m)])


def test_row_structure(cfg0_system):
    s = cfg0_system
    for i in range(0, s.m, 97):
        c = s.col[s.row_ptr[i]:s.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
        node, dep = c // s.nz, c % s.nz
        # each lateral node owns one run of consecutive depth columns (eq. 7 ordering)
        for k in np.unique(node):
            d = dep[node == k]
            assert np.all(np.diff(d) == 1)
    assert s.col.min() >= 0 and s.col.max() < s.n


def test_sensitivity_sums_to_minus_traveltime(cfg0_system):
    s = cfg0_system
    g1 = s.matvec(np.ones(s.n))
    assert np.allclose(g1, -s.t_ref, rtol=1e-12, atol=0)


def test_path_lengths_partition_of_unity():
    cfg = synth.config0()
    rng = np.random.default_rng(1)
    a = rng.uniform(0, cfg.region_deg, size=(50, 2))
    b = rng.uniform(0, cfg.region_deg, size=(50, 2))
    bend = rng.uniform(-0.05, 0.05, 50) * np.hypot(*(b - a).T)
    pt_ptr, px, py = synth.polylines(a, b, cfg.h, cfg.region_deg, bend)
    node_ptr, node_k, ln, plen = synth.bilinear_split(pt_ptr, px, py, cfg.h, cfg.nx, cfg.ny)
    sums = np.add.reduceat(ln, node_ptr[:-1])
    assert np.allclose(sums, plen, rtol=1e-12)
    assert np.all(ln > 0)


def test_grid_aligned_ray():
    # a ray along the grid line y = 3h from node x=2 to node x=9: the hat
    # functions integrate to h at interior nodes and h/2 at the two end nodes
    h, nx = 0.125, 16                      # binary-exact grid positions
    a = np.array([[2 * h, 3 * h]])
    b = np.array([[9 * h, 3 * h]])
    pt_ptr, px, py = synth.polylines(a, b, h, 15 * h)
    node_ptr, node_k, ln, plen = synth.bilinear_split(pt_ptr, px, py, h, nx, nx)
    hk = h * synth.KM_PER_DEG
    got = dict(zip(node_k.tolist(), ln.tolist()))
    expect = {3 * nx + i: (hk / 2 if i in (2, 9) else hk) for i in range(2, 10)}
    assert set(got) == set(expect)
    for k in expect:
        assert abs(got[k] - expect[k]) < 1e-12 * hk


def test_cell_diagonal_ray():
    # corner-to-corner inside one cell: weights L/3, L/3 (ends), L/6, L/6 (others)
    h, nx = 0.125, 16
    a = np.array([[4 * h, 5 * h]])
    b = np.array([[5 * h, 6 * h]])
    pt_ptr, px, py = synth.polylines(a, b, h, 15 * h)
    node_ptr, node_k, ln, plen = synth.bilinear_split(pt_ptr, px, py, h, nx, nx)
    L = np.sqrt(2) * h * synth.KM_PER_DEG
    got = dict(zip(node_k.tolist(), ln.tolist()))
    expect = {5 * nx + 4: L / 3, 6 * nx + 5: L / 3, 5 * nx + 5: L / 6, 6 * nx + 4: L / 6}
    assert set(got) == set(expect)
    for k in expect:
        assert abs(got[k] - expect[k]) < 1e-12 * L


def test_depth_kernel():
    z = np.linspace(0, 80, 20)
    for T in np.linspace(1, 40, 20):
        j0, w = synth.depth_kernel(z, T)
        assert j0 == 0            # the surface node is always kept
        assert abs(w.sum() - 1) < 1e-15 and np.all(w > 0)


def test_wavelength_filter():
    cfg = synth.small_config(nx=10, ny=10, nz=5, n_stations=14, region=2.0, min_wavelengths=2.0)
    s = synth.make_system(cfg)
    T = s.periods[s.row_period]
    lam = synth.phase_velocity(T) * T
    assert np.all(s.path_len[s.row_pair] >= 2.0 * lam)
    assert s.m < (14 * 13 // 2) * len(s.periods)


def test_noise_statistics(cfg0_system):
    s = cfg0_system
    z = (s.dt - s.gm_true) / (0.005 * s.t_ref)
    assert abs(z.mean()) < 0.05 and abs(z.std() - 1) < 0.05


def test_checker_rhs_batch():
    s = synth.make_system(synth.small_config())
    B = synth.checker_rhs_batch(s, 4, 3)
    assert B.shape == (s.m, 7)
    # bootstrap columns share G m_true and differ only by noise
    assert np.allclose((B[:, 4] - s.gm_true).std() / (0.005 * s.t_ref).mean(), 1, atol=0.5)
    assert not np.array_equal(B[:, 4], B[:, 5])


@pytest.mark.slow
def test_config1_size():
    s = synth.make_system(synth.config1())
    assert s.n == 128000
    assert 450_000 < s.m < 520_000
    assert 0.5e9 < s.nnz < 0.7e9
