"""Seeded synthetic input images: reproducibility, porosity and percolation."""
import numpy as np

from lbm_inputs import (sphere, slit, duct, pipe, triangle_channel, sphere_pack,
                        gaussian_random_field, percolating_x, random_mask, porosity, workload)


def test_single_sphere_voxel_count():
    m = sphere(32, (15.5, 15.5, 15.5), 8.0)
    assert m.shape == (32, 32, 32) and m.dtype == np.uint8
    assert int(m.sum()) == 2176
    assert abs(porosity(m) - 0.93359375) < 1e-12


def test_channels():
    assert porosity(slit(4, 10, 3, 8)) == 0.8
    d = duct(5, 6, wall=2)
    assert d.shape == (8, 8, 5) and int((d == 0).sum()) == 36 * 5
    p = pipe(3, 33, 8.0)
    area = int((p[:, :, 0] == 0).sum())
    assert abs(area / (np.pi * 64) - 1) < 0.05
    t = triangle_channel(2, 64, 40.0)
    area = int((t[:, :, 0] == 0).sum())
    assert abs(area / (np.sqrt(3) / 4 * 1600) - 1) < 0.05


def test_pack_seeded_and_porosity():
    a = sphere_pack(48, 5.0, 0.45, seed=3, hard_core=4.0)
    b = sphere_pack(48, 5.0, 0.45, seed=3, hard_core=4.0)
    assert np.array_equal(a, b)
    assert 0.42 < porosity(a) <= 0.45


def test_grf_seeded_porosity_and_spanning():
    a = gaussian_random_field(40, 3.0, 0.3, seed=4, filter_percolation=False)
    b = gaussian_random_field(40, 3.0, 0.3, seed=4, filter_percolation=False)
    assert np.array_equal(a, b)
    assert abs(porosity(a) - 0.3) < 1e-6
    f = percolating_x(a)
    assert porosity(f) <= porosity(a) and porosity(f) > 0.2
    assert np.all(a[f == 0] == 0)                       # only fluid is kept
    assert (f[:, :, 0] == 0).any() and (f[:, :, -1] == 0).any()


def test_percolation_removes_isolated_pocket():
    m = slit(10, 12, 5, 4)
    m[2, 8, 4] = 0                      # a fluid pocket inside the solid slab
    f = percolating_x(m)
    assert f[2, 8, 4] == 1
    assert np.array_equal(f[:, :4, :], m[:, :4, :])


def test_percolation_links_across_periodic_faces():
    # a channel that is only connected through the periodic y face
    m = np.ones((3, 6, 8), np.uint8)
    m[1, 5, :4] = 0
    m[1, 0, 3:] = 0
    f = percolating_x(m)
    assert np.array_equal(f, m)


def test_random_mask_and_workload_table():
    m = random_mask((5, 6, 7), 0.3, seed=1)
    assert m.shape == (5, 6, 7) and abs(m.mean() - 0.3) < 0.15
    s = workload("sc_sphere_32")
    assert int(s.sum()) == 2176
