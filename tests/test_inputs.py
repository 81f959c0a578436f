"""Seeded input generators: determinism, counts and the stated properties."""
import math

import numpy as np

from paper_1012_5082_amd import inputs as I


def test_bcc_shape_and_box():
    x, y, z, box = I.bcc(10, 10, 10)
    assert x.size == 2000
    assert np.allclose(box, 28.7)
    assert x.min() >= 0 and x.max() < box[0]


def test_initial_species_exact_count_and_seeded():
    a = I.initial_species(2000, 0.05, 3)
    b = I.initial_species(2000, 0.05, 3)
    assert a.sum() == 100 and np.array_equal(a, b)
    assert not np.array_equal(a, I.initial_species(2000, 0.05, 4))


def test_thermalize_sigma_and_wrap():
    x, y, z, box = I.bcc(20, 20, 20)
    xt, yt, zt = I.thermalize(x, y, z, box, 0.05, 1)
    d = xt - x
    d -= box[0] * np.round(d / box[0])
    assert abs(d.std() - 0.05) < 0.002
    for u, L in ((xt, box[0]), (yt, box[1]), (zt, box[2])):
        assert u.min() >= 0.0 and u.max() < L


def test_mb_velocities_exact_temperature_zero_momentum():
    sp = I.initial_species(4000, 0.1, 2)
    vx, vy, vz = I.mb_velocities(sp, 700.0, 3)
    T, _ = I.kinetic_temperature(vx, vy, vz, sp)
    assert abs(T - 700.0) < 1e-9
    m = np.where(sp == 0, I.MASS_A, I.MASS_B)
    for v in (vx, vy, vz):
        assert abs(math.fsum(m * v)) < 1e-10


def test_voronoi_small():
    x, y, z, box, grain = I.voronoi_poly(ncell=24, n_grains=4, seed=5)
    n_ideal = 2 * 24 ** 3
    assert 0.9 * n_ideal < x.size < 1.05 * n_ideal
    assert set(np.unique(grain)) == {0, 1, 2, 3}
    from scipy.spatial import cKDTree
    P = np.stack([x, y, z], 1)
    t = cKDTree(P, boxsize=box[0])
    pairs = t.query_pairs(2.0, output_type="ndarray")
    assert pairs.size == 0 or np.all(grain[pairs[:, 0]] == grain[pairs[:, 1]])
    # deterministic
    x2, *_ = I.voronoi_poly(ncell=24, n_grains=4, seed=5)
    assert np.array_equal(x, x2)
