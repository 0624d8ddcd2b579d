"""Input generator (RSA + voxelization, Sec. 2 of arXiv:1504.07499) against
the paper's tables and basic invariants.  CPU only."""
import os

import numpy as np
import pytest

from paper_1504_07499_amd import geom

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NSP = [30, 40, 50, 60, 70, 80, 90, 100]


def _table(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


@pytest.mark.parametrize("name,res", [("coating_voxels_tab1_res64.txt", 64),
                                      ("coating_voxels_tab2_res128.txt", 128),
                                      ("coating_voxels_tab3_res256.txt", 256)])
def test_coating_thickness_tables(name, res):
    """Tables 1-3: thickness = l * Res * r(n_sp) with the generator's radius
    r = (3 f / (4 pi n))^(1/3), f = 0.3 (the printed formula has n_sp in the
    numerator; every entry matches only the n^(-1/3) form)."""
    tab = _table(name)
    for row in tab:
        layer, vals = row[0], row[1:]
        got = np.array([layer * res * geom.radius(n, 0.3) for n in NSP])
        assert np.abs(got - vals).max() <= 0.0051, (layer, got, vals)


def test_coating_fraction_table_tab0():
    """Table tab0: f_coating(l) = f_sp (1 - (1 - l)^3), the coating being the
    outer shell of relative width l of each sphere of fraction 0.3."""
    tab = _table("coating_fraction_tab0.txt")
    for layer, fc in tab:
        assert abs(0.3 * (1 - (1 - layer) ** 3) - fc) <= 6e-5


@pytest.mark.parametrize("layer", [0.1, 0.2, 0.5])
def test_voxelized_coating_fraction_approaches_tab0(layer):
    tab = dict(map(tuple, _table("coating_fraction_tab0.txt")))
    ph, _, _ = geom.generate(128, 30, 0.3, layer, 5)
    frac = np.bincount(ph.ravel(), minlength=3) / ph.size
    assert abs(frac[2] - tab[layer]) <= 0.03 * tab[layer]
    assert abs(frac[1] + frac[2] - 0.3) <= 0.01


def _min_pair_distance(c):
    d = c[:, None, :] - c[None, :, :]
    d -= np.round(d)
    r = np.sqrt((d ** 2).sum(-1))
    r[np.arange(len(c)), np.arange(len(c))] = np.inf
    return r.min()


@pytest.mark.parametrize("n,f", [(8, 0.2), (50, 0.3), (100, 0.3), (100, 0.4), (20, 0.4)])
def test_rsa_non_overlap_and_determinism(n, f):
    c1, m1 = geom.place(n, f, 17)
    c2, m2 = geom.place(n, f, 17)
    c3, _ = geom.place(n, f, 18)
    assert np.array_equal(c1, c2) and m1 == m2
    assert not np.array_equal(c1, c3)
    assert np.all((c1 >= 0) & (c1 < 1))
    assert _min_pair_distance(c1) >= 2 * geom.radius(n, f) * (1 - 1e-12)


def test_dense_packing_uses_shaking():
    """40 % with 100 spheres exceeds what plain RSA reaches; the generator
    reports the Monte Carlo fallback."""
    _, method = geom.place(100, 0.4, 3)
    assert method == 1
    _, method = geom.place(30, 0.3, 3)
    assert method == 0


def test_single_sphere_voxel_volume():
    r = 0.3
    ph = geom.voxelize(64, np.array([[0.25, 0.5, 0.9]]), r, 0.5)
    frac = np.bincount(ph.ravel(), minlength=3) / ph.size
    vol = 4.0 / 3.0 * np.pi * r ** 3
    assert abs(frac[1] + frac[2] - vol) <= 0.01 * vol
    assert abs(frac[1] - vol / 8) <= 0.02 * vol / 8


def test_generate_equals_place_then_voxelize():
    ph, c, _ = geom.generate(48, 12, 0.25, 0.2, 99)
    ph2 = geom.voxelize(48, c, geom.radius(12, 0.25), 0.2)
    assert np.array_equal(ph, ph2)


def test_generator_rejects_bad_input():
    with pytest.raises(ValueError):
        geom.generate(32, 1, 0.9, 0.1, 1)  # radius >= 0.5
    with pytest.raises(ValueError):
        geom.generate(32, 5, 0.2, 1.5, 1)


# ------------------------------------------------------------ aligned fibres
def _min_pair_distance_2d(c):
    d = c[:, None, :] - c[None, :, :]
    d -= np.round(d)
    dist = np.sqrt((d ** 2).sum(-1))
    dist[np.diag_indices(len(c))] = np.inf
    return dist.min()


@pytest.mark.parametrize("n,f", [(20, 0.3), (50, 0.5)])
def test_fiber_rsa_non_overlap_and_determinism(n, f):
    """Fibre axes: periodic minimum distance >= 2 r, seeded, in the unit square."""
    c1, m1 = geom.place_fibers(n, f, 17)
    c2, m2 = geom.place_fibers(n, f, 17)
    c3, _ = geom.place_fibers(n, f, 18)
    assert np.array_equal(c1, c2) and m1 == m2
    assert not np.array_equal(c1, c3)
    assert np.all((c1 >= 0) & (c1 < 1))
    assert _min_pair_distance_2d(c1) >= 2 * geom.fiber_radius(n, f) * (1 - 1e-12)


def test_fiber_image_is_invariant_along_z_and_fills_f():
    """The image of fibres along z repeats one cross-section on every z plane;
    the voxel fraction of fibre (core + coating) approaches f, that of the
    core (1 - l)^2 f."""
    ph, c, _ = geom.generate_fibers(96, 12, 0.35, 0.25, 4)
    assert np.array_equal(ph, np.broadcast_to(ph[0], ph.shape))
    frac = np.bincount(ph.ravel(), minlength=3) / ph.size
    assert abs(frac[1] + frac[2] - 0.35) <= 0.01 * 0.35
    assert abs(frac[1] - 0.75 ** 2 * 0.35) <= 0.02 * 0.35
    assert np.array_equal(ph, geom.voxelize_fibers(96, c, geom.fiber_radius(12, 0.35), 0.25))


def test_fiber_generator_rejects_bad_input():
    with pytest.raises(ValueError):
        geom.generate_fibers(32, 1, 0.9, 0.1, 1)  # radius >= 0.5
    with pytest.raises(ValueError):
        geom.generate_fibers(32, 5, 0.2, 1.5, 1)


def test_mixed_spheres_and_fibers():
    """Mixed inclusions: spheres keep rs + rf from every fibre axis and 2 rs
    from each other; both shapes' voxel fractions approach their targets."""
    cs, cf = geom.place_mixed(10, 0.1, 8, 0.2, 3)
    rs, rf = geom.radius(10, 0.1), geom.fiber_radius(8, 0.2)
    d = cs[:, None, :2] - cf[None, :, :]
    d -= np.round(d)
    assert np.sqrt((d ** 2).sum(-1)).min() >= (rs + rf) * (1 - 1e-12)
    assert _min_pair_distance(cs) >= 2 * rs * (1 - 1e-12)
    assert _min_pair_distance_2d(cf) >= 2 * rf * (1 - 1e-12)
    ph = geom.generate_mixed(96, 10, 0.1, 8, 0.2, 0.2, 3)
    fib = geom.voxelize_fibers(96, cf, rf, 0.2)
    sph = geom.voxelize(96, cs, rs, 0.2)
    assert np.array_equal(ph[(fib > 0) & (sph == 0)], fib[(fib > 0) & (sph == 0)])
    assert np.array_equal(ph[sph == 1], sph[sph == 1])
    frac = np.bincount(ph.ravel(), minlength=3) / ph.size
    assert abs(frac[1] + frac[2] - 0.3) <= 0.02 * 0.3
