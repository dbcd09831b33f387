"""Host-side checks of the seeded input generators (no GPU)."""
import numpy as np

import workloads as W


def test_paper_regular_is_column_major_pinhole_grid():
    pos, d, life = W.primaries.paper_regular()
    assert pos.shape == (100_000, 3) and not pos.any()
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)
    assert np.all(life == 1.0)
    # column-major: the first 250 rays share a column (same x / z ratio), rows vary
    ratio = d[:, 0] / d[:, 2]
    assert np.allclose(ratio[:250], ratio[0]) and not np.isclose(ratio[250], ratio[0])
    assert np.all(np.diff(d[:250, 1] / d[:250, 2]) > 0)
    # square pixels spanning [-1, 1] x [-0.625, 0.625] on the plane z = 1
    assert np.isclose(ratio.min(), -1 + 0.0025) and np.isclose(ratio.max(), 1 - 0.0025)
    ry = d[:, 1] / d[:, 2]
    assert np.isclose(ry.min(), -0.625 + 0.0025) and np.isclose(ry.max(), 0.625 - 0.0025)


def test_paper_random_isotropic_exponential():
    pos, d, life = W.primaries.paper_random(200_000, seed=3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)
    assert np.all(life > 0)
    assert abs(life.mean() - 1.0) < 0.01 and abs(life.var() - 1.0) < 0.03
    assert np.all(np.abs(d.mean(axis=0)) < 0.01)


def test_spheres_geometry_matches_the_paper_layout():
    g = W.geometry.spheres()
    assert g.n_pv == 8000
    c = g.pv_trans
    assert np.allclose(np.unique(c[:, 0]), -2500 + 125 + 250 * np.arange(20))
    # the centre (the particles' start) lies in vacuum between balls
    assert np.min(np.linalg.norm(c, axis=1)) > 100.0
