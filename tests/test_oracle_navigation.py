"""Pins of the oracle's navigation: locate, ComputeStep, ComputeSafety, touchables."""
import numpy as np
import pytest

import workloads as W
from tests.geomref import locate_bruteforce

GEOMS = {
    "tiny": lambda: W.geometry.tiny(),
    "tiny_rot": lambda: W.geometry.tiny(rotated=True),
    "zoo": lambda: W.geometry.solids_zoo(),
    "calorimeter": lambda: W.geometry.calorimeter(n_layers=8, n_cells=6),
    "barrel": lambda: W.geometry.barrel(n_layers=8, n_seg=16, n_rings=4, n_orbs=8),
    "zoo_more": lambda: W.geometry.solids_zoo_more(),
    "endcap": lambda: W.geometry.endcap(n_wedges=12),
}


def _points(desc, rng, n):
    s = desc.lv_solid[desc.world_lv]
    h = desc.solid_par[s][:3] if desc.solid_type[s] == 0 else np.array([1600, 1600, 3000.0])
    pts = rng.uniform(-1.05, 1.05, size=(n, 3)) * h
    # concentrate half of them near the daughters of the world
    if desc.n_pv:
        k = rng.integers(0, desc.lv_dau_cnt[desc.world_lv], n // 2)
        pv = desc.lv_dau_off[desc.world_lv] + k
        pts[: n // 2] = desc.pv_trans[pv] + rng.normal(0, 150, size=(n // 2, 3))
    return pts


@pytest.mark.parametrize("name", list(GEOMS))
def test_touchables_breadth_first(oracle_lib, name):
    desc = GEOMS[name]()
    g = oracle_lib.Geometry(desc)
    parent, pv, lv, depth = g.touchables()
    assert g.n_touchables == desc.n_touchables()
    assert parent[0] == -1 and lv[0] == desc.world_lv
    # children of each touchable are contiguous, in slot order, after it
    for t in range(1, g.n_touchables):
        P = parent[t]
        assert P < t and depth[t] == depth[P] + 1
        assert desc.pv_lv[pv[t]] == lv[t]
        assert desc.lv_dau_off[lv[P]] <= pv[t] < desc.lv_dau_off[lv[P]] + desc.lv_dau_cnt[lv[P]]


@pytest.mark.parametrize("name", list(GEOMS))
def test_locate_matches_bruteforce(oracle_lib, name):
    desc = GEOMS[name]()
    g = oracle_lib.Geometry(desc)
    parent, pv, lv, depth = g.touchables()
    rng = np.random.Generator(np.random.Philox(key=31))
    pts = _points(desc, rng, 1500)
    ref, margin = locate_bruteforce(desc, parent, pv, lv, depth, pts)
    keep = margin > 1e-6
    got = g.locate(pts[keep])
    assert np.array_equal(got, ref[keep])
    # with a direction the answer is the same away from surfaces
    d = W.primaries.isotropic(rng, int(keep.sum()))
    assert np.array_equal(g.locate(pts[keep], d), ref[keep])


def test_locate_surface_direction_rule(oracle_lib):
    """On a shared face the direction decides; tangent means 'not in'."""
    desc = W.geometry.calorimeter(n_layers=2, n_cells=2)
    g = oracle_lib.Geometry(desc)
    parent, pv, lv, depth = g.touchables()
    # the face between the two cells of layer 0 at x = 0 (cells are 20 mm wide)
    z0 = desc.pv_trans[desc.lv_dau_off[1]][2]
    p = np.array([[0.0, 5.0, z0]] * 3)
    d = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0]])
    t = g.locate(p, d)
    # +x goes to the cell at ix = 1, -x to ix = 0, tangent stays in the layer
    assert depth[t[0]] == 3 and depth[t[1]] == 3 and t[0] != t[1]
    assert depth[t[2]] == 2


@pytest.mark.parametrize("name", list(GEOMS))
def test_compute_step_consistency(oracle_lib, name):
    desc = GEOMS[name]()
    g = oracle_lib.Geometry(desc)
    parent, pv, lv, depth = g.touchables()
    rng = np.random.Generator(np.random.Philox(key=41))
    pts = _points(desc, rng, 1200)
    ref, margin = locate_bruteforce(desc, parent, pv, lv, depth, pts)
    keep = (margin > 1e-6) & (ref >= 0)
    pts = pts[keep]
    T = ref[keep]
    d = W.primaries.isotropic(rng, len(pts))
    step, lim, nxt = g.compute_step(pts, d, T)
    assert np.all(step > 0) and np.all(np.isfinite(step))
    # halfway along the step the point is still in the same touchable
    mid = pts + 0.5 * step[:, None] * d
    ref_mid, m_mid = locate_bruteforce(desc, parent, pv, lv, depth, mid)
    ok = m_mid > 1e-6
    assert np.array_equal(ref_mid[ok], T[ok])
    # just past the step the point is in the relocated touchable
    past = pts + (step[:, None] + 2e-5) * d
    ref_past, m_past = locate_bruteforce(desc, parent, pv, lv, depth, past)
    ok = m_past > 1e-6
    assert np.array_equal(ref_past[ok], nxt[ok])
    # daughter limiters point at children of T, mother limiters leave T
    for t, l, n in zip(T, lim, nxt):
        if l >= 0:
            assert depth[n] > depth[t]
        else:
            assert n != t


@pytest.mark.parametrize("name", list(GEOMS))
def test_safety_is_lower_bound(oracle_lib, name):
    desc = GEOMS[name]()
    g = oracle_lib.Geometry(desc)
    parent, pv, lv, depth = g.touchables()
    rng = np.random.Generator(np.random.Philox(key=51))
    pts = _points(desc, rng, 300)
    ref, margin = locate_bruteforce(desc, parent, pv, lv, depth, pts)
    keep = (margin > 1e-6) & (ref >= 0)
    pts, T = pts[keep], ref[keep]
    saf = g.compute_safety(pts, T)
    assert np.all(saf >= 0)
    dirs = W.primaries.isotropic(rng, 200)
    for p, t, s in zip(pts, T, saf):
        if s <= 1e-6:
            continue
        sph = p + s * (1 - 1e-9) * dirs
        loc, m = locate_bruteforce(desc, parent, pv, lv, depth, sph)
        assert np.all(loc[m > 1e-7] == t)


def _surface_queries(desc, g, rng, n):
    """Points where rays from random points cross a boundary (the brute-force
    answer), with directions that graze, enter and leave."""
    pts = _points(desc, rng, n)
    dirs = W.primaries.isotropic(rng, n)
    T = g.locate(pts, dirs)
    ok = T >= 0
    s, lim, _ = g.compute_step(pts[ok], dirs[ok], T[ok].astype(np.int32))
    fin = np.isfinite(s)
    end = pts[ok][fin] + s[fin, None] * dirs[ok][fin]
    return end, W.primaries.isotropic(rng, end.shape[0])


FULL = dict(GEOMS, calorimeter_full=lambda: W.geometry.calorimeter(),
            barrel_full=lambda: W.geometry.barrel())


@pytest.mark.parametrize("name", list(FULL))
def test_voxel_mode_equals_bruteforce(oracle_lib, name):
    """The oracle's cell-grid search returns exactly the brute-force locate,
    step length, limiter and next touchable, including points on surfaces."""
    desc = FULL[name]()
    a = oracle_lib.Geometry(desc)
    b = oracle_lib.Geometry(desc)
    b.set_voxels(True)
    rng = np.random.Generator(np.random.Philox(key=31))
    pts = _points(desc, rng, 6000)
    dirs = W.primaries.isotropic(rng, 6000)
    end, d2 = _surface_queries(desc, a, rng, 3000)
    pts, dirs = np.concatenate([pts, end]), np.concatenate([dirs, d2])
    assert np.array_equal(a.locate(pts, dirs), b.locate(pts, dirs))
    assert np.array_equal(a.locate(pts), b.locate(pts))
    sa, la, na = a.compute_step(pts, dirs)
    sb, lb, nb = b.compute_step(pts, dirs)
    assert np.array_equal(sa.view(np.uint64), sb.view(np.uint64))
    assert np.array_equal(la, lb) and np.array_equal(na, nb)


@pytest.mark.parametrize("name,n", [("tiny", 3000), ("calorimeter", 1500), ("barrel", 400), ("endcap", 1500)])
def test_voxel_mode_transport_identical(oracle_lib, name, n):
    """Whole transports in voxel mode reproduce the brute-force per-step logs."""
    geoms, prim, _ = W.WORKLOADS[name](n=n)
    a = oracle_lib.Geometry(geoms[0])
    b = oracle_lib.Geometry(geoms[0])
    b.set_voxels(True)
    ra = a.transport(prim, seed=0, log_cap=256)
    rb = b.transport(prim, seed=0, log_cap=256)
    assert ra["counters"] == rb["counters"]
    assert np.array_equal(ra["log"], rb["log"]) and np.array_equal(ra["log_n"], rb["log_n"])
    assert np.array_equal(ra["edep_event"], rb["edep_event"])
