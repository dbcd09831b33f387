"""Pins of the oracle's solids: closed-form distances, ray marching, safeties."""
import math

import numpy as np
import pytest

import workloads as W
from tests.geomref import member, BOX, TUBS, CONS, ORB

INF = float("inf")


def ev(o, st, par, op, p, v=None):
    return o.solid_eval(st, par, op, np.atleast_2d(p), None if v is None else np.atleast_2d(v))


def close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(1.0, abs(b))


def test_box_closed_forms(oracle_lib):
    o = oracle_lib
    par = [100, 100, 100]
    # Tiny: ray from the world origin to the cube centred at (250,250,250)
    # along (1,1,1)/sqrt3 enters at 150 sqrt3 (local frame: origin at -250).
    u = np.ones(3) / math.sqrt(3)
    assert close(ev(o, BOX, par, "dist_in", [-250, -250, -250], u)[0], 150 * math.sqrt(3))
    # a ray from (0, 250, 250) along +x meets the face x = 150 at 150 mm
    assert close(ev(o, BOX, par, "dist_in", [-250, 0, 0], [1, 0, 0])[0], 150.0)
    assert ev(o, BOX, par, "dist_in", [-250, 0, 0], [-1, 0, 0])[0] == INF
    assert ev(o, BOX, par, "dist_in", [-250, 150, 0], [1, 0, 0])[0] == INF
    assert close(ev(o, BOX, par, "dist_out", [0, 0, 0], [0, 0, 1])[0], 100.0)
    assert close(ev(o, BOX, par, "dist_out", [30, 40, 0], u)[0], 60 * math.sqrt(3))
    # on the surface moving in -> 0 ; moving out -> dist_out 0, dist_in inf
    assert ev(o, BOX, par, "dist_in", [100, 0, 0], [-1, 0, 0])[0] == 0.0
    assert ev(o, BOX, par, "dist_in", [100, 0, 0], [1, 0, 0])[0] == INF
    assert ev(o, BOX, par, "dist_out", [100, 0, 0], [1, 0, 0])[0] == 0.0
    assert ev(o, BOX, par, "inside", [100, 0, 0], [-1, 0, 0])[0] == 1
    assert ev(o, BOX, par, "inside", [100, 0, 0], [0, 1, 0])[0] == -1  # tangent: not in
    assert ev(o, BOX, par, "inside", [100, 0, 0])[0] == 1  # no direction: surface counts as in
    assert close(ev(o, BOX, par, "safety_in", [150, 120, 0])[0], 50.0)
    assert close(ev(o, BOX, par, "safety_out", [50, 70, -20])[0], 30.0)


def test_orb_closed_forms(oracle_lib):
    o = oracle_lib
    R = 50.0
    par = [R]
    assert close(ev(o, ORB, par, "dist_out", [0, 0, 0], [0.6, 0.8, 0])[0], R)
    D, b = 200.0, 30.0
    assert close(ev(o, ORB, par, "dist_in", [-D, b, 0], [1, 0, 0])[0], D - math.sqrt(R * R - b * b))
    assert ev(o, ORB, par, "dist_in", [-D, 60, 0], [1, 0, 0])[0] == INF
    assert close(ev(o, ORB, par, "dist_out", [-math.sqrt(R * R - b * b), b, 0], [1, 0, 0])[0],
                 2 * math.sqrt(R * R - b * b), 1e-11)
    assert close(ev(o, ORB, par, "safety_in", [0, 0, 80])[0], 30.0)


def test_tubs_closed_forms(oracle_lib):
    o = oracle_lib
    rmin, rmax, dz = 40.0, 110.0, 90.0
    par = [rmin, rmax, dz, 0.0, 2 * math.pi]
    # radial ray from the axis: enters at rmin, leaves at rmax
    assert close(ev(o, TUBS, par, "dist_in", [0, 0, 10], [1, 0, 0])[0], rmin)
    assert close(ev(o, TUBS, par, "dist_out", [rmin, 0, 10], [1, 0, 0])[0], rmax - rmin)
    # oblique ray from the axis at polar angle theta: rmin / sin(theta)
    th = 0.7
    v = [math.sin(th), 0, math.cos(th)]
    assert close(ev(o, TUBS, par, "dist_in", [0, 0, -20], v)[0], rmin / math.sin(th))
    # chord of the bore at offset b: from the inner surface moving inward,
    # the next entry is on the far side, 2 sqrt(rmin^2 - b^2) away
    bb = 25.0
    x0 = -math.sqrt(rmin * rmin - bb * bb)
    assert close(ev(o, TUBS, par, "dist_in", [x0, bb, 0], [1, 0, 0])[0],
                 2 * math.sqrt(rmin * rmin - bb * bb), 1e-10)
    # along z at radius r0 inside the shell: the z face
    assert close(ev(o, TUBS, par, "dist_out", [60, 0, 0], [0, 0, 1])[0], dz)
    assert close(ev(o, TUBS, par, "dist_in", [60, 0, -200], [0, 0, 1])[0], 200 - dz)
    assert ev(o, TUBS, par, "dist_in", [20, 0, -200], [0, 0, 1])[0] == INF  # in the bore
    # phi section: ray in the xy plane hitting the start plane (phi = 0.3)
    sphi, dphi = 0.3, 1.2
    ps = [rmin, rmax, dz, sphi, dphi]
    beta = sphi
    r0 = 80.0
    # point just below the plane at radius r0, moving perpendicular to it
    n_out = np.array([math.sin(beta), -math.cos(beta), 0.0])
    on = np.array([r0 * math.cos(beta), r0 * math.sin(beta), 0.0])
    p = on + 7.0 * n_out
    assert close(ev(o, TUBS, ps, "dist_in", p, -n_out)[0], 7.0)
    assert close(ev(o, TUBS, ps, "safety_in", p)[0], 7.0)
    # end plane: from inside moving across it
    be = sphi + dphi
    n_end = np.array([-math.sin(be), math.cos(be), 0.0])
    q = np.array([r0 * math.cos(be), r0 * math.sin(be), 0.0]) - 5.0 * n_end
    assert close(ev(o, TUBS, ps, "dist_out", q, n_end)[0], 5.0)


def test_cons_closed_forms(oracle_lib):
    o = oracle_lib
    rmin1, rmax1, rmin2, rmax2, dz = 20.0, 90.0, 50.0, 130.0, 80.0
    par = [rmin1, rmax1, rmin2, rmax2, dz, 0.0, 2 * math.pi]

    def rmax(z):
        return rmax1 + (rmax2 - rmax1) * (z + dz) / (2 * dz)

    def rmin(z):
        return rmin1 + (rmin2 - rmin1) * (z + dz) / (2 * dz)

    for z in [-50.0, 0.0, 33.0]:
        # radial ray from the axis at height z: rmin(z), then rmax(z)
        assert close(ev(o, CONS, par, "dist_in", [0, 0, z], [0, 1, 0])[0], rmin(z), 1e-11)
        assert close(ev(o, CONS, par, "dist_out", [0, rmin(z), z], [0, 1, 0])[0],
                     rmax(z) - rmin(z), 1e-11)
    # ray along +z at radius r0 inside the shell: leaves where rmax(z) = r0
    r0 = 100.0
    zc = -dz + (r0 - rmax1) / (rmax2 - rmax1) * 2 * dz
    assert close(ev(o, CONS, par, "dist_in", [r0, 0, -200], [0, 0, 1])[0], 200 + zc, 1e-11)
    # at radius 35 going +z: in the bore until rmin(z) = 35 ... it starts inside
    # the material at z = -dz (rmin1 = 20 < 35) and leaves into the bore
    r1 = 35.0
    zi = -dz + (r1 - rmin1) / (rmin2 - rmin1) * 2 * dz
    assert close(ev(o, CONS, par, "dist_out", [r1, 0, -dz + 1], [0, 0, 1])[0], zi - (-dz + 1), 1e-11)
    # perpendicular safety to the outer cone
    z = 0.0
    slope = (rmax2 - rmax1) / (2 * dz)
    p = [rmax(z) + 10.0, 0, z]
    assert close(ev(o, CONS, par, "safety_in", p)[0], 10.0 / math.sqrt(1 + slope * slope), 1e-11)


ZOO = W.geometry.solids_zoo()
ZOO_SOLIDS = [(int(ZOO.solid_type[s]), ZOO.solid_par[s]) for s in range(1, ZOO.n_solids)]


def _march(st, par, p, v, tmax, first_inside, dt=0.02):
    """First t along the ray where membership changes to `first_inside`."""
    t = np.arange(0.0, tmax, dt)
    ins, _ = member(st, par, p + t[:, None] * v)
    hit = np.nonzero(ins == first_inside)[0]
    if len(hit) == 0:
        return INF
    i = hit[0]
    if i == 0:
        return 0.0
    lo, hi = t[i - 1], t[i]
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if member(st, par, (p + mid * v)[None])[0][0] == first_inside:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("k", range(len(ZOO_SOLIDS)))
def test_ray_marching_dist_in_out(oracle_lib, k):
    st, par = ZOO_SOLIDS[k]
    rng = np.random.Generator(np.random.Philox(key=100 + k))
    nrays = 120
    bad = 0
    for _ in range(nrays):
        # start outside on a sphere, aim at a random point near the solid
        d = W.primaries.isotropic(rng, 1)[0]
        p = 400.0 * d
        target = rng.uniform(-120, 120, 3)
        v = target - p
        v /= np.linalg.norm(v)
        if member(st, par, p[None])[1][0] < 1e-6:
            continue
        t_or = ev(oracle_lib, st, par, "dist_in", p, v)[0]
        t_ref = _march(st, par, p, v, 900.0, True)
        if t_ref == INF or t_or == INF:
            # a miss must be a miss on both sides, unless the chord is thinner than the grid
            if t_ref != t_or:
                q = p + t_or * v if t_or < INF else None
                chord = ev(oracle_lib, st, par, "dist_out", q + 1e-9 * v, v)[0] if q is not None else 0
                if chord > 0.05:
                    bad += 1
            continue
        if abs(t_or - t_ref) > 1e-7 * max(1, t_ref):
            bad += 1
            continue
        # from just inside the entry point, dist_out against marching to the exit
        q = p + (t_ref + 1e-4) * v
        if member(st, par, q[None])[1][0] < 1e-6:
            continue
        o_out = ev(oracle_lib, st, par, "dist_out", q, v)[0]
        r_out = _march(st, par, q, v, 900.0, False)
        if abs(o_out - r_out) > 1e-7 * max(1, r_out):
            bad += 1
    assert bad == 0


@pytest.mark.parametrize("k", range(len(ZOO_SOLIDS)))
def test_inside_and_safety_sampling(oracle_lib, k):
    st, par = ZOO_SOLIDS[k]
    rng = np.random.Generator(np.random.Philox(key=200 + k))
    pts = rng.uniform(-180, 180, size=(3000, 3))
    ins, m = member(st, par, pts)
    keep = m > 1e-6
    got = ev(oracle_lib, st, par, "inside", pts[keep])
    assert np.all((got == 1) == ins[keep])
    # safeties are lower bounds: a sphere of that radius never crosses the surface
    s_in = ev(oracle_lib, st, par, "safety_in", pts)
    s_out = ev(oracle_lib, st, par, "safety_out", pts)
    assert np.all(s_in >= 0) and np.all(s_out >= 0)
    assert np.all((s_in == 0) | (s_out == 0))
    dirs = W.primaries.isotropic(rng, 64)
    for i in range(0, len(pts), 15):
        s = max(s_in[i], s_out[i]) * (1 - 1e-9)
        if s <= 0:
            continue
        sph = pts[i] + s * dirs
        ins_s, _ = member(st, par, sph)
        if s_in[i] > 0:
            assert not ins_s.any()
        else:
            assert ins_s.all()


def test_distances_invariant_under_placement(oracle_lib):
    """A placed daughter's entry distance equals the local-frame distance."""
    g = oracle_lib.Geometry(ZOO)
    rng = np.random.Generator(np.random.Philox(key=9))
    n = 400
    pos = rng.uniform(-950, 950, size=(n, 3))
    k = rng.integers(0, ZOO.n_pv, n)
    tgt = ZOO.pv_trans[k] + rng.uniform(-40, 40, size=(n, 3))
    v = tgt - pos
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    T = g.locate(pos, v)
    sel = T == 0
    step, lim, _ = g.compute_step(pos[sel], v[sel], T[sel])
    for p, d, s, l in zip(pos[sel], v[sel], step, lim):
        if l < 0:
            continue
        R = ZOO.pv_rot[l].reshape(3, 3)
        t = ZOO.pv_trans[l]
        pl = R.T @ (p - t)
        vl = R.T @ d
        s_id = ZOO.lv_solid[ZOO.pv_lv[l]]
        loc = ev(oracle_lib, int(ZOO.solid_type[s_id]), ZOO.solid_par[s_id], "dist_in", pl, vl)[0]
        assert abs(loc - s) <= 1e-9 * max(1, s)
