"""Pins of the oracle's trapezoid and sphere section (solids of the Sec. 3.5
CMS case beyond boxes, tubes, cones and balls): closed-form distances and
normals, ray marching and sampling against an independent membership test
(angles by arccos and atan2), placement invariance."""
import math

import numpy as np
import pytest

import workloads as W
from tests.geomref import TRD, member

INF = float("inf")


def ev(o, st, par, op, p, v=None):
    return o.solid_eval(st, par, op, np.atleast_2d(p), None if v is None else np.atleast_2d(v))


def close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(1.0, abs(b))


def test_trd_closed_forms(oracle_lib):
    o = oracle_lib
    dx1, dx2, dy1, dy2, dz = 10.0, 20.0, 30.0, 10.0, 10.0
    par = [dx1, dx2, dy1, dy2, dz]
    hx = lambda z: dx1 + (dx2 - dx1) * (z + dz) / (2 * dz)  # noqa: E731
    hy = lambda z: dy1 + (dy2 - dy1) * (z + dz) / (2 * dz)  # noqa: E731
    # along the axes from outside and from the centre
    assert close(ev(o, TRD, par, "dist_in", [-100, 0, 0], [1, 0, 0])[0], 100 - hx(0))
    assert close(ev(o, TRD, par, "dist_out", [0, 0, 0], [1, 0, 0])[0], hx(0))
    assert close(ev(o, TRD, par, "dist_out", [0, 0, 0], [0, -1, 0])[0], hy(0))
    assert close(ev(o, TRD, par, "dist_out", [0, 0, 0], [0, 0, 1])[0], dz)
    assert close(ev(o, TRD, par, "dist_in", [0, 0, 50], [0, 0, -1])[0], 50 - dz)
    # at another height the half widths follow the taper
    for z in (-7.5, 3.0, 9.0):
        assert close(ev(o, TRD, par, "dist_out", [0, 0, z], [-1, 0, 0])[0], hx(z))
        assert close(ev(o, TRD, par, "dist_out", [0, 0, z], [0, 1, 0])[0], hy(z))
    # a ray along z at x inside the small end but outside the large one exits the slanted face:
    # x = hx(z) at z = -dz + 2 dz (x - dx1) / (dx2 - dx1)
    x0 = 14.0
    z_hit = -dz + 2 * dz * (x0 - dx1) / (dx2 - dx1)
    assert close(ev(o, TRD, par, "dist_in", [x0, 0, -50], [0, 0, 1])[0], z_hit + 50)
    # y tapers the other way: along +z from y0 the ray leaves through the slanted y face
    y0 = 20.0
    z_out = -dz + 2 * dz * (y0 - dy1) / (dy2 - dy1)
    assert close(ev(o, TRD, par, "dist_out", [0, y0, -dz + 1e-3], [0, 0, 1])[0], z_out - (-dz + 1e-3))
    # misses and surface rules
    assert ev(o, TRD, par, "dist_in", [-100, 0, 0], [-1, 0, 0])[0] == INF
    assert ev(o, TRD, par, "dist_in", [-100, 0, 50], [1, 0, 0])[0] == INF
    assert ev(o, TRD, par, "dist_in", [hx(0), 0, 0], [-1, 0, 0])[0] == 0.0
    assert ev(o, TRD, par, "dist_out", [hx(0), 0, 0], [1, 0, 0])[0] == 0.0
    # a ray along the outward normal of the slanted +x face, from outside, enters at its length
    b = (dx2 - dx1) / (2 * dz)
    n = np.array([1.0, 0.0, -b]) / math.sqrt(1 + b * b)
    foot = np.array([hx(2.0), 0.0, 2.0])
    for t in (0.5, 7.0, 40.0):
        assert close(ev(o, TRD, par, "dist_in", foot + t * n, -n)[0], t, 1e-11)
        # the signed value is the perpendicular distance to the face there
        assert close(ev(o, TRD, par, "d", foot + t * n)[0], t, 1e-11)
    assert close(ev(o, TRD, par, "d", foot - 0.25 * n)[0], -0.25, 1e-11)


def test_trd_normals(oracle_lib):
    o = oracle_lib
    dx1, dx2, dy1, dy2, dz = 10.0, 20.0, 30.0, 10.0, 10.0
    par = [dx1, dx2, dy1, dy2, dz]
    bx, by = (dx2 - dx1) / (2 * dz), (dy2 - dy1) / (2 * dz)
    pts = np.array([[15.0, 0, 0], [-15.0, 0, 0], [0, 20.0, 0], [0, -20.0, 0], [0, 0, 10.0], [0, 0, -10.0]])
    ref = np.array([[1, 0, -bx], [-1, 0, -bx], [0, 1, -by], [0, -1, -by], [0, 0, 1], [0, 0, -1]], float)
    ref /= np.linalg.norm(ref, axis=1)[:, None]
    n, faces = o.solid_normal(TRD, par, pts)
    assert np.allclose(n, ref, atol=1e-15) and np.all(faces == 1)
    # an edge: the lower face in +x, -x, +y, -y, +z, -z order wins the tie
    n, faces = o.solid_normal(TRD, par, np.array([[20.0, 0, 10.0]]))
    assert faces[0] == 2 and np.allclose(n[0], ref[0])


def test_trd_rejects_bad_parameters(oracle_lib):
    for par in ([0, 1, 1, 1, 1], [1, 1, 1, 1, 0], [1, -1, 1, 1, 1]):
        with pytest.raises(ValueError):
            oracle_lib.solid_eval(TRD, par, "d", np.zeros((1, 3)))


MORE = W.geometry.solids_zoo_more()
MORE_SOLIDS = [(int(MORE.solid_type[s]), MORE.solid_par[s]) for s in range(1, MORE.n_solids)]


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
    return hi


@pytest.mark.parametrize("k", range(len(MORE_SOLIDS)))
def test_ray_marching(oracle_lib, k):
    st, par = MORE_SOLIDS[k]
    rng = np.random.Generator(np.random.Philox(key=300 + k))
    checked_in = checked_out = 0
    while checked_in < 60 or checked_out < 30:
        p = rng.uniform(-160, 160, 3)
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        if member(st, par, p[None])[1][0] < 1e-6:
            continue
        inside = member(st, par, p[None])[0][0]
        if inside:
            got = ev(oracle_lib, st, par, "dist_out", p, v)[0]
            ref = _march(st, par, p, v, 600.0, False)
            assert abs(got - ref) < 1e-6, (p, v, got, ref)
            checked_out += 1
        else:
            got = ev(oracle_lib, st, par, "dist_in", p, v)[0]
            ref = _march(st, par, p, v, 600.0, True)
            if ref == INF:
                assert got == INF
            else:
                q = p + ref * v
                if member(st, par, q[None])[1][0] < 1e-6:
                    assert abs(got - ref) < 1e-6, (p, v, got, ref)
            checked_in += 1
    assert checked_out > 0


@pytest.mark.parametrize("k", range(len(MORE_SOLIDS)))
def test_inside_and_safety_sampling(oracle_lib, k):
    st, par = MORE_SOLIDS[k]
    rng = np.random.Generator(np.random.Philox(key=400 + k))
    pts = rng.uniform(-250, 250, (4000, 3))
    ins, m = member(st, par, pts)
    keep = m > 1e-6
    pts, ins = pts[keep], ins[keep]
    cls = ev(oracle_lib, st, par, "inside", pts)
    assert np.array_equal(cls == 1, ins)
    s_in = ev(oracle_lib, st, par, "safety_out", pts[ins])
    s_out = ev(oracle_lib, st, par, "safety_in", pts[~ins])
    # spheres of the safety radius stay on their side
    sph = rng.normal(size=(64, 3))
    sph /= np.linalg.norm(sph, axis=1)[:, None]
    for p, s in zip(pts[ins][:200], s_in[:200]):
        assert np.all(member(st, par, p + 0.999999 * s * sph)[0])
    for p, s in zip(pts[~ins][:200], s_out[:200]):
        assert not np.any(member(st, par, p + 0.999999 * s * sph)[0])


def test_distances_invariant_under_placement(oracle_lib):
    g = oracle_lib.Geometry(MORE)
    rng = np.random.Generator(np.random.Philox(key=17))
    n = 2000
    k = rng.integers(0, MORE.n_pv, n)
    tgt = MORE.pv_trans[k] + rng.uniform(-60, 60, size=(n, 3))
    src = rng.uniform(-900, 900, size=(n, 3))
    v = tgt - src
    v /= np.linalg.norm(v, axis=1)[:, None]
    T = g.locate(src, v)
    ok = T == 0
    s, lim, _ = g.compute_step(src[ok], v[ok], T[ok])
    hits = np.nonzero(lim >= 0)[0]
    assert len(hits) > 100
    for i in hits[:300]:
        l = lim[i]
        R = MORE.pv_rot[l].reshape(3, 3)
        t = MORE.pv_trans[l]
        pl = (src[ok][i] - t) @ R
        vl = v[ok][i] @ R
        s_id = MORE.lv_solid[MORE.pv_lv[l]]
        loc = ev(oracle_lib, int(MORE.solid_type[s_id]), MORE.solid_par[s_id], "dist_in", pl, vl)[0]
        assert abs(loc - s[i]) <= 1e-9 * max(1.0, s[i])


SPHERE = 5


def test_sphere_closed_forms(oracle_lib):
    o = oracle_lib
    shell = [50.0, 100.0, 0.0, 2 * math.pi, 0.0, math.pi]
    assert close(ev(o, SPHERE, shell, "dist_in", [-200, 0, 0], [1, 0, 0])[0], 100.0)
    assert close(ev(o, SPHERE, shell, "dist_out", [75, 0, 0], [1, 0, 0])[0], 25.0)
    assert close(ev(o, SPHERE, shell, "dist_out", [75, 0, 0], [-1, 0, 0])[0], 25.0)
    # from the bore the ray enters through the inner sphere
    assert close(ev(o, SPHERE, shell, "dist_in", [0, 0, 0], [0, 1, 0])[0], 50.0)
    # chord through the shell missing the bore: impact parameter 60 > rmin
    b = 60.0
    assert close(ev(o, SPHERE, shell, "dist_out", [-math.sqrt(90.0 ** 2 - b * b), b, 0], [1, 0, 0])[0],
                 math.sqrt(90.0 ** 2 - b * b) + math.sqrt(100.0 ** 2 - b * b))
    # a 45 degree cone around +z (theta in [0, pi/4])
    cone = [0.0, 100.0, 0.0, 2 * math.pi, 0.0, math.pi / 4]
    assert close(ev(o, SPHERE, cone, "dist_out", [0, 0, 50], [1, 0, 0])[0], 50.0)
    assert close(ev(o, SPHERE, cone, "dist_out", [0, 0, 50], [0, 0, 1])[0], 50.0)
    assert close(ev(o, SPHERE, cone, "dist_in", [60, 0, 10], [-1, 0, 0])[0], 50.0)
    assert ev(o, SPHERE, cone, "dist_in", [0, 0, -10], [1, 0, 0])[0] == INF
    # the band 45 to 135 degrees around the equator
    band = [0.0, 100.0, 0.0, 2 * math.pi, math.pi / 4, math.pi / 2]
    assert close(ev(o, SPHERE, band, "dist_out", [50, 0, 0], [0, 0, 1])[0], 50.0)
    assert close(ev(o, SPHERE, band, "dist_out", [50, 0, 0], [0, 0, -1])[0], 50.0)
    assert close(ev(o, SPHERE, band, "dist_in", [0, 0, 40], [1, 0, 0])[0], 40.0)
    # upper hemisphere: the equatorial plane
    hemi = [0.0, 100.0, 0.0, 2 * math.pi, 0.0, math.pi / 2]
    assert close(ev(o, SPHERE, hemi, "dist_in", [0, 0, -50], [0, 0, 1])[0], 50.0)
    assert close(ev(o, SPHERE, hemi, "dist_out", [0, 30, 20], [0, 0, -1])[0], 20.0)
    # a phi wedge [0, pi/2]: leaving through the phi = pi/2 plane
    wedge = [0.0, 100.0, 0.0, math.pi / 2, 0.0, math.pi]
    assert close(ev(o, SPHERE, wedge, "dist_out", [20, 10, 0], [-1, 0, 0])[0], 20.0)
    assert close(ev(o, SPHERE, wedge, "dist_in", [-30, 10, 0], [1, 0, 0])[0], 30.0)
    # signed value: perpendicular distance to the cone surface
    assert close(ev(o, SPHERE, cone, "d", [0, 0, 50])[0], -50 * math.sin(math.pi / 4), 1e-12)
    assert close(ev(o, SPHERE, band, "d", [0, 0, 80])[0], 80 * math.sin(math.pi / 4), 1e-12)


def test_sphere_normals(oracle_lib):
    o = oracle_lib
    cone = [20.0, 100.0, 0.0, 2 * math.pi, 0.0, math.pi / 4]
    pts = np.array([[0, 0, 100.0], [0, 0, 20.0], [30 * math.cos(0.3), 30 * math.sin(0.3), 30.0]])
    n, faces = o.solid_normal(SPHERE, cone, pts)
    # outer sphere radial, inner sphere inward, the cone's outward normal (cos, sin tilted by 45 deg)
    s = math.sqrt(0.5)
    ref = np.array([[0, 0, 1.0], [0, 0, -1.0], [s * math.cos(0.3), s * math.sin(0.3), -s]])
    assert np.allclose(n, ref, atol=1e-15) and np.all(faces == 1)
    band = [0.0, 100.0, 0.0, 2 * math.pi, 2.0, 1.0]  # theta in [2, 3]: below the equator
    q = 50 * np.array([math.sin(2.0), 0.0, math.cos(2.0)])  # on the theta = 2 cone
    n, faces = o.solid_normal(SPHERE, band, q[None])
    # outward = towards smaller theta: -(d/dtheta) of the unit position
    ref = -np.array([math.cos(2.0), 0.0, -math.sin(2.0)])
    assert np.allclose(n[0], ref, atol=1e-14) and faces[0] == 1
    hemi = [0.0, 100.0, 0.0, 2 * math.pi, 0.0, math.pi / 2]
    n, faces = o.solid_normal(SPHERE, hemi, np.array([[10.0, 5.0, 0.0]]))
    assert np.allclose(n[0], [0, 0, -1.0]) and faces[0] == 1


def test_sphere_rejects_bad_parameters(oracle_lib):
    for par in ([50, 40, 0, 1, 0, 1], [0, 10, 0, 4.0, 0, 1], [0, 10, 0, 1, 2.0, 1.5], [0, 10, 0, 1, 0, 0]):
        with pytest.raises(ValueError):
            oracle_lib.solid_eval(SPHERE, par, "d", np.zeros((1, 3)))
