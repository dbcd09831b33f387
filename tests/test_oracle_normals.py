"""Pins of the oracle's surface normal (Sec. 3.2: the normal of the boundary
surface at the crossing point).

* closed forms: box faces, orb radial, tube outer/inner radial, z caps, the
  outward normals of the two phi half-planes;
* slanted cone faces: unit length, perpendicular to both surface tangents
  (along the generator and around the axis), and pointing outward (a small
  step along it leaves the solid, one against it enters);
* every family: the normal equals the central finite-difference gradient of
  the signed value d(p), itself pinned by the solid tests;
* edges and corners report two or more faces;
* queries: exit normals on the tiny geometry along rays with known crossings.
"""
import math

import numpy as np

import workloads as W
from tests.geomref import BOX, CONS, ORB, TUBS


def test_box_faces_edges_corners(oracle_lib):
    o = oracle_lib
    h = [10.0, 20.0, 30.0]
    rng = np.random.default_rng(1)
    for axis in range(3):
        for sign in (-1.0, 1.0):
            p = rng.uniform(-0.9, 0.9, (50, 3)) * h
            p[:, axis] = sign * h[axis]
            n, f = o.solid_normal(BOX, h, p)
            want = np.zeros(3)
            want[axis] = sign
            assert np.array_equal(n, np.tile(want, (50, 1)))
            assert np.all(f == 1)
    n, f = o.solid_normal(BOX, h, [[10, 20, 0], [-10, 0, 30], [10, -20, -30]])
    assert list(f) == [2, 2, 3]
    # on an edge or a corner the first face in x, y, z order defines the normal
    assert np.array_equal(n, [[1.0, 0, 0], [-1.0, 0, 0], [1.0, 0, 0]])


def test_orb_radial(oracle_lib):
    o = oracle_lib
    R = 50.0
    u = W.primaries.isotropic(np.random.default_rng(2), 200)
    n, f = o.solid_normal(ORB, [R], R * u)
    assert np.allclose(n, u, rtol=0, atol=1e-15)
    assert np.all(f == 1)


def test_tubs_faces(oracle_lib):
    o = oracle_lib
    rmin, rmax, dz, sphi, dphi = 40.0, 110.0, 90.0, 0.3, 1.2
    par = [rmin, rmax, dz, sphi, dphi]
    rng = np.random.default_rng(3)
    phi = rng.uniform(sphi + 0.05, sphi + dphi - 0.05, 40)
    z = rng.uniform(-80, 80, 40)
    radial = np.stack([np.cos(phi), np.sin(phi), np.zeros(40)], 1)
    n, f = o.solid_normal(TUBS, par, rmax * radial + np.stack([0 * z, 0 * z, z], 1))
    assert np.allclose(n, radial, atol=1e-15) and np.all(f == 1)
    n, f = o.solid_normal(TUBS, par, rmin * radial + np.stack([0 * z, 0 * z, z], 1))
    assert np.allclose(n, -radial, atol=1e-15) and np.all(f == 1)
    r = rng.uniform(50, 100, 40)
    for sgn in (-1.0, 1.0):
        p = np.stack([r * np.cos(phi), r * np.sin(phi), np.full(40, sgn * dz)], 1)
        n, f = o.solid_normal(TUBS, par, p)
        assert np.array_equal(n, np.tile([0, 0, sgn], (40, 1))) and np.all(f == 1)
    # the start half-plane at angle sphi faces towards smaller phi, the end one
    # (angle sphi + dphi) towards larger phi
    for ang, want in ((sphi, [math.sin(sphi), -math.cos(sphi), 0.0]),
                      (sphi + dphi, [-math.sin(sphi + dphi), math.cos(sphi + dphi), 0.0])):
        p = np.stack([r * math.cos(ang), r * math.sin(ang), z], 1)
        n, f = o.solid_normal(TUBS, par, p)
        assert np.allclose(n, np.tile(want, (40, 1)), atol=1e-15) and np.all(f == 1)
    # rim of the outer surface and the cap: an edge, where the outer face (first in
    # order) defines the normal
    n, f = o.solid_normal(TUBS, par, [[rmax * math.cos(1.0), rmax * math.sin(1.0), dz]])
    assert f[0] == 2
    assert np.allclose(n[0], [math.cos(1.0), math.sin(1.0), 0.0], atol=1e-15)


def test_cons_slanted_faces_tangent_and_outward(oracle_lib):
    o = oracle_lib
    r1i, r1o, r2i, r2o, dz = 20.0, 60.0, 50.0, 140.0, 75.0
    par = [r1i, r1o, r2i, r2o, dz, 0.0, 2 * math.pi]
    rng = np.random.default_rng(4)
    for rin, rout, sign in ((r1o, r2o, 1.0), (r1i, r2i, -1.0)):
        slope = (rout - rin) / (2 * dz)
        phi = rng.uniform(0, 2 * math.pi, 60)
        z = rng.uniform(-70, 70, 60)
        rho = rin + slope * (z + dz)
        p = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], 1)
        n, f = o.solid_normal(CONS, par, p)
        assert np.all(f == 1)
        assert np.allclose(np.linalg.norm(n, axis=1), 1, atol=1e-15)
        t_gen = np.stack([slope * np.cos(phi), slope * np.sin(phi), np.ones(60)], 1)
        t_az = np.stack([-np.sin(phi), np.cos(phi), np.zeros(60)], 1)
        assert np.allclose(np.sum(n * t_gen, 1), 0, atol=1e-14)
        assert np.allclose(np.sum(n * t_az, 1), 0, atol=1e-14)
        out = o.solid_eval(CONS, par, "d", p + 1e-3 * n)
        inn = o.solid_eval(CONS, par, "d", p - 1e-3 * n)
        assert np.all(out > 0) and np.all(inn < 0)
        # outer face normals lean towards -z when the cone widens with z
        assert np.all(np.sign(n[:, 2]) == -sign)


def _fd_grad(o, st, par, p, h=1e-5):
    g = np.zeros_like(p)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        g[:, k] = (o.solid_eval(st, par, "d", p + e) - o.solid_eval(st, par, "d", p - e)) / (2 * h)
    return g


def test_normal_is_gradient_of_signed_value(oracle_lib):
    """On faces away from edges the normal is grad d (central differences)."""
    o = oracle_lib
    rng = np.random.default_rng(6)
    solids = [(BOX, [30.0, 40.0, 50.0]), (ORB, [45.0]),
              (TUBS, [20.0, 70.0, 60.0, 0.4, 1.5]), (TUBS, [0.0, 70.0, 60.0, 0.0, 2 * math.pi]),
              (CONS, [10.0, 40.0, 30.0, 90.0, 55.0, -0.7, 2.0]),
              (CONS, [0.0, 80.0, 0.0, 20.0, 40.0, 0.0, 2 * math.pi])]
    for st, par in solids:
        # surface points: march random rays from inside out to the boundary
        p = rng.uniform(-1, 1, (4000, 3)) * 100
        inside = o.solid_eval(st, par, "inside", p) == 1
        p = p[inside][:300]
        v = W.primaries.isotropic(rng, len(p))
        s = o.solid_eval(st, par, "dist_out", p, v)
        q = p + s[:, None] * v
        n, f = o.solid_normal(st, par, q)
        face = f == 1
        # keep points well away from edges so the difference stays on one face
        g = _fd_grad(o, st, par, q[face])
        assert face.sum() > 100, (st, face.sum())
        assert np.allclose(n[face], g, atol=1e-6), st
        # exit points are left along the normal's side: v . n >= 0
        assert np.all(np.sum(n * v, 1)[face] > -1e-12)


def test_query_exit_normals_tiny(oracle_lib):
    desc = W.geometry.tiny()
    og = oracle_lib.Geometry(desc)
    # from (0, 250, 250) along +x: enters the box at (250, 250, 250) through x = 150
    pos = np.array([[0.0, 250.0, 250.0], [250.0, 250.0, 250.0], [0.0, 0.0, 0.0], [0.0, 250.0, 250.0]])
    dirs = np.array([[1.0, 0, 0], [0, 0, -1.0], [0, 0, 1.0], [0, -1.0, 0]])
    step, lim, nxt, n, val = og.compute_step_normal(pos, dirs)
    assert np.isclose(step[0], 150.0) and lim[0] >= 0 and val[0] == 1
    assert np.array_equal(n[0], [1.0, 0, 0])  # inward normal of the entered box
    assert np.isclose(step[1], 100.0) and lim[1] == -1 and val[1] == 1
    assert np.array_equal(n[1], [0, 0, -1.0])  # outward normal of the box left
    assert np.isclose(step[2], 500.0) and lim[2] == -1 and np.array_equal(n[2], [0, 0, 1.0])
    # from the world, along -y from (0,250,250): the world face y = -500 ... after
    # passing the gap between the boxes at x = 0 (no box spans x = 0)
    assert np.isclose(step[3], 750.0) and np.array_equal(n[3], [0, -1.0, 0])


def test_query_exit_normals_rotated_frames(oracle_lib):
    """In rotated placements the global normal of a face equals the rotated
    local normal: check grad of the crossed solid's d composed with the
    touchable's frame, by central differences in global coordinates."""
    desc = W.geometry.tiny(rotated=True)
    og = oracle_lib.Geometry(desc)
    rng = np.random.default_rng(8)
    pos = rng.uniform(-400, 400, (3000, 3))
    dirs = W.primaries.isotropic(rng, 3000)
    T = og.locate(pos, dirs)
    ok = T >= 0
    pos, dirs, T = pos[ok], dirs[ok], T[ok]
    step, lim, nxt, n, val = og.compute_step_normal(pos, dirs, T)
    fin = (val == 1)
    assert fin.sum() > 1000
    assert np.allclose(np.linalg.norm(n[fin], axis=1), 1, atol=1e-14)
    # exit normals point along the direction of travel
    assert np.all(np.sum(n[fin] * dirs[fin], 1) >= -1e-12)
    # just past the end point along the normal lies the next touchable, just before it
    # (against the normal) the current one
    q = pos + step[:, None] * dirs
    a = og.locate(q[fin] + 1e-6 * n[fin])
    b = og.locate(q[fin] - 1e-6 * n[fin])
    assert np.mean(a == nxt[fin]) > 0.999 and np.mean(b == T[fin]) > 0.999
